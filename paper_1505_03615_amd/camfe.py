"""Python binding of libcamfe.so: argument marshalling only.

Each function has the name of the C entry point it calls (include/camfe.h)
and does nothing but convert arguments: numpy arrays or torch tensors (host
or device) go in as pointers, handles are opaque integers, and C status codes
become CamfeError.  Every step of the method runs in the library's HIP
kernels; importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcamfe.so")

STATUS = {0: "CAMFE_OK", -1: "CAMFE_EINVAL", -2: "CAMFE_ENOMEM", -3: "CAMFE_EDEVICE",
          -4: "CAMFE_ENOCONV", -5: "CAMFE_ESINGULAR", -6: "CAMFE_ETOOSMALL", -7: "CAMFE_ESTATE"}

EXPORTS = [
    "camfe_last_error", "camfe_ctx_create", "camfe_ctx_destroy", "camfe_hierarchy_build",
    "camfe_hierarchy_levels", "camfe_hierarchy_cube", "camfe_hierarchy_info", "camfe_export_pairs",
    "camfe_export_functions", "camfe_export_support_entries", "camfe_export_prolongation",
    "camfe_hierarchy_destroy", "camfe_assemble", "camfe_reassemble_mass", "camfe_export_matrix",
    "camfe_load_vector", "camfe_gradient_load", "camfe_apply", "camfe_linear_coeffs", "camfe_eval_vertices", "camfe_solve",
    "camfe_system_destroy", "camfe_ctx_kernel_timing", "camfe_ctx_kernel_time", "camfe_measure_kernel",
    "camfe_model_create", "camfe_model_params", "camfe_model_destroy", "camfe_smoother_attach",
    "camfe_smoother_omega", "camfe_smoother_loss_grad", "camfe_smoother_train", "camfe_flow_step",
    "camfe_batch_create", "camfe_batch_info", "camfe_batch_solve", "camfe_batch_destroy", "camfe_eigs",
    "camfe_ctx_last_error", "camfe_export_cells", "camfe_system_set_sell_sort", "camfe_system_import_csr",
    "camfe_smoother_save", "camfe_smoother_load", "camfe_apply_noalloc", "camfe_system_autotune",
    "camfe_batch_autotune", "camfe_block_damping", "camfe_system_set_sell_columns", "camfe_system_sell_stats",
    "camfe_system_set_block_colouring", "camfe_radix_sort", "camfe_exclusive_sum",
]
TILES = [(8, 4), (4, 4), (8, 2), (16, 2), (16, 4), (4, 8), (2, 16)]   # colour-sweep tiles: (wavefronts per slice, entries per lane)
MLP_PARAMS = 2081   # parameters of one relative depth's MLP (30-32-32-1)
DEFAULT_COARSE_EPS = 1e-6   # eps * Id on the unit-diagonal-scaled coarsest matrix (the library's own default)
KERNELS = ["gs_colour", "residual", "spmv_dot", "restrict", "prolong", "coarse_solve", "assemble", "pairs",
           "uf_link", "support_sort", "cg_vector"]


class CamfeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class HierOpts(C.Structure):
    _fields_ = [("depth", C.c_int), ("degree", C.c_int), ("split", C.c_int), ("min_depth", C.c_int),
                ("max_coarse", C.c_int64), ("box_origin", C.c_double * 3), ("box_side", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("t", C.c_double), ("rtol", C.c_double), ("max_iter", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("method", C.c_int), ("precision", C.c_int), ("x0_given", C.c_int),
                ("coarse_eps", C.c_double), ("smoother", C.c_int), ("omega", C.c_double), ("judge", C.c_int),
                ("cycle", C.c_int), ("nu_coarse", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("fell_back", C.c_int), ("cycles", C.c_int), ("eps_regularised", C.c_int),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("setup_seconds", C.c_double),
                ("judge_rel", C.c_double * 2)]


def _stats_dict(st):
    return {f: (list(getattr(st, f)) if f == "judge_rel" else getattr(st, f)) for f, _ in SolveStats._fields_}


class EigOpts(C.Structure):
    _fields_ = [("nev", C.c_int), ("block", C.c_int), ("sigma", C.c_double), ("max_iter", C.c_int),
                ("tol", C.c_double), ("solve_rtol", C.c_double), ("precision", C.c_int), ("seed", C.c_uint64)]


class EigStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("solve_cycles", C.c_int), ("max_residual", C.c_double),
                ("seconds", C.c_double)]


class LevelCSR(C.Structure):
    _fields_ = [("depth", C.c_int), ("n", C.c_int64), ("keys", C.c_void_p), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("M", C.c_void_p), ("L", C.c_void_p), ("p_rowptr", C.c_void_p),
                ("p_col", C.c_void_p), ("p_w", C.c_void_p)]


class TrainOpts(C.Structure):
    _fields_ = [("t", C.c_double), ("levels", C.c_int), ("steps", C.c_int), ("nu", C.c_int), ("bf16", C.c_int),
                ("lr", C.c_double), ("seed", C.c_uint64), ("sweep", C.c_int), ("cycle", C.c_int),
                ("samples", C.c_int), ("t_each", C.c_void_p)]


_lib = None


def load():
    """The loaded library; raises ImportError (never falls back) when absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1505_03615_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P, I, I64, D, H = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "camfe_last_error": (C.c_char_p, []),
        "camfe_ctx_create": (I, [I, P, C.POINTER(H)]),
        "camfe_ctx_destroy": (None, [H]),
        "camfe_hierarchy_build": (I, [H, P, I64, P, I64, C.POINTER(HierOpts), C.POINTER(H)]),
        "camfe_hierarchy_levels": (I, [H, C.POINTER(I), C.POINTER(I)]),
        "camfe_hierarchy_cube": (I, [H, P]),
        "camfe_hierarchy_info": (I, [H, I, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
        "camfe_export_pairs": (I, [H, I, P, P, I64, C.POINTER(I64)]),
        "camfe_export_functions": (I, [H, I, P, P, P, I64, C.POINTER(I64)]),
        "camfe_export_support_entries": (I, [H, I, P, P, P, I64, C.POINTER(I64)]),
        "camfe_export_prolongation": (I, [H, I, P, P, P, I64, C.POINTER(I64)]),
        "camfe_hierarchy_destroy": (None, [H]),
        "camfe_assemble": (I, [H, P, C.POINTER(H)]),
        "camfe_reassemble_mass": (I, [H, P]),
        "camfe_export_matrix": (I, [H, I, I, P, P, P, I64, C.POINTER(I64)]),
        "camfe_load_vector": (I, [H, P, I, P]),
        "camfe_gradient_load": (I, [H, P, I, P]),
        "camfe_eigs": (I, [H, P, P, P, P]),
        "camfe_apply": (I, [H, I, D, P, I, P]),
        "camfe_linear_coeffs": (I, [H, P]),
        "camfe_eval_vertices": (I, [H, P, I, P]),
        "camfe_solve": (I, [H, C.POINTER(SolveOpts), P, I, P, C.POINTER(SolveStats)]),
        "camfe_system_destroy": (None, [H]),
        "camfe_ctx_kernel_timing": (I, [H, I]),
        "camfe_ctx_kernel_time": (I, [H, C.c_char_p, C.POINTER(D), C.POINTER(I64), C.POINTER(D)]),
        "camfe_measure_kernel": (I, [H, C.c_char_p, I, I, C.POINTER(D), C.POINTER(D)]),
        "camfe_model_create": (I, [P, I, I, I, C.POINTER(H)]),
        "camfe_model_params": (I, [H, P, I64, C.POINTER(I64), C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
        "camfe_model_destroy": (None, [H]),
        "camfe_smoother_attach": (I, [H, H]),
        "camfe_smoother_omega": (I, [H, H, I, D, P]),
        "camfe_smoother_loss_grad": (I, [H, I, D, P, I, I, I, P, I, I, C.POINTER(D), P]),
        "camfe_smoother_train": (I, [H, P, I, C.POINTER(TrainOpts), C.POINTER(H), P]),
        "camfe_flow_step": (I, [H, D, P, C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
        "camfe_batch_create": (I, [H, P, I, D, D, C.POINTER(H)]),
        "camfe_batch_info": (I, [H, C.POINTER(I), C.POINTER(I64)]),
        "camfe_batch_solve": (I, [H, C.POINTER(SolveOpts), P, P, P, P]),
        "camfe_batch_destroy": (None, [H]),
        "camfe_ctx_last_error": (C.c_char_p, [H]),
        "camfe_export_cells": (I, [H, I, P, I64, C.POINTER(I64)]),
        "camfe_system_set_sell_sort": (I, [H, I64]),
        "camfe_system_import_csr": (I, [H, I, I, P, I64, C.POINTER(H)]),
        "camfe_smoother_save": (I, [H, C.c_char_p]),
        "camfe_smoother_load": (I, [C.c_char_p, C.POINTER(H)]),
        "camfe_apply_noalloc": (I, [H, I, D, P, I, P]),
        "camfe_system_autotune": (I, [H, D, I, I, P, P, I, C.POINTER(I)]),
        "camfe_batch_autotune": (I, [H, I, I, P, P, I, C.POINTER(I)]),
        "camfe_block_damping": (I, [H, D, D, P, P, I, C.POINTER(I)]),
        "camfe_system_set_sell_columns": (I, [H, I]),
        "camfe_system_set_block_colouring": (I, [H, I64]),
        "camfe_system_sell_stats": (I, [H, I, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
        "camfe_radix_sort": (I, [H, P, I, P, I64, I]),
        "camfe_exclusive_sum": (I, [H, P, P, I64, I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        raise CamfeError(code, load().camfe_last_error().decode())


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    if a is None:
        return None
    if _is_torch(a):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _rowmajor(a, dtype):
    if _is_torch(a):
        import torch
        return a.to(getattr(torch, dtype)).contiguous()
    return np.ascontiguousarray(a, dtype=dtype)


def _colmajor(a):
    """(array with column-major n x k storage, n, k) for numpy or torch input."""
    if _is_torch(a):
        import torch
        a = a.to(torch.float64)
        if a.dim() == 1:
            a = a.unsqueeze(1)
        if a.stride(0) != 1 or (a.shape[1] > 1 and a.stride(1) != a.shape[0]):
            a = a.t().contiguous().t()
        return a, a.shape[0], a.shape[1]
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return np.asfortranarray(a), a.shape[0], a.shape[1]


def _empty_like_kind(a, n, k):
    """Column-major n x k output of the same kind/device as `a`."""
    if _is_torch(a):
        import torch
        return torch.empty((k, n), dtype=torch.float64, device=a.device).t()
    return np.zeros((n, k), order="F")


# ----------------------------------------------------------------- context
def camfe_ctx_create(device: int = 0, stream=None):
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    lib = load()
    h = C.c_void_p()
    s = None
    if stream is not None:
        s = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(lib.camfe_ctx_create(device, s, C.byref(h)))
    return h


def camfe_ctx_destroy(ctx):
    load().camfe_ctx_destroy(ctx)


def camfe_ctx_last_error(ctx):
    """Message of the last failed call that reached this context ('' if none)."""
    return load().camfe_ctx_last_error(ctx).decode()


def camfe_ctx_kernel_timing(ctx, enable: bool):
    _check(load().camfe_ctx_kernel_timing(ctx, 1 if enable else 0))


def camfe_ctx_kernel_time(ctx, kernel: str):
    """(total ms, launches, algorithmic work) of one kernel since timing was enabled."""
    ms, n, w = C.c_double(), C.c_int64(), C.c_double()
    _check(load().camfe_ctx_kernel_time(ctx, kernel.encode(), C.byref(ms), C.byref(n), C.byref(w)))
    return ms.value, n.value, w.value


# --------------------------------------------------------------- hierarchy
def camfe_hierarchy_build(ctx, V, F, depth, degree=1, split=1, min_depth=0, max_coarse=4096, box=None):
    lib = load()
    Vc, Fc = _rowmajor(V, "float64"), _rowmajor(F, "int32")
    o = HierOpts()
    o.depth, o.degree, o.split, o.min_depth, o.max_coarse = depth, degree, split, min_depth, max_coarse
    if box is not None:
        o.box_origin[0], o.box_origin[1], o.box_origin[2], o.box_side = (float(v) for v in box)
    h = C.c_void_p()
    _check(lib.camfe_hierarchy_build(ctx, _ptr(Vc), Vc.shape[0], _ptr(Fc), Fc.shape[0], C.byref(o),
                                     C.byref(h)))
    return h


def camfe_hierarchy_levels(h):
    a, b = C.c_int(), C.c_int()
    _check(load().camfe_hierarchy_levels(h, C.byref(a), C.byref(b)))
    return a.value, b.value


def camfe_hierarchy_cube(h):
    out = np.zeros(4)
    _check(load().camfe_hierarchy_cube(h, _ptr(out)))
    return out


def camfe_hierarchy_info(h, depth):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().camfe_hierarchy_info(h, depth, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def _two_call(fn, h, depth, makers):
    n = C.c_int64()
    _check(fn(h, depth, *([None] * len(makers)), 0, C.byref(n)))
    outs = [m(n.value) for m in makers]
    if n.value:
        _check(fn(h, depth, *[_ptr(o) for o in outs], n.value, C.byref(n)))
    return outs


def camfe_export_cells(h, depth):
    """Occupied cells at one depth: Morton keys ascending."""
    return _two_call(load().camfe_export_cells, h, depth, [lambda n: np.zeros(n, np.uint64)])[0]


def camfe_export_pairs(h, depth):
    return tuple(_two_call(load().camfe_export_pairs, h, depth,
                           [lambda n: np.zeros(n, np.uint64), lambda n: np.zeros(n, np.int32)]))


def camfe_export_functions(h, depth):
    return tuple(_two_call(load().camfe_export_functions, h, depth,
                           [lambda n: np.zeros(n, np.uint64), lambda n: np.zeros(n, np.int32),
                            lambda n: np.zeros(n, np.int32)]))


def camfe_export_support_entries(h, depth):
    return tuple(_two_call(load().camfe_export_support_entries, h, depth,
                           [lambda n: np.zeros(n, np.uint64), lambda n: np.zeros(n, np.int32),
                            lambda n: np.zeros(n, np.int32)]))


def camfe_export_prolongation(h, depth):
    import scipy.sparse as sp
    lib = load()
    nf = camfe_hierarchy_info(h, depth)[2]
    nc = camfe_hierarchy_info(h, depth - 1)[2]
    nnz = C.c_int64()
    _check(lib.camfe_export_prolongation(h, depth, None, None, None, 0, C.byref(nnz)))
    ptr = np.zeros(nf + 1, np.int64); col = np.zeros(nnz.value, np.int32); w = np.zeros(nnz.value)
    _check(lib.camfe_export_prolongation(h, depth, _ptr(ptr), _ptr(col), _ptr(w), max(nnz.value, 1),
                                         C.byref(nnz)))
    return sp.csr_matrix((w, col, ptr), shape=(nf, nc))


def camfe_hierarchy_destroy(h):
    load().camfe_hierarchy_destroy(h)


# ---------------------------------------------------------------- assembly
def camfe_assemble(h, tri_weight=None):
    s = C.c_void_p()
    tw = None if tri_weight is None else _rowmajor(tri_weight, "float64")
    _check(load().camfe_assemble(h, _ptr(tw), C.byref(s)))
    return s


def camfe_reassemble_mass(s, tri_weight=None):
    tw = None if tri_weight is None else _rowmajor(tri_weight, "float64")
    _check(load().camfe_reassemble_mass(s, _ptr(tw)))


def camfe_export_matrix(s, h, depth, which):
    """which: 0 = M, 1 = L; returns scipy CSR (the hierarchy handle gives n)."""
    import scipy.sparse as sp
    lib = load()
    n = camfe_hierarchy_info(h, depth)[2]
    nnz = C.c_int64()
    _check(lib.camfe_export_matrix(s, depth, which, None, None, None, 0, C.byref(nnz)))
    ptr = np.zeros(n + 1, np.int64); col = np.zeros(nnz.value, np.int32); val = np.zeros(nnz.value)
    _check(lib.camfe_export_matrix(s, depth, which, _ptr(ptr), _ptr(col), _ptr(val), max(nnz.value, 1),
                                   C.byref(nnz)))
    return sp.csr_matrix((val, col, ptr), shape=(n, n))


def camfe_load_vector(s, h, vertex_f):
    fv, nv, k = _colmajor(vertex_f)
    n = camfe_hierarchy_info(h, camfe_hierarchy_levels(h)[0])[2]
    b = _empty_like_kind(fv, n, k)
    _check(load().camfe_load_vector(s, _ptr(fv), k, _ptr(b)))
    return b


def camfe_gradient_load(s, h, vertex_f):
    """b_i = int <grad f, grad b_i> (the colour fit's gradient constraint)."""
    fv, nv, k = _colmajor(vertex_f)
    n = camfe_hierarchy_info(h, camfe_hierarchy_levels(h)[0])[2]
    b = _empty_like_kind(fv, n, k)
    _check(load().camfe_gradient_load(s, _ptr(fv), k, _ptr(b)))
    return b


def camfe_apply(s, which, t, x):
    xc, n, k = _colmajor(x)
    y = _empty_like_kind(xc, n, k)
    _check(load().camfe_apply(s, which, t, _ptr(xc), k, _ptr(y)))
    return y


def camfe_apply_noalloc(s, which, t, x, y):
    """y = A x through the entry point that allocates nothing: x and y are
    column-major n x k device tensors (y is written in place)."""
    if not (_is_torch(x) and _is_torch(y)):
        raise TypeError("x and y must be device tensors")
    n, k = x.shape if x.dim() == 2 else (x.shape[0], 1)
    for a in (x, y):
        if a.dtype != x.dtype or tuple(a.shape[:1]) != (n,) or a.stride(0) != 1 or (k > 1 and a.stride(1) != n):
            raise ValueError("x and y must be column-major n x k float64 tensors")
    _check(load().camfe_apply_noalloc(s, which, t, _ptr(x), k, _ptr(y)))
    return y


def camfe_radix_sort(ctx, keys, end_bit, vals=None):
    """Stable in-place sort of a 1-D device tensor of uint64/int64 or
    uint32/int32 keys by bits [0, end_bit), carrying an int32/uint32 tensor
    of values along when given."""
    if not _is_torch(keys) or keys.dim() != 1 or not keys.is_contiguous():
        raise TypeError("keys must be a contiguous 1-D device tensor")
    kb = keys.element_size()
    if vals is not None and (not _is_torch(vals) or vals.shape != keys.shape or vals.element_size() != 4
                             or not vals.is_contiguous()):
        raise TypeError("vals must be a contiguous 32-bit device tensor shaped like keys")
    _check(load().camfe_radix_sort(ctx, _ptr(keys), kb, None if vals is None else _ptr(vals), keys.numel(),
                                   end_bit))
    return keys, vals


def camfe_exclusive_sum(ctx, x, out=None):
    """Exclusive prefix sum of a 1-D int32/int64 device tensor (out may be x)."""
    if not _is_torch(x) or x.dim() != 1 or not x.is_contiguous():
        raise TypeError("x must be a contiguous 1-D device tensor")
    if out is None:
        out = x.new_empty(x.shape)
    _check(load().camfe_exclusive_sum(ctx, _ptr(x), _ptr(out), x.numel(), x.element_size()))
    return out


def camfe_linear_coeffs(s, h):
    n = camfe_hierarchy_info(h, camfe_hierarchy_levels(h)[0])[2]
    X = np.zeros((n, 3), order="F")
    _check(load().camfe_linear_coeffs(s, _ptr(X)))
    return X


def camfe_eval_vertices(s, nv, x):
    xc, n, k = _colmajor(x)
    out = _empty_like_kind(xc, nv, k)
    _check(load().camfe_eval_vertices(s, _ptr(xc), k, _ptr(out)))
    return out


def camfe_solve(s, b, t, rtol=1e-8, max_iter=200, nu_pre=2, nu_post=2, method=0, precision=0, x0=None,
                coarse_eps=DEFAULT_COARSE_EPS, raise_on_noconv=False, smoother=0, omega=0.0, judge=0, cycle=1,
                nu_coarse=0):
    """Returns (x, stats dict).  method 0 = cycle-preconditioned CG, 1 = stationary cycles;
    smoother 0 = multicolour Gauss-Seidel, 1 = Jacobi(omega), 2 = attached learned model;
    judge > 0: smoother 1/2 and Gauss-Seidel each run `judge` CG iterations, the better continues;
    cycle 1 = V-cycle, 2 = W-cycle."""
    bc, n, k = _colmajor(b)
    if x0 is None:
        x = _empty_like_kind(bc, n, k)
    else:
        x = _colmajor(x0.clone() if _is_torch(x0) else np.array(x0, dtype=np.float64, copy=True))[0]
    o = SolveOpts()
    o.t, o.rtol, o.max_iter, o.nu_pre, o.nu_post = t, rtol, max_iter, nu_pre, nu_post
    o.method, o.precision, o.x0_given, o.coarse_eps = method, precision, 0 if x0 is None else 1, coarse_eps
    o.smoother, o.omega, o.judge, o.cycle, o.nu_coarse = smoother, omega, judge, cycle, nu_coarse
    st = SolveStats()
    code = load().camfe_solve(s, C.byref(o), _ptr(bc), k, _ptr(x), C.byref(st))
    if code != 0 and (code != -4 or raise_on_noconv):
        _check(code)
    stats = _stats_dict(st)
    stats["converged"] = code == 0
    return x, stats


def camfe_eigs(s, h, nev, sigma, block=0, max_iter=200, tol=1e-8, solve_rtol=1e-10, precision=0, seed=1,
               vectors=True, raise_on_noconv=False, device=None):
    """Smallest eigenpairs of L x = lambda M x: (evals, evecs n x nev or None, stats dict).
    device: a torch device for the outputs (default: numpy on the host)."""
    n = camfe_hierarchy_info(h, camfe_hierarchy_levels(h)[0])[2]
    if device is not None:
        import torch
        ev = torch.empty(nev, dtype=torch.float64, device=device)
        X = torch.empty((nev, n), dtype=torch.float64, device=device).t() if vectors else None
    else:
        ev = np.zeros(nev)
        X = np.zeros((n, nev), order="F") if vectors else None
    o = EigOpts()
    o.nev, o.block, o.sigma, o.max_iter, o.tol = nev, block, sigma, max_iter, tol
    o.solve_rtol, o.precision, o.seed = solve_rtol, precision, seed
    st = EigStats()
    code = load().camfe_eigs(s, C.byref(o), _ptr(ev), None if X is None else _ptr(X), C.byref(st))
    if code != 0 and (code != -4 or raise_on_noconv):
        _check(code)
    stats = {f: getattr(st, f) for f, _ in EigStats._fields_}
    stats["converged"] = code == 0
    return ev, X, stats


def camfe_measure_kernel(s, kernel: str, precision: int = 0, reps: int = 50):
    """(average ms per launch, algorithmic bytes per launch) of a finest-depth kernel."""
    ms, by = C.c_double(), C.c_double()
    _check(load().camfe_measure_kernel(s, kernel.encode(), precision, reps, C.byref(ms), C.byref(by)))
    return ms.value, by.value


def camfe_system_destroy(s):
    load().camfe_system_destroy(s)


def camfe_system_set_sell_columns(s, bits):
    _check(load().camfe_system_set_sell_columns(s, bits))


def camfe_system_set_block_colouring(s, min_blocks):
    _check(load().camfe_system_set_block_colouring(s, min_blocks))


def camfe_system_sell_stats(s, depth):
    """(slices, slices with 16-bit column codes, stored entries) of one depth."""
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().camfe_system_sell_stats(s, depth, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def camfe_system_set_sell_sort(s, min_rows):
    """Length-sort the rows of colours with at least min_rows rows (<= 0: the default 2^19)."""
    _check(load().camfe_system_set_sell_sort(s, int(min_rows)))


def _autotune(fn, *args):
    nl = C.c_int()
    _check(fn(*args, None, None, 0, C.byref(nl)))
    tile = np.zeros(nl.value, np.int32)
    ms = np.zeros(nl.value)
    _check(fn(*args, _ptr(tile), _ptr(ms), nl.value, C.byref(nl)))
    return tile, ms


def camfe_system_autotune(s, t, precision=1, reps=10):
    """(tile index per depth, coarsest first; ms per sweep with it)."""
    return _autotune(load().camfe_system_autotune, s, t, precision, reps)


def camfe_batch_autotune(bt, precision=0, reps=10):
    """(tile index per batch level, coarsest first; ms per sweep with it)."""
    return _autotune(load().camfe_batch_autotune, bt, precision, reps)


def camfe_block_damping(s, t, coarse_eps=DEFAULT_COARSE_EPS):
    """(automatic damping of smoother 3 per depth, the lambda_max estimates), coarsest first."""
    nl = C.c_int()
    _check(load().camfe_block_damping(s, t, coarse_eps, None, None, 0, C.byref(nl)))
    om = np.zeros(nl.value)
    lam = np.zeros(nl.value)
    _check(load().camfe_block_damping(s, t, coarse_eps, _ptr(om), _ptr(lam), nl.value, C.byref(nl)))
    return om, lam


def camfe_system_import_csr(ctx, degree, levels, max_coarse=4096):
    """System from given matrices.  levels: coarsest first, one dict per depth with
    'depth', 'keys' (uint64), 'M' and 'L' (scipy CSR on one pattern) and, except
    for the coarsest, 'P' (scipy CSR prolongation from the depth below)."""
    keep = []

    def arr(a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a.ctypes.data

    lv = (LevelCSR * len(levels))()
    for i, d in enumerate(levels):
        M, L = d["M"].tocsr(), d["L"].tocsr()
        M.sort_indices(); L.sort_indices()
        if not (np.array_equal(M.indptr, L.indptr) and np.array_equal(M.indices, L.indices)):
            raise ValueError("M and L must share one pattern")
        lv[i].depth, lv[i].n = int(d["depth"]), M.shape[0]
        lv[i].keys = arr(d["keys"], np.uint64)
        lv[i].rowptr, lv[i].col = arr(M.indptr, np.int64), arr(M.indices, np.int32)
        lv[i].M, lv[i].L = arr(M.data, np.float64), arr(L.data, np.float64)
        if d.get("P") is not None:
            P = d["P"].tocsr()
            P.sort_indices()
            lv[i].p_rowptr, lv[i].p_col = arr(P.indptr, np.int64), arr(P.indices, np.int32)
            lv[i].p_w = arr(P.data, np.float64)
    s = C.c_void_p()
    _check(load().camfe_system_import_csr(ctx, int(degree), len(levels), C.cast(lv, C.c_void_p), int(max_coarse),
                                          C.byref(s)))
    return s


def camfe_flow_step(s, X, delta, rtol=1e-8, max_iter=400, nu_pre=2, nu_post=2, precision=0, smoother=0,
                    omega=0.0, coarse_eps=DEFAULT_COARSE_EPS, raise_on_noconv=False, cycle=1, nu_coarse=0):
    """One tracked cMCF step; X (n x 3, numpy or torch) is updated in place and returned with the stats."""
    Xc, n, k = _colmajor(X)
    if k != 3:
        raise ValueError("X must have three columns")
    o = SolveOpts()
    o.rtol, o.max_iter, o.nu_pre, o.nu_post, o.precision = rtol, max_iter, nu_pre, nu_post, precision
    o.coarse_eps, o.smoother, o.omega = coarse_eps, smoother, omega
    o.cycle, o.nu_coarse = cycle, nu_coarse
    st = SolveStats()
    code = load().camfe_flow_step(s, delta, _ptr(Xc), C.byref(o), C.byref(st))
    if code != 0 and (code != -4 or raise_on_noconv):
        _check(code)
    if Xc is not X:
        X[...] = Xc
    stats = _stats_dict(st)
    stats["converged"] = code == 0
    return X, stats


def _handle(x):
    return x.value if isinstance(x, C.c_void_p) else x


def camfe_batch_create(ctx, systems, t, coarse_eps=DEFAULT_COARSE_EPS):
    arr = (C.c_void_p * len(systems))(*[_handle(x) for x in systems])
    b = C.c_void_p()
    _check(load().camfe_batch_create(ctx, C.cast(arr, C.c_void_p), len(systems), t, coarse_eps, C.byref(b)))
    return b.value


def camfe_batch_info(bt):
    lv, rows = C.c_int(), C.c_int64()
    _check(load().camfe_batch_info(bt, C.byref(lv), C.byref(rows)))
    return lv.value, rows.value


def camfe_batch_solve(bt, bs, t, rtol=1e-8, max_iter=400, nu_pre=2, nu_post=2, precision=0, x0s=None,
                      coarse_eps=DEFAULT_COARSE_EPS, raise_on_noconv=False, cycle=1, nu_coarse=0):
    """bs: list of n_m x k_m right-hand sides.  Returns (list of solutions, list of stats dicts).
    The batch takes V-cycles only (cycle 1); other values are passed on and rejected."""
    cols = [_colmajor(b) for b in bs]
    if x0s is None:
        xs = [_empty_like_kind(bc, n, k) for bc, n, k in cols]
    else:
        xs = [_colmajor(x.clone() if _is_torch(x) else np.array(x, dtype=np.float64, copy=True))[0] for x in x0s]
    m = len(bs)
    bp = (C.c_void_p * m)(*[_ptr(bc).value for bc, _, _ in cols])
    xp = (C.c_void_p * m)(*[_ptr(x).value for x in xs])
    kk = (C.c_int * m)(*[k for _, _, k in cols])
    o = SolveOpts()
    o.t, o.rtol, o.max_iter, o.nu_pre, o.nu_post = t, rtol, max_iter, nu_pre, nu_post
    o.method, o.precision, o.x0_given, o.coarse_eps = 0, precision, 0 if x0s is None else 1, coarse_eps
    o.cycle, o.nu_coarse = cycle, nu_coarse
    st = (SolveStats * m)()
    code = load().camfe_batch_solve(bt, C.byref(o), C.cast(bp, C.c_void_p), C.cast(kk, C.c_void_p),
                                    C.cast(xp, C.c_void_p), C.cast(st, C.c_void_p))
    if code != 0 and (code != -4 or raise_on_noconv):
        _check(code)
    stats = [{f: getattr(x, f) for f, _ in SolveStats._fields_} for x in st]
    for x in stats:
        x["converged"] = x["rel_residual"] <= rtol
    return xs, stats


def camfe_batch_destroy(bt):
    load().camfe_batch_destroy(bt)


# ------------------------------------------------------------ learned smoother
SWEEP_JACOBI, SWEEP_SOR = 0, 1


def camfe_model_create(params=None, levels=1, bf16=True, sweep=SWEEP_JACOBI):
    """Model handle from packed FP32 parameters (levels x 2081) or the default initialisation;
    sweep 0 = damped Jacobi (l1-bounded weights), 1 = multicolour SOR."""
    p = None
    if params is not None:
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if p.size % MLP_PARAMS:
            raise ValueError("parameters must be a multiple of 2081 floats")
        levels = p.size // MLP_PARAMS
    m = C.c_void_p()
    _check(load().camfe_model_create(_ptr(p), int(levels), 1 if bf16 else 0, int(sweep), C.byref(m)))
    return m.value


def camfe_model_params(m):
    """(params float32 [levels, 2081], bf16 flag, sweep type)."""
    n, lv, bf, sw = C.c_int64(), C.c_int(), C.c_int(), C.c_int()
    _check(load().camfe_model_params(m, None, 0, C.byref(n), C.byref(lv), C.byref(bf), C.byref(sw)))
    out = np.zeros(n.value, dtype=np.float32)
    _check(load().camfe_model_params(m, _ptr(out), n.value, C.byref(n), None, None, None))
    return out.reshape(lv.value, MLP_PARAMS), bool(bf.value), sw.value


def camfe_model_destroy(m):
    load().camfe_model_destroy(m)


def camfe_smoother_attach(s, m):
    _check(load().camfe_smoother_attach(s, m))


def camfe_smoother_omega(s, h, m, depth, t):
    """omega of every function at one depth (canonical order)."""
    out = np.zeros(camfe_hierarchy_info(h, depth)[2])
    _check(load().camfe_smoother_omega(s, m, depth, t, _ptr(out)))
    return out


def camfe_smoother_loss_grad(s, depth, t, params, e0, nu, bf16=True, want_grad=True, sweep=SWEEP_JACOBI, cycle=0):
    """(loss, gradient float64[2081] or None) for one MLP's parameters and n_d x S samples."""
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    if p.size != MLP_PARAMS:
        raise ValueError("one MLP has 2081 parameters")
    e = np.asfortranarray(np.asarray(e0, dtype=np.float64))
    if e.ndim == 1:
        e = e.reshape(-1, 1, order="F")
    loss = C.c_double()
    g = np.zeros(MLP_PARAMS) if want_grad else None
    _check(load().camfe_smoother_loss_grad(s, depth, t, _ptr(p), 1 if bf16 else 0, int(sweep), int(cycle), _ptr(e),
                                           e.shape[1], nu, C.byref(loss), _ptr(g)))
    return loss.value, g


def camfe_smoother_train(ctx, systems, t, levels=3, steps=200, nu=2, bf16=True, lr=3e-3, seed=1, samples=0,
                         sweep=SWEEP_JACOBI, cycle=0):
    """(model handle, loss history) trained on the GPU over the given systems.
    t: one value, or one per system (each system then listed once);
    samples: 0 random vectors, 1 errors left by one plain V-cycle, 2 two of each;
    sweep: 0 damped Jacobi, 1 multicolour SOR; cycle: 0 smoothing loss, 1 two-grid loss."""
    arr = (C.c_void_p * len(systems))(*[x.value if isinstance(x, C.c_void_p) else x for x in systems])
    o = TrainOpts()
    t_each = None
    if np.ndim(t):
        t_each = np.ascontiguousarray(t, dtype=np.float64)
        if t_each.shape != (len(systems),):
            raise ValueError("t: one value per system")
        t = 0.0
    o.t, o.levels, o.steps, o.nu, o.bf16, o.lr, o.seed = t, levels, steps, nu, 1 if bf16 else 0, lr, seed
    o.samples, o.sweep, o.cycle = samples, sweep, cycle
    o.t_each = None if t_each is None else t_each.ctypes.data
    hist = np.zeros(max(steps, 1))
    m = C.c_void_p()
    _check(load().camfe_smoother_train(ctx, C.cast(arr, C.c_void_p), len(systems), C.byref(o), C.byref(m),
                                       _ptr(hist)))
    return m.value, hist[:steps]


def camfe_smoother_save(m, path):
    """Write the model as the library's plain binary record."""
    _check(load().camfe_smoother_save(m, os.fsencode(path)))


def camfe_smoother_load(path):
    """A new model handle read from the library's binary record."""
    m = C.c_void_p()
    _check(load().camfe_smoother_load(os.fsencode(path), C.byref(m)))
    return m.value
