"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Discrete structure (cube, pairs, functions, (support, triangle) labels,
prolongation) must match bit for bit; M, L and load vectors within 1e-12
relative (max-norm); solutions within 1e-6 relative residual measured with
the oracle's matrices.  Cases span several tiles, ragged tails, exact
touching (dyadic coordinates on grid planes), the split and unsplit spaces,
both degrees, and a singular (axis-aligned planar) system.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_1505_03615_amd import meshgen
from tests.test_oracle_assembly import sheet_fields_coeffs
from tests.test_oracle_structure import dyadic_sheet

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    V1, F1, f1 = meshgen.config_mesh("icosphere_l3")
    Vs, Fs, fs = meshgen.config_mesh("two_sheets", n=64, gap=1.0 / 64)
    Va, Fa, fa = meshgen.config_mesh("two_sheets", n=32, gap=1.0 / 32, rotate=False)
    Vk, Fk = meshgen.torus_knot(nu=1024, nv=16, seed=3)
    Vd, Fd = dyadic_sheet(104, n=6)
    return {
        "sphere_deg1": dict(V=V1, F=F1, f=f1, depth=5, degree=1, max_coarse=512),
        "sphere_deg2": dict(V=V1, F=F1, f=f1, depth=4, degree=2, max_coarse=512),
        "sheets_split": dict(V=Vs, F=Fs, f=fs, depth=6, degree=1, max_coarse=512),
        "sheets_unsplit": dict(V=Vs, F=Fs, f=fs, depth=6, degree=1, split=0, max_coarse=512),
        "sheets_axis": dict(V=Va, F=Fa, f=fa, depth=5, degree=1, max_coarse=256),
        "knot": dict(V=Vk, F=Fk, f=Vk, depth=7, degree=1, max_coarse=512),
        "dyadic": dict(V=Vd, F=Fd, f=Vd[:, 2], depth=2, degree=1, max_coarse=0, box=[0, 0, 0, 4.0]),
        "dyadic_deg2": dict(V=Vd, F=Fd, f=Vd[:, 2], depth=2, degree=2, max_coarse=0, box=[0, 0, 0, 4.0]),
    }


CASES = _cases()


@pytest.fixture(scope="module")
def cf():
    import torch
    from paper_1505_03615_amd import camfe
    assert torch.cuda.is_available()
    return camfe


@pytest.fixture(scope="module")
def ctx(cf):
    c = cf.camfe_ctx_create(0)
    yield c
    cf.camfe_ctx_destroy(c)


_built = {}


def built(cf, ctx, name):
    if name not in _built:
        c = CASES[name]
        kw = dict(depth=c["depth"], degree=c["degree"], split=c.get("split", 1), min_depth=0,
                  max_coarse=c["max_coarse"], box=c.get("box"))
        say(f"[gpu] build {name} nt={len(c['F'])} depth={c['depth']} degree={c['degree']}")
        h = cf.camfe_hierarchy_build(ctx, c["V"], c["F"], **kw)
        say(f"[gpu] assemble {name}")
        s = cf.camfe_assemble(h)
        o = Oracle(c["V"], c["F"], c["depth"], degree=c["degree"], split=kw["split"], min_depth=0,
                   max_coarse=c["max_coarse"], box=c.get("box")).check().assemble()
        _built[name] = (h, s, o)
    return _built[name]


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_bit_exact(cf, ctx, name):
    h, s, o = built(cf, ctx, name)
    D = CASES[name]["depth"]
    assert np.array_equal(cf.camfe_hierarchy_cube(h), o.cube())
    fin, d0 = cf.camfe_hierarchy_levels(h)
    assert (fin, d0) == (D, o.coarsest)
    for d in range(D, -1, -1):
        k, t = cf.camfe_export_pairs(h, d)
        ko, to = o.pairs(d)
        assert np.array_equal(k, ko) and np.array_equal(t, to), f"pairs depth {d}"
        if d < d0:
            continue
        for a, b in zip(cf.camfe_export_functions(h, d), o.functions(d)):
            assert np.array_equal(a, b), f"functions depth {d}"
        for a, b in zip(cf.camfe_export_support_entries(h, d), o.support_entries(d)):
            assert np.array_equal(a, b), f"support entries depth {d}"
        if d > d0:
            P, Po = cf.camfe_export_prolongation(h, d), o.prolongation(d)
            assert np.array_equal(P.indptr, Po.indptr) and np.array_equal(P.indices, Po.indices)
            assert np.array_equal(P.data, Po.data), f"prolongation depth {d}"


@pytest.mark.parametrize("name", list(CASES))
def test_matrices_match(cf, ctx, name):
    h, s, o = built(cf, ctx, name)
    fin, d0 = cf.camfe_hierarchy_levels(h)
    for d in range(d0, fin + 1):
        Mo, Lo = o.matrices(d)
        M = cf.camfe_export_matrix(s, h, d, 0)
        L = cf.camfe_export_matrix(s, h, d, 1)
        em = abs(M - Mo).max() / abs(Mo).max()
        el = abs(L - Lo).max() / abs(Lo).max()
        assert em <= 1e-12 and el <= 1e-12, (d, em, el)


@pytest.mark.parametrize("name", ["sphere_deg1", "sphere_deg2", "knot", "dyadic", "sheets_split"])
def test_load_vector_and_vertex_values(cf, ctx, name):
    h, s, o = built(cf, ctx, name)
    c = CASES[name]
    b = cf.camfe_load_vector(s, h, c["f"])
    bo = o.load_vector(c["f"])
    assert abs(b - bo).max() <= 1e-12 * abs(bo).max()
    X = cf.camfe_linear_coeffs(s, h)
    assert np.array_equal(X, o.linear_coeffs())
    ev = cf.camfe_eval_vertices(s, len(c["V"]), X)
    assert np.allclose(ev, o.eval_vertices(X), rtol=0, atol=1e-13)
    # coefficients that differ between the components of a split support: a
    # linear field per half of the triangle list, chosen by each function's
    # representative triangle (on the two sheets, one field per sheet)
    _, _, rep = o.functions(c["depth"])
    fields = np.array([[0.7, -1.3, 0.4], [-0.9, 0.5, 1.6]])
    xs = sheet_fields_coeffs(X, rep, len(c["F"]) // 2, fields)
    ev = cf.camfe_eval_vertices(s, len(c["V"]), xs)
    evo = o.eval_vertices(xs)
    assert np.allclose(ev, evo, rtol=0, atol=1e-13)
    if name == "sheets_split":
        sheet = meshgen.two_sheets(64, 1.0 / 64)[3]
        assert np.abs(ev[:, 0] - np.einsum("ij,ij->i", c["V"], fields[sheet])).max() <= 1e-13


@pytest.mark.parametrize("name", ["sphere_deg1", "sphere_deg2", "sheets_split", "sheets_axis", "knot"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("method", [0, 1])
def test_solve_residual(cf, ctx, name, precision, method):
    h, s, o = built(cf, ctx, name)
    c = CASES[name]
    t = 1e-4 if name == "knot" else 1e-3
    b = o.load_vector(c["f"])
    # the restricted quadratic space is nearly rank-deficient on flat facets
    # and needs several hundred iterations
    rtol = 1e-8
    iters = (600 if c["degree"] == 1 else 1500) if method == 0 else 60
    say(f"[gpu] solve {name} precision={precision} method={method}")
    x, st = cf.camfe_solve(s, b, t=t, rtol=rtol if method == 0 else 1e-30, max_iter=iters,
                           precision=precision, method=method)
    Mo, Lo = o.matrices(c["depth"])
    A = Mo + t * Lo
    r = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
    if method == 0:
        assert st["converged"], st
        assert np.all(r <= 1e-6), r
        assert st["rel_residual"] <= rtol
    else:
        # stationary cycles: the residual after the same number of cycles as the
        # oracle's.  FP64 cycles repeat the oracle's arithmetic up to summation
        # order; FP32 sweeps (with the FP64 residual of every cycle) change each
        # correction by about 1e-7 relative, and over 60 cycles of contraction
        # 0.85-0.95 that moves the residual by well under 1 %.
        xo, io = o.solve(t, b, rtol=1e-30, max_iter=iters, mode="vcycle")
        assert st["iterations"] == iters and io["iterations"] == iters
        ro = io["history"][-1]
        rg = float(r.max())
        tol = 1e-9 if precision == 0 else 1e-2
        say(f"[gpu] stationary {name} p{precision}: gpu {rg:.6e} oracle {ro:.6e}")
        # (the singular axis-aligned sheets reach the FP64 rounding floor, about
        # 1e-16 relative, within the 60 cycles: there both are noise)
        assert abs(rg - ro) <= tol * ro + 1e-14, (rg, ro)
        assert ro < io["history"][0]
        if precision == 0 and name != "sheets_axis":
            # (the axis-aligned sheets are singular: rounding moves x along the
            # null space without changing the residual)
            assert abs(x - xo).max() <= 1e-9 * abs(xo).max()


def test_stationary_cycles_track_oracle(cf, ctx):
    h, s, o = built(cf, ctx, "sphere_deg1")
    c = CASES["sphere_deg1"]
    b = o.load_vector(c["f"])
    for cyc in (1, 3):
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-30, max_iter=cyc, method=1)
        xo, io = o.solve(1e-3, b, rtol=1e-30, max_iter=cyc, mode="vcycle")
        assert abs(x - xo).max() <= 1e-9 * abs(xo).max(), cyc


def test_large_direct_coarsest_tracks_oracle(cf, ctx):
    """Coarsest depth with ~2k functions solved through the blocked dense
    inverse: stationary cycles match the oracle's (dense Cholesky) cycles."""
    c = CASES["sphere_deg1"]
    h = cf.camfe_hierarchy_build(ctx, c["V"], c["F"], depth=5, max_coarse=2048)
    s = cf.camfe_assemble(h)
    o = Oracle(c["V"], c["F"], 5, max_coarse=2048).check().assemble()
    fin, d0 = cf.camfe_hierarchy_levels(h)
    assert d0 == o.coarsest and cf.camfe_hierarchy_info(h, d0)[2] > 1024
    b = o.load_vector(c["f"])
    for cyc in (1, 3):
        say(f"[gpu] large coarsest: {cyc} cycles")
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-30, max_iter=cyc, method=1)
        xo, io = o.solve(1e-3, b, rtol=1e-30, max_iter=cyc, mode="vcycle")
        assert st["eps_regularised"] == 1
        assert abs(x - xo).max() <= 1e-9 * abs(xo).max(), cyc
    for precision in (0, 1):
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-10, max_iter=200, precision=precision)
        Mo, Lo = o.matrices(5)
        r = np.linalg.norm(b - (Mo + 1e-3 * Lo) @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert st["converged"] and np.all(r <= 1e-9), (precision, r)
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_reassemble_mass_with_triangle_weights(cf, ctx):
    # the first re-weighting runs the quadrature (and keeps each pair's degree-1
    # block); the later ones weight the kept blocks: all must match the oracle
    c = CASES["knot"]
    h = cf.camfe_hierarchy_build(ctx, c["V"], c["F"], depth=6, max_coarse=256)
    s = cf.camfe_assemble(h)
    rng = np.random.default_rng(7)
    fin, d0 = cf.camfe_hierarchy_levels(h)
    for w in (rng.uniform(0.5, 1.5, len(c["F"])), rng.uniform(0.1, 3.0, len(c["F"])), None):
        say(f"[gpu] reassemble mass, weights {'none' if w is None else 'random'}")
        cf.camfe_reassemble_mass(s, w)
        o = Oracle(c["V"], c["F"], 6, max_coarse=256).check().assemble(tri_weight=w)
        for d in range(d0, fin + 1):
            Mo, Lo = o.matrices(d)
            M = cf.camfe_export_matrix(s, h, d, 0)
            L = cf.camfe_export_matrix(s, h, d, 1)
            assert abs(M - Mo).max() <= 1e-12 * abs(Mo).max()
            assert abs(L - Lo).max() <= 1e-12 * abs(Lo).max()
            assert abs(M - M.T).max() <= 1e-14 * abs(Mo).max()
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


@pytest.mark.parametrize("name", ["sphere_deg1", "sphere_deg2", "knot"])
def test_apply_matches_oracle_matrices(cf, ctx, name):
    h, s, o = built(cf, ctx, name)
    c = CASES[name]
    Mo, Lo = o.matrices(c["depth"])
    rng = np.random.default_rng(11)
    t = 1e-3
    for k in (1, 3, 6):
        say(f"[gpu] apply {name} k={k}")
        x = rng.standard_normal((Mo.shape[0], k))
        for which, A in ((0, Mo), (1, Lo), (2, Mo + t * Lo)):
            y = cf.camfe_apply(s, which, t, x)
            ref = A @ x
            assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), (which, k)


def test_cg_rejects_an_unsymmetric_cycle(cf, ctx):
    h, s, o = built(cf, ctx, "sphere_deg1")
    b = o.load_vector(CASES["sphere_deg1"]["f"])
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_solve(s, b, t=1e-3, nu_pre=1, nu_post=2)
    x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-30, max_iter=2, nu_pre=1, nu_post=2, method=1)
    assert st["iterations"] == 2


def test_kernel_measurement_and_references(cf, ctx):
    h, s, o = built(cf, ctx, "sheets_split")
    b = o.load_vector(CASES["sheets_split"]["f"])
    x1, st1 = cf.camfe_solve(s, b, t=1e-3, max_iter=600)
    say("measure: gs_colour, residual, spmv_dot, empty, copy")
    gs_ms, gs_by = cf.camfe_measure_kernel(s, "gs_colour", 0, 5)
    gs32_ms, gs32_by = cf.camfe_measure_kernel(s, "gs_colour", 1, 5)
    assert gs_ms > 0 and gs32_ms > 0 and 0 < gs32_by < gs_by
    for name in ("residual", "spmv_dot"):
        ms, by = cf.camfe_measure_kernel(s, name, 0, 5)
        assert ms > 0 and by > gs_by
    e_ms, e_by = cf.camfe_measure_kernel(s, "empty", 0, 5)
    assert e_ms > 0 and e_by == 0
    for _ in range(2):   # the copy's graph is rebuilt on new buffers each call
        c_ms, c_by = cf.camfe_measure_kernel(s, "copy", 0, 5)
        assert c_ms > 0 and abs(c_by - gs_by) <= 32
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_measure_kernel(s, "no_such_kernel")
    # whole cycles under a sweep schedule: a V(3,3)-cycle with V(1,1) below
    # sweeps more at the finest depth and less below than V(2,2)
    say("measure: vcycle, vcycle:3,1, vcycle:1,0")
    v22, vb = cf.camfe_measure_kernel(s, "vcycle", 0, 5)
    v31, _ = cf.camfe_measure_kernel(s, "vcycle:3,1", 0, 5)
    v11, _ = cf.camfe_measure_kernel(s, "vcycle:1,0", 0, 5)
    assert vb == 0 and v22 > 0 and v31 > 0 and 0 < v11 < v22
    for bad in ("vcycle:0,1", "vcycle:3", "vcycle:3,1x", "vcycle:17,1", "vcycle:3,-1"):
        with pytest.raises(cf.CamfeError, match="EINVAL"):
            cf.camfe_measure_kernel(s, bad, 0, 5)
    # the measurements leave the solver as it was: the same solve again
    x2, st2 = cf.camfe_solve(s, b, t=1e-3, max_iter=600)
    assert st1["converged"] and st2["iterations"] == st1["iterations"]
    assert np.array_equal(x1, x2)


def test_invalid_inputs_and_exports(cf, ctx):
    V = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5], [0.5, 1.5, 0.5]])
    F = np.array([[0, 1, 2]], np.int32)
    with pytest.raises(cf.CamfeError, match="grid plane"):
        cf.camfe_hierarchy_build(ctx, V, F, depth=2, box=[0, 0, 0, 2.0])
    with pytest.raises(cf.CamfeError, match="CAMFE_EINVAL"):
        cf.camfe_hierarchy_build(ctx, V, np.array([[0, 1, 7]], np.int32), depth=3)
    h, s, o = built(cf, ctx, "sphere_deg1")
    import ctypes
    lib = cf.load()
    n = ctypes.c_int64()
    k = np.zeros(4, np.uint64)
    t = np.zeros(4, np.int32)
    rc = lib.camfe_export_pairs(h, 5, k.ctypes.data_as(ctypes.c_void_p), t.ctypes.data_as(ctypes.c_void_p), 4,
                                ctypes.byref(n))
    assert rc == -6 and n.value > 4
    with pytest.raises(cf.CamfeError, match="CAMFE_ESTATE"):
        cf.camfe_export_functions(h, 0)


def test_full_size_two_sheets_properties(cf, ctx):
    """Config 2 at its full size (2 x 131,072 triangles, depth 8): properties
    that hold at any size, checked on the GPU's own exports - partition of
    unity, zero row sums, symmetry, the Galerkin identity at every depth, no
    coupling across the sheets in the split space - plus the FP64 and mixed
    solves to 1e-8 checked with the exported FP64 matrix."""
    V, F, f = meshgen.config_mesh("two_sheets_256")
    _, _, _, sheet = meshgen.two_sheets(256)
    say("[gpu] build two_sheets_256 depth 8")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=8, max_coarse=2048)
    s = cf.camfe_assemble(h)
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    fin, d0 = cf.camfe_hierarchy_levels(h)
    tri_sheet = sheet[F[:, 0]]
    mats = {}
    for d in range(d0, fin + 1):
        M = cf.camfe_export_matrix(s, h, d, 0)
        L = cf.camfe_export_matrix(s, h, d, 1)
        mats[d] = (M, L)
        assert abs(M.sum() - area) <= 1e-12 * area
        assert abs(L @ np.ones(L.shape[0])).max() <= 1e-11 * abs(L).max()
        assert abs(M - M.T).max() <= 1e-14 * abs(M).max()
        rep = cf.camfe_export_functions(h, d)[2]
        Mc = M.tocoo()
        assert np.all(tri_sheet[rep][Mc.row] == tri_sheet[rep][Mc.col])
    for d in range(d0 + 1, fin + 1):
        P = cf.camfe_export_prolongation(h, d)
        Mf, Lf = mats[d]
        Mc, Lc = mats[d - 1]
        assert abs(P.T @ Mf @ P - Mc).max() <= 1e-12 * abs(Mc).max()
        assert abs(P.T @ Lf @ P - Lc).max() <= 1e-12 * abs(Lc).max()
    b = cf.camfe_load_vector(s, h, f)
    M, L = mats[fin]
    for precision in (0, 1):
        say(f"[gpu] solve two_sheets_256 precision={precision}")
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-8, max_iter=500, precision=precision)
        r = np.linalg.norm(b - (M + 1e-3 * L) @ x) / np.linalg.norm(b)
        assert st["converged"] and r <= 1e-6, (st, r)
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_full_size_knot_flow_system(cf, ctx):
    """Config 3 at its full size ((3,5) knot tube, 2,097,152 triangles, depth
    10, t = 1e-4, three right-hand sides): partition of unity and zero row
    sums on the GPU's exports at the finest depth, and FP64, mixed-precision
    and learned-smoother solves to 1e-8 checked with the exported FP64
    matrices.  The mesh has rounding-sliver functions whose diagonal has no
    FP32 inverse; the mixed solve must skip them in its FP32 sweeps."""
    V, F = meshgen.torus_knot(nu=16384, nv=64, seed=3)
    say("[gpu] build knot 2M depth 10")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=10, max_coarse=4096)
    s = cf.camfe_assemble(h)
    fin, d0 = cf.camfe_hierarchy_levels(h)
    M = cf.camfe_export_matrix(s, h, fin, 0)
    L = cf.camfe_export_matrix(s, h, fin, 1)
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    # at this size a wrong (support, triangle) -> function label shows here: a
    # race in the component labelling once lost ~3e-8 of the area
    assert abs(M.sum() - area) <= 1e-12 * area
    assert abs(L @ np.ones(L.shape[0])).max() <= 1e-11 * abs(L).max()
    X0 = cf.camfe_linear_coeffs(s, h)
    b = M @ X0
    A = M + 1e-4 * L
    model = cf.camfe_model_create(None, levels=3, bf16=True)
    cf.camfe_smoother_attach(s, model)
    try:
        for precision, smoother in ((0, 0), (1, 0), (1, 2)):
            say(f"[gpu] solve knot 2M precision={precision} smoother={smoother}")
            x, st = cf.camfe_solve(s, b, t=1e-4, rtol=1e-8, max_iter=1500, precision=precision, smoother=smoother)
            r = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
            assert st["converged"] and not st["fell_back"] and np.all(r <= 1e-6), (precision, smoother, st, r)
    finally:
        cf.camfe_smoother_attach(s, None)
        cf.camfe_model_destroy(model)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)


def test_length_sorted_layout_on_a_7m_function_system(cf, ctx):
    """A noise-displaced sphere of 2,097,152 triangles at depth 10 (7.4M
    functions, about 930k rows per colour), whose finest colours take the
    length-sorted SELL order (colours of 2^19 rows or more).  Properties that
    hold at any size: partition of unity and zero row sums of the exports,
    and FP64 and mixed solves to 1e-8 checked with the exported FP64 matrices
    (the row order inside a colour changes no row's arithmetic)."""
    V, F = meshgen.noisy_sphere(9, seed=7, base="octa")
    say("[gpu] build noisy sphere 2M depth 10")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=10, max_coarse=4096)
    s = cf.camfe_assemble(h)
    fin, d0 = cf.camfe_hierarchy_levels(h)
    M = cf.camfe_export_matrix(s, h, fin, 0)
    L = cf.camfe_export_matrix(s, h, fin, 1)
    assert M.shape[0] >= 8 * (1 << 19)
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    assert abs(M.sum() - area) <= 1e-12 * area
    assert abs(L @ np.ones(L.shape[0])).max() <= 1e-11 * abs(L).max()
    b = cf.camfe_load_vector(s, h, V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)
    A = M + 1e-3 * L
    try:
        for precision in (0, 1):
            say(f"[gpu] solve noisy sphere 2M precision={precision}")
            x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-8, max_iter=1500, precision=precision)
            r = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
            assert st["converged"] and np.all(r <= 1e-6), (precision, st, r)
    finally:
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)


def test_headline_knot_at_full_size(cf, ctx):
    """The headline workload at its stated size: the held-out (3,5) knot tube
    of 65536 x 64 quads (8,388,608 triangles, jitter seed 5901) at depth 11,
    t = 1e-4, f = z + 0.1 x^2.  Properties that hold at any size, on the GPU's
    exports: partition of unity (M sums to the mesh area) and zero row sums of
    L at the finest depth, and prolongation rows that sum to exactly 1 (the
    dyadic weights of the parents of a fine function, Eq. (3), whatever
    component chi picks).  Each solver of the bench, with the sweep schedule
    the bench picks for it on this mesh, reaches 1e-8 checked with the
    exported FP64 matrices (the learned weights here are an untrained model's,
    which still go through the learned SOR kernels)."""
    V, F = meshgen.torus_knot(nu=65536, nv=64, seed=5901)
    say("[gpu] build knot 8.4M depth 11")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=11, max_coarse=4096)
    s = cf.camfe_assemble(h)
    fin, d0 = cf.camfe_hierarchy_levels(h)
    assert (fin, d0) == (11, 5)
    M = cf.camfe_export_matrix(s, h, fin, 0)
    L = cf.camfe_export_matrix(s, h, fin, 1)
    assert M.shape[0] > 9_000_000
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    assert abs(M.sum() - area) <= 1e-12 * area
    assert abs(L @ np.ones(L.shape[0])).max() <= 1e-11 * abs(L).max()
    for d in (fin, fin - 3, d0 + 1):
        P = cf.camfe_export_prolongation(h, d)
        assert np.array_equal(np.asarray(P.sum(axis=1)).ravel(), np.ones(P.shape[0])), d
    b = cf.camfe_load_vector(s, h, V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)
    A = M + 1e-4 * L
    model = cf.camfe_model_create(None, levels=3, bf16=True, sweep=1)
    cf.camfe_smoother_attach(s, model)
    try:
        for precision, smoother, (nu, nc) in ((0, 0, (3, 1)), (1, 0, (3, 1)), (1, 2, (3, 1)), (0, 3, (1, 0))):
            say(f"[gpu] solve knot 8.4M precision={precision} smoother={smoother} sweeps=({nu},{nc})")
            x, st = cf.camfe_solve(s, b, t=1e-4, rtol=1e-8, max_iter=500 if smoother == 3 else 3000,
                                   precision=precision, smoother=smoother, nu_pre=nu, nu_post=nu, nu_coarse=nc)
            r = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
            assert st["converged"] and not st["fell_back"] and np.all(r <= 1e-6), (precision, smoother, st, r)
    finally:
        cf.camfe_smoother_attach(s, None)
        cf.camfe_model_destroy(model)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)


def test_held_out_sphere_at_full_size(cf, ctx):
    """The second held-out mesh at its stated size: the octahedron subdivided
    ten times (8,388,608 triangles) with 16 Gaussian bumps (seed 5902), depth
    11, t = 1e-3 (30.5M functions, whose finest colours take the
    length-sorted layout).  Partition of unity and zero row sums of the
    exports at the finest depth, prolongation rows summing to 1, and the
    mixed solve to 1e-8 checked with the exported FP64 matrices."""
    V, F = meshgen.noisy_sphere(10, seed=5902, base="octa")
    say("[gpu] build noisy sphere 8.4M depth 11")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=11, max_coarse=4096)
    s = cf.camfe_assemble(h)
    fin, d0 = cf.camfe_hierarchy_levels(h)
    M = cf.camfe_export_matrix(s, h, fin, 0)
    assert M.shape[0] > 30_000_000
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    assert abs(M.sum() - area) <= 1e-12 * area
    L = cf.camfe_export_matrix(s, h, fin, 1)
    assert abs(L @ np.ones(L.shape[0])).max() <= 1e-11 * abs(L).max()
    P = cf.camfe_export_prolongation(h, fin)
    assert np.array_equal(np.asarray(P.sum(axis=1)).ravel(), np.ones(P.shape[0]))
    del P
    b = cf.camfe_load_vector(s, h, V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)
    try:
        say("[gpu] solve noisy sphere 8.4M, mixed")
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-8, max_iter=3000, precision=1)
        r = np.linalg.norm(b - M @ x - 1e-3 * (L @ x), axis=0) / np.linalg.norm(b, axis=0)
        assert st["converged"] and not st["fell_back"] and np.all(r <= 1e-6), (st, r)
    finally:
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)


@pytest.mark.parametrize("nu_coarse", [1, 3])
def test_coarse_sweep_count_tracks_oracle(cf, ctx, nu_coarse):
    """Fewer (or more) sweeps below the finest depth: stationary cycles track
    the oracle's cycles with the same counts, and CG still reaches 1e-8."""
    h, s, o = built(cf, ctx, "sphere_deg1")
    c = CASES["sphere_deg1"]
    b = o.load_vector(c["f"])
    for cyc in (1, 3):
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-30, max_iter=cyc, method=1, nu_coarse=nu_coarse)
        xo, _ = o.solve(1e-3, b, rtol=1e-30, max_iter=cyc, mode="vcycle", nu_coarse=nu_coarse)
        assert abs(x - xo).max() <= 1e-9 * abs(xo).max(), cyc
    for precision in (0, 1):
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-8, max_iter=600, precision=precision, nu_coarse=nu_coarse)
        Mo, Lo = o.matrices(c["depth"])
        r = np.linalg.norm(b - (Mo + 1e-3 * Lo) @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert st["converged"] and np.all(r <= 1e-6), (precision, r)
