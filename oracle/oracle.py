"""ctypes front end of the C++ oracle (test infrastructure only).

Every method mirrors one exported function of oracle.cpp; arrays cross as
numpy buffers.  Matrices come back as scipy CSR.  The oracle is independent of
the HIP library: it shares no code with it and never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SO = os.path.join(HERE, "liboracle.so")
ORACLE_OMP_SO = os.path.join(HERE, "liboracle_omp.so")
ORACLE_SRC = os.path.join(HERE, "oracle.cpp")


def build_oracle(force: bool = True) -> str:
    """Compile oracle.cpp with g++ (-O2, no FP contraction, no -march=native),
    sequential (liboracle.so) and with OpenMP row loops (liboracle_omp.so, the
    benchmark's all-cores timing only)."""
    for so, extra in ((ORACLE_SO, []), (ORACLE_OMP_SO, ["-fopenmp"])):
        if force or not os.path.exists(so):
            tmp = so + ".tmp"
            subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-shared", "-fPIC"] + extra +
                                  [ORACLE_SRC, "-o", tmp])
            os.replace(tmp, so)
    return ORACLE_SO


_libs = {}


def _load(openmp=False):
    so = ORACLE_OMP_SO if openmp else ORACLE_SO
    if so not in _libs:
        if not os.path.exists(so):
            build_oracle(force=True)
        lib = C.CDLL(so)
        vp, L, I, D = C.c_void_p, C.c_long, C.c_int, C.c_double
        P = C.c_void_p
        lib.oracle_build.restype = vp
        lib.oracle_build.argtypes = [P, L, P, L, I, I, I, I, L, P]
        lib.oracle_ok.argtypes = [vp]
        lib.oracle_error.argtypes = [vp]; lib.oracle_error.restype = C.c_char_p
        lib.oracle_free.argtypes = [vp]
        lib.oracle_cube.argtypes = [vp, P]
        lib.oracle_coarsest.argtypes = [vp]
        lib.oracle_timing.argtypes = [vp, I]; lib.oracle_timing.restype = D
        lib.oracle_count.argtypes = [vp, I, I]; lib.oracle_count.restype = L
        lib.oracle_pairs.argtypes = [vp, I, P, P]
        lib.oracle_functions.argtypes = [vp, I, P, P, P]
        lib.oracle_support_entries.argtypes = [vp, I, P, P, P]
        lib.oracle_prolongation.argtypes = [vp, I, P, P, P]
        lib.oracle_assemble.argtypes = [vp, P]
        lib.oracle_matrix.argtypes = [vp, I, P, P, P, P]
        lib.oracle_load_vector.argtypes = [vp, I, P, I, P]
        lib.oracle_solve.argtypes = [vp, D, D, I, I, I, P, I, P, I, P, P, I, D, I, I, I, D, P]
        lib.oracle_block_sweep.argtypes = [vp, I, D, P, I, P, I, D, D]
        lib.oracle_gradient_load.argtypes = [vp, I, P, I, P]
        lib.oracle_apply.argtypes = [vp, I, D, P, I, P]
        lib.oracle_gs_sweep.argtypes = [vp, I, D, P, I, P, I]
        lib.oracle_eval_vertices.argtypes = [vp, P, I, P]
        lib.oracle_linear_coeffs.argtypes = [vp, P]
        _libs[so] = lib
    return _libs[so]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _colmajor(a, n):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    assert a.shape[0] == n
    return np.asfortranarray(a), a.shape[1]


class Oracle:
    """Hierarchy + matrices + solver for one mesh (all FP64, CPU)."""

    def __init__(self, V, F, depth, degree=1, split=1, min_depth=0, max_coarse=2048, box=None, openmp=False):
        """openmp: use the build whose row loops run on all OpenMP threads
        (same results; for timing only)."""
        self.lib = _load(openmp)
        self.V = np.ascontiguousarray(V, dtype=np.float64)
        self.F = np.ascontiguousarray(F, dtype=np.int32)
        self.depth, self.degree = depth, degree
        bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
        self.h = self.lib.oracle_build(_p(self.V), len(self.V), _p(self.F), len(self.F), depth,
                                       degree, split, min_depth, max_coarse,
                                       None if bx is None else _p(bx))
        self.ok = bool(self.lib.oracle_ok(self.h))
        self.error = self.lib.oracle_error(self.h).decode()

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.oracle_free(self.h)
            self.h = None

    def check(self):
        if not self.ok:
            raise RuntimeError("oracle: " + self.error)
        return self

    @property
    def coarsest(self):
        return self.lib.oracle_coarsest(self.h)

    def cube(self):
        out = np.zeros(4)
        self.lib.oracle_cube(self.h, _p(out))
        return out

    def timing(self):
        return {k: self.lib.oracle_timing(self.h, i)
                for i, k in enumerate(("build", "assemble", "setup", "solve"))}

    def count(self, d, what):
        return self.lib.oracle_count(self.h, d, {"pairs": 0, "functions": 1, "entries": 2,
                                                 "prolongation": 3, "nnz": 4, "cells": 5}[what])

    def pairs(self, d):
        n = self.count(d, "pairs")
        k = np.zeros(n, np.uint64); t = np.zeros(n, np.int32)
        self.lib.oracle_pairs(self.h, d, _p(k), _p(t))
        return k, t

    def cells(self, d):
        return np.unique(self.pairs(d)[0])

    def functions(self, d):
        n = self.count(d, "functions")
        k = np.zeros(n, np.uint64); c = np.zeros(n, np.int32); r = np.zeros(n, np.int32)
        self.lib.oracle_functions(self.h, d, _p(k), _p(c), _p(r))
        return k, c, r

    def support_entries(self, d):
        n = self.count(d, "entries")
        k = np.zeros(n, np.uint64); t = np.zeros(n, np.int32); f = np.zeros(n, np.int32)
        self.lib.oracle_support_entries(self.h, d, _p(k), _p(t), _p(f))
        return k, t, f

    def prolongation(self, d):
        """P_d: rows = functions at depth d, columns = functions at d-1 (scipy CSR)."""
        import scipy.sparse as sp
        nnz = self.count(d, "prolongation")
        nf, nc = self.count(d, "functions"), self.count(d - 1, "functions")
        ptr = np.zeros(nf + 1, np.int64); col = np.zeros(nnz, np.int32); w = np.zeros(nnz)
        self.lib.oracle_prolongation(self.h, d, _p(ptr), _p(col), _p(w))
        return sp.csr_matrix((w, col, ptr), shape=(nf, nc))

    def assemble(self, tri_weight=None):
        tw = None if tri_weight is None else np.ascontiguousarray(tri_weight, dtype=np.float64)
        if self.lib.oracle_assemble(self.h, None if tw is None else _p(tw)) != 0:
            raise RuntimeError("oracle assemble: " + self.lib.oracle_error(self.h).decode())
        return self

    def matrices(self, d):
        import scipy.sparse as sp
        n, nnz = self.count(d, "functions"), self.count(d, "nnz")
        ptr = np.zeros(n + 1, np.int64); col = np.zeros(nnz, np.int32)
        m = np.zeros(nnz); l = np.zeros(nnz)
        self.lib.oracle_matrix(self.h, d, _p(ptr), _p(col), _p(m), _p(l))
        return (sp.csr_matrix((m, col, ptr), shape=(n, n)), sp.csr_matrix((l, col, ptr), shape=(n, n)))

    def load_vector(self, fv, d=None):
        d = self.depth if d is None else d
        fv, k = _colmajor(fv, len(self.V))
        b = np.zeros((self.count(d, "functions"), k), order="F")
        if self.lib.oracle_load_vector(self.h, d, _p(fv), k, _p(b)) != 0:
            raise RuntimeError("oracle load vector failed")
        return b

    def gradient_load(self, fv, d=None):
        """b_i = int <grad f, grad b_i> for f linear on each triangle (Section 5.2)."""
        d = self.depth if d is None else d
        fv, k = _colmajor(fv, len(self.V))
        b = np.zeros((self.count(d, "functions"), k), order="F")
        if self.lib.oracle_gradient_load(self.h, d, _p(fv), k, _p(b)) != 0:
            raise RuntimeError("oracle gradient load failed")
        return b

    def eigenvalues(self, k, d=None):
        """The k smallest generalised eigenvalues L x = lambda M x at depth d
        (Section 5.1), by a dense symmetric solve of the unit-diagonal-scaled
        pair (the scaling keeps the eigenvalues).  Functions of zero computed
        mass have all-zero rows and columns in both matrices and are left out."""
        import scipy.linalg as la
        d = self.depth if d is None else d
        M, L = self.matrices(d)
        m = M.diagonal()
        keep = m > 0.0
        s = 1.0 / np.sqrt(m[keep])
        Ms = M[keep][:, keep].toarray() * np.outer(s, s)
        Ls = L[keep][:, keep].toarray() * np.outer(s, s)
        return la.eigh(Ls, Ms, eigvals_only=True, subset_by_index=[0, k - 1])

    def solve(self, t, b, rtol=1e-10, max_iter=200, nu1=2, nu2=2, x0=None, mode="pcg",
              coarse_eps=1e-6, gamma=1, nu_coarse=0, smoother="gs", block_omega=1.0):
        """mode 'pcg' (CG preconditioned by one cycle) or 'vcycle' (stationary
        cycles); gamma 1 for V-cycles, 2 for W-cycles; nu_coarse > 0 sweeps
        each way below the finest depth; smoother 'gs' (multicolour
        Gauss-Seidel) or 'block' (cell-block Schwarz, degree 1, corrections
        damped by block_omega: one value, or one per depth, coarsest first)."""
        n = self.count(self.depth, "functions")
        b, k = _colmajor(b, n)
        level_omega = None
        if np.ndim(block_omega) > 0:
            level_omega = np.ascontiguousarray(block_omega, dtype=np.float64)
            if level_omega.shape != (self.depth - self.coarsest + 1,):
                raise ValueError("block_omega: one value per depth from the coarsest")
            block_omega = 0.0
        x = np.zeros((n, k), order="F") if x0 is None else np.array(_colmajor(x0, n)[0], order="F")
        stats = np.zeros(5); hist = np.zeros(max_iter + 1)
        rc = self.lib.oracle_solve(self.h, t, rtol, max_iter, nu1, nu2, _p(b), k, _p(x),
                                   0 if x0 is None else 1, _p(stats), _p(hist),
                                   {"vcycle": 0, "pcg": 1}[mode], coarse_eps, gamma, nu_coarse,
                                   {"gs": 0, "block": 1}[smoother], block_omega,
                                   None if level_omega is None else _p(level_omega))
        if rc < 0:
            raise RuntimeError("oracle solve: " + self.lib.oracle_error(self.h).decode())
        it = int(stats[4])
        info = {"cycles": int(stats[0]), "iterations": it, "rel_residual": stats[1],
                "eps_regularised": int(stats[2]), "seconds": stats[3],
                "history": hist[: it + 1].copy(), "converged": rc == 0}
        return x, info

    def apply(self, d, t, x):
        n = self.count(d, "functions")
        x, k = _colmajor(x, n)
        y = np.zeros((n, k), order="F")
        self.lib.oracle_apply(self.h, d, t, _p(x), k, _p(y))
        return y

    def gs_sweep(self, d, t, b, x, forward=True):
        n = self.count(d, "functions")
        b, k = _colmajor(b, n)
        x = np.array(_colmajor(x, n)[0], order="F")
        self.lib.oracle_gs_sweep(self.h, d, t, _p(b), k, _p(x), 1 if forward else 0)
        return x

    def block_sweep(self, d, t, b, x, forward=True, eps=1e-6, omega=1.0):
        """One cell-block Schwarz sweep at depth d (degree 1), damped by omega."""
        n = self.count(d, "functions")
        b, k = _colmajor(b, n)
        x = np.array(_colmajor(x, n)[0], order="F")
        if self.lib.oracle_block_sweep(self.h, d, t, _p(b), k, _p(x), 1 if forward else 0, eps, omega) != 0:
            raise RuntimeError("oracle block sweep: " + self.lib.oracle_error(self.h).decode())
        return x

    def eval_vertices(self, x):
        n = self.count(self.depth, "functions")
        x, k = _colmajor(x, n)
        out = np.zeros((len(self.V), k), order="F")
        self.lib.oracle_eval_vertices(self.h, _p(x), k, _p(out))
        return out

    def linear_coeffs(self):
        n = self.count(self.depth, "functions")
        X = np.zeros((n, 3), order="F")
        self.lib.oracle_linear_coeffs(self.h, _p(X))
        return X
