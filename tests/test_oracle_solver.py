"""Pins of the oracle's multigrid solver (Sections 3.2, 4.3, 5.2; the Discussion closing Section 5).

Against a dense direct solve, a textbook sequential Gauss-Seidel sweep, the
colour-independence that makes the multicolour order a Gauss-Seidel order,
and the consistent singular (planar) case.
"""
import numpy as np
import pytest
import scipy.linalg as la

from oracle import Oracle
from paper_1505_03615_amd import meshgen


def _decode(keys):
    k = keys.astype(np.int64)
    c = np.zeros((len(k), 3), np.int64)
    for b in range(21):
        for a in range(3):
            c[:, a] |= ((k >> (3 * b + a)) & 1) << b
    return c


@pytest.fixture(scope="module")
def small():
    V, F = meshgen.icosphere(2)
    o = Oracle(V, F, 4, max_coarse=64).check().assemble()
    rng = np.random.default_rng(11)
    f = V[:, 2] + rng.normal(0, 0.01, len(V))
    return o, o.load_vector(f)


def test_pcg_matches_dense_direct(small):
    o, b = small
    t = 1e-3
    x, info = o.solve(t, b, rtol=1e-11, mode="pcg")
    assert info["converged"] and info["rel_residual"] <= 1e-11
    M, L = o.matrices(o.depth)
    A = (M + t * L).toarray()
    xs = la.solve(A, b[:, 0], assume_a="pos")
    e = x[:, 0] - xs
    assert np.sqrt(e @ A @ e) <= 1e-9 * np.sqrt(xs @ A @ xs)
    r = b[:, 0] - A @ x[:, 0]
    assert np.linalg.norm(r) <= 1.0001e-11 * np.linalg.norm(b)


def test_stationary_vcycle_decreases_residual(small):
    o, b = small
    x, info = o.solve(1e-3, b, rtol=1e-30, max_iter=8, mode="vcycle")
    h = info["history"]
    assert len(h) == 9 and np.all(np.diff(h) < 0)
    assert h[1] < 0.1


def test_same_colour_rows_never_couple(small):
    o, _ = small
    for d in range(o.coarsest, o.depth + 1):
        M, L = o.matrices(d)
        col = (_decode(o.functions(d)[0]) & 1) @ np.array([1, 2, 4])
        A = (M + L).tocoo()
        off = A.row != A.col
        assert not np.any(col[A.row[off]] == col[A.col[off]])


def test_gs_sweep_equals_sequential_textbook(small):
    """One multicolour sweep equals plain row-by-row Gauss-Seidel visiting the
    rows colour by colour (0..7 forward, 7..0 reverse)."""
    o, b = small
    t = 1e-3
    d = o.depth
    M, L = o.matrices(d)
    A = (M + t * L).toarray()
    col = (_decode(o.functions(d)[0]) & 1) @ np.array([1, 2, 4])
    rng = np.random.default_rng(2)
    x0 = rng.normal(size=A.shape[0])
    for forward in (True, False):
        ref = x0.copy()
        order = range(8) if forward else range(7, -1, -1)
        for c in order:
            for i in np.where(col == c)[0]:
                ref[i] = (b[i, 0] - A[i] @ ref + A[i, i] * ref[i]) / A[i, i]
        got = o.gs_sweep(d, t, b, x0, forward=forward)[:, 0]
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-14 * abs(ref).max())


def test_multiple_rhs_columns_independent(small):
    o, b = small
    B = np.concatenate([b, 2 * b + 1e-4], axis=1)
    X, info = o.solve(1e-3, B, rtol=1e-10)
    x1, _ = o.solve(1e-3, B[:, 1:], rtol=1e-10)
    M, L = o.matrices(o.depth)
    A = M + 1e-3 * L
    for q in range(2):
        assert np.linalg.norm(B[:, q] - A @ X[:, q]) <= 1.0001e-10 * np.linalg.norm(B[:, q])
    assert np.allclose(X[:, 1], x1[:, 0], rtol=1e-6, atol=1e-8 * abs(x1).max())


def test_singular_planar_system_still_solves():
    """Planar sheets make (M + tL) singular (Discussion closing Section 5); the
    system stays consistent and the eps-regularised coarse solve keeps the
    iteration bounded."""
    V, F, xl, sheet = meshgen.two_sheets(32, gap=1.0 / 32, rotate=False)
    o = Oracle(V, F, 5, max_coarse=256).check().assemble()
    f = np.where(sheet == 0, 1.0, -1.0) * np.sin(6 * np.pi * xl)
    b = o.load_vector(f)
    x, info = o.solve(1e-3, b, rtol=1e-8, max_iter=300)
    assert info["converged"] and np.isfinite(info["rel_residual"]), info["history"][-5:]
    assert np.all(np.isfinite(x))
    M, L = o.matrices(5)
    r = b[:, 0] - (M + 1e-3 * L) @ x[:, 0]
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(b)
    # functions kept by a rounding-level overlap have all-zero rows and
    # columns: Gauss-Seidel never divides by their zero diagonal, and their
    # coefficient has no effect on A x
    zero = np.where(M.diagonal() == 0)[0]
    assert len(zero) > 0
    assert np.all(abs(M[zero]).sum(axis=1) == 0) and np.all(abs(L[zero]).sum(axis=1) == 0)
    assert np.all(abs(M[:, zero]).sum(axis=0) == 0)


def test_nan_right_hand_side_is_reported_not_converged(small):
    o, b = small
    bb = b.copy()
    bb[3, 0] = np.nan
    x, info = o.solve(1e-3, bb, rtol=1e-8, max_iter=5)
    assert not info["converged"] and not np.isfinite(info["rel_residual"])


def test_warm_start_and_zero_rhs(small):
    o, b = small
    x, _ = o.solve(1e-3, b, rtol=1e-10)
    x2, info = o.solve(1e-3, b, rtol=1e-10, x0=x)
    assert info["iterations"] == 0
    z, info = o.solve(1e-3, np.zeros_like(b), rtol=1e-10)
    assert np.all(z == 0)


def test_pcg_with_fewer_coarse_sweeps_still_matches_the_dense_solve(small):
    """One sweep each way below the finest depth keeps the cycle symmetric
    positive definite (forward before, reverse after, at every depth), so
    CG preconditioned by it reaches the same solution."""
    o, b = small
    t = 1e-3
    x, info = o.solve(t, b, rtol=1e-11, mode="pcg", nu_coarse=1)
    assert info["converged"]
    M, L = o.matrices(o.depth)
    A = (M + t * L).toarray()
    xs = la.solve(A, b[:, 0], assume_a="pos")
    e = x[:, 0] - xs
    assert np.sqrt(e @ A @ e) <= 1e-9 * np.sqrt(xs @ A @ xs)


def test_openmp_build_gives_the_same_bits():
    """The all-cores build shares independent rows among threads; every row is
    still one thread's sequential sum, so cycles, iterates and residual
    histories equal the sequential build's bit for bit."""
    V, F = meshgen.torus_knot(nu=512, nv=16, seed=3)
    f = V[:, 2] + 0.1 * V[:, 0] ** 2
    out = []
    for omp in (False, True):
        o = Oracle(V, F, 6, max_coarse=256, openmp=omp).check().assemble()
        b = o.load_vector(f)
        x, info = o.solve(1e-4, b, rtol=1e-10, max_iter=300)
        xs, infos = o.solve(1e-4, b, rtol=1e-30, max_iter=5, mode="vcycle")
        out.append((x, info["history"], xs, infos["history"]))
    for a, b in zip(*out):
        assert np.array_equal(a, b)
