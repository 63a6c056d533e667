"""Pins of the oracle's colour-fitting pieces (Section 5.2, Figure cubes).

The gradient constraint b_i = int <grad f, grad b_i> is pinned by linear
reproduction (a linear f is sum_i (a . node_i) b_i exactly, at both degrees
and through the split, so its constraint must equal L times those
coefficients), by the partition of unity (the constraints of any f sum to
zero), and on a flat square with f = x by the boundary integral that the
fundamental theorem of calculus gives (independent of the assembled L).  The W-cycle is pinned against a textbook composition written here
from the oracle's sweep, prolongation and matrix exports.  The
minimum-depth experiment of Figure cubes reproduces the paper's qualitative
finding: with the split, coarse corrections keep reducing the residual of
one W-cycle; without it they stop helping below the finest depths.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1505_03615_amd import meshgen

ALPHA = 0.01


@pytest.fixture(scope="module", params=[1, 2], ids=["degree1", "degree2"])
def sphere(request):
    V, F = meshgen.icosphere(2)
    return Oracle(V, F, 4, degree=request.param, max_coarse=64).check().assemble()


def _linear_coeffs(o):
    n = o.count(o.depth, "functions")
    X = np.zeros((n, 3), order="F")
    o.lib.oracle_linear_coeffs(o.h, X.ctypes.data_as(__import__("ctypes").c_void_p))
    return X


def test_gradient_load_of_linear_function_is_stiffness_times_nodes(sphere):
    o = sphere
    X = _linear_coeffs(o)
    _, L = o.matrices(o.depth)
    a = np.array([[0.3, -1.1, 0.7], [1.0, 0.0, 0.0], [0.0, 0.0, 2.0]]).T   # three directions
    fv = o.V @ a
    g = o.gradient_load(fv)
    want = L @ (X @ a)
    assert np.abs(g - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(want).max() > 1e-3   # not trivially zero


def test_gradient_load_sums_to_zero_for_any_f(sphere):
    o = sphere
    f = np.random.default_rng(21).normal(size=(len(o.V), 2))
    g = o.gradient_load(f)
    assert np.all(np.abs(g.sum(0)) <= 1e-13 * np.abs(g).sum(0))
    assert np.all(np.abs(o.gradient_load(np.full(len(o.V), 3.5))) <= 1e-15)


def test_gradient_load_sees_only_the_tangential_gradient():
    # f = z on the flat sheet z = const has zero surface gradient
    V, F, _, _ = meshgen.two_sheets(8, gap=0.25, rotate=False)
    o = Oracle(V + 0.0137, F, 4, max_coarse=64).check().assemble()
    assert np.abs(o.gradient_load(V[:, 2])).max() <= 1e-15
    assert np.abs(o.gradient_load(V[:, 0])).max() > 1e-3


def _textbook_cycle(o, t, b, x, d, nu, gamma, coarsest, nu_below=None):
    """One multigrid cycle at depth d written out from the definition: nu
    forward sweeps, residual, restriction by P^T, gamma cycles at d - 1 from
    zero (with nu_below sweeps when given), prolongation, nu reverse sweeps;
    the coarsest depth only relaxes."""
    below = nu if nu_below is None else nu_below
    if d == coarsest:
        for _ in range(nu):
            x = o.gs_sweep(d, t, b, x, forward=True)
        for _ in range(nu):
            x = o.gs_sweep(d, t, b, x, forward=False)
        return x
    for _ in range(nu):
        x = o.gs_sweep(d, t, b, x, forward=True)
    M, L = o.matrices(d)
    r = b - (M + t * L) @ x
    P = o.prolongation(d)
    bc = P.T @ r
    xc = np.zeros_like(bc)
    for _ in range(gamma):
        xc = _textbook_cycle(o, t, bc, xc, d - 1, below, gamma, coarsest, nu_below)
    x = x + P @ xc
    for _ in range(nu):
        x = o.gs_sweep(d, t, b, x, forward=False)
    return x


@pytest.mark.parametrize("gamma,nu_coarse", [(1, 0), (2, 0), (1, 1), (2, 2)])
def test_cycle_matches_textbook_composition(gamma, nu_coarse):
    V, F = meshgen.icosphere(2)
    o = Oracle(V, F, 5, min_depth=2, max_coarse=0).check().assemble()
    assert o.coarsest == 2
    t = 0.1
    n = o.count(5, "functions")
    rng = np.random.default_rng(5)
    b = rng.normal(size=(n, 2))
    x0 = rng.uniform(0, 1, size=(n, 2))
    x, _ = o.solve(t, b, rtol=0.0, max_iter=1, nu1=3, nu2=3, x0=x0, mode="vcycle", gamma=gamma,
                   nu_coarse=nu_coarse)
    # the stationary step is x0 + cycle(b - A x0) with a zero start
    M, L = o.matrices(5)
    e = _textbook_cycle(o, t, b - (M + t * L) @ x0, np.zeros_like(b), 5, 3, gamma, 2,
                        nu_coarse if nu_coarse > 0 else None)
    assert np.abs(x - (x0 + e)).max() <= 1e-12 * np.abs(x).max()


def test_w_cycle_equals_v_cycle_over_two_levels_with_exact_coarse_solve():
    V, F = meshgen.icosphere(2)
    n3 = Oracle(V, F, 4, min_depth=3, max_coarse=0).check().count(3, "functions")
    o = Oracle(V, F, 4, min_depth=3, max_coarse=n3).check().assemble()   # depth 3 solved directly
    assert o.coarsest == 3
    n = o.count(4, "functions")
    b = np.random.default_rng(8).normal(size=(n, 1))
    xv, _ = o.solve(1e-2, b, rtol=0.0, max_iter=2, mode="vcycle", gamma=1)
    xw, _ = o.solve(1e-2, b, rtol=0.0, max_iter=2, mode="vcycle", gamma=2)
    assert np.array_equal(xv, xw)


def _one_w_cycle_residual(V, F, col, depth, split, min_depth):
    o = Oracle(V, F, depth, split=split, min_depth=min_depth, max_coarse=0).check().assemble()
    # (L + alpha M) u = g + alpha s  <=>  (M + L / alpha) u = (g + alpha s) / alpha
    b = (o.gradient_load(col) + ALPHA * o.load_vector(col)) / ALPHA
    n = b.shape[0]
    x0 = np.random.default_rng(6200).uniform(0.0, 1.0, size=(n, 3))
    x, _ = o.solve(1.0 / ALPHA, b, rtol=0.0, max_iter=1, nu1=10, nu2=10, x0=x0, mode="vcycle", gamma=2)
    r = ALPHA * (b - o.apply(depth, 1.0 / ALPHA, x))
    return (np.linalg.norm(r, axis=0) / np.linalg.norm(x0, axis=0)).max(), n


def test_minimum_depth_experiment_reproduces_figure_cubes():
    V, F, col = meshgen.cubes_checker(n=4, subdiv=2)
    D = 4
    split = [_one_w_cycle_residual(V, F, col, D, 1, m) for m in range(D + 1)]
    plain = [_one_w_cycle_residual(V, F, col, D, 0, m) for m in range(D + 1)]
    # the cubes are farther apart than a finest support: both spaces agree there
    assert split[D][1] == plain[D][1]
    assert abs(split[D][0] - plain[D][0]) <= 1e-12 * plain[D][0]
    rs = np.array([r for r, _ in split])
    rp = np.array([r for r, _ in plain])
    # with the split, every coarser minimum depth helps (up to rounding), and
    # the full W-cycle gains three orders of magnitude over the finest alone
    assert np.all(rs[:-1] <= rs[1:] * (1 + 1e-6))
    assert rs[0] < 1e-3 * rs[D]
    # without it, the corrections below depth 2 change it by less than 0.1 %
    assert abs(rp[0] - rp[2]) <= 1e-3 * rp[2]
    assert rp[0] > 0.1 * rp[D]
    assert rs[0] < 1e-2 * rp[0]


def _hat_integral(c, h, a, b):
    """int_a^b max(0, 1 - |y - c| / h) dy, exact (trapezoid rule on the
    breakpoints of a piecewise-linear function)."""
    pts = np.unique(np.clip([a, b, c - h, c, c + h], a, b))
    v = np.maximum(0.0, 1.0 - np.abs(pts - c) / h)
    return float(np.sum(0.5 * (v[1:] + v[:-1]) * np.diff(pts)))


def test_gradient_load_on_a_flat_square_matches_the_boundary_integral():
    """Unit square [0,1]^2 at z = 0.3 (cells of an explicit cube, no face or
    edge on a grid plane), f = x: grad f = e_x on the sheet, so
    g_i = int_0^1 [b_i(1, y) - b_i(0, y)] dy, a product of trilinear hat
    values and one hat integral, for every function."""
    n = 10
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    V = np.stack([i.ravel() / n, j.ravel() / n, np.full(i.size, 0.3)], 1)
    q = (i[:-1, :-1] * (n + 1) + j[:-1, :-1]).ravel()
    F = np.concatenate([np.stack([q, q + n + 1, q + n + 2], 1), np.stack([q, q + n + 2, q + 1], 1)]).astype(np.int32)
    box = [-0.1, -0.1, 0.0, 1.25]
    D = 4
    o = Oracle(V, F, D, max_coarse=64, box=box).check().assemble()
    g = o.gradient_load(V[:, 0])[:, 0]
    X = _linear_coeffs(o)                      # node positions of the functions
    h = box[3] / 2 ** D
    hat = lambda u: np.maximum(0.0, 1.0 - np.abs(u) / h)
    want = np.array([hat(0.3 - z) * (hat(1.0 - x) - hat(0.0 - x)) * _hat_integral(y, h, 0.0, 1.0)
                     for x, y, z in X])
    assert np.abs(want).max() > 1e-3
    assert np.abs(g - want).max() <= 1e-13
