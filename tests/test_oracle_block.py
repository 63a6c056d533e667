"""Pins of the oracle's cell-block Schwarz smoother (not in the paper: an
alternative to its Gauss-Seidel smoother, Section 5.2, for the trilinear
space).  A block holds the functions of one occupied cell; a sweep adds
omega sum_B w_B R_B^T A_B^-1 R_B r with r = b - A x and the block weight
w_B = 1 / (the largest number of blocks holding one of its functions).

Pinned here against things the definition fixes without restating it:
- a mesh inside one cell gives one block holding every function (weight 1),
  so one sweep is a dense solve of the (unit-diagonal-scaled, eps-shifted)
  system, checked against a library solver;
- the sweep is A-self-adjoint, <A S e, g> = <A e, S g> (a weight or scaling
  applied on one side only breaks it);
- the solution of A x = b is a fixed point (fails on a sign slip in the
  residual);
- the sweep is an A-norm contraction on these small cases at omega = 1
  (the largest eigenvalue of the weighted block sum times A is 1.15 on the
  sheets and 1.55 on the knot; it is not bounded by 2 in general, since
  blocks that share no function still couple, so the damping is an input):
  stationary cycles converge, and CG preconditioned by the cycle reaches the
  dense solution in fewer cycles than Gauss-Seidel on a knot tube;
- the damping scales the correction (the sweep is affine in omega), and a
  per-depth damping list equal to one value everywhere gives that value's
  cycles bit for bit, while changing only the finest depth's entry changes
  them.
"""
import numpy as np
import pytest
import scipy.linalg as la

from oracle import Oracle
from paper_1505_03615_amd import meshgen


def test_one_cell_mesh_is_one_dense_block():
    # a triangle strictly inside the cell [1, 2]^3 of the depth-2 grid on [0, 4]^3
    V = np.array([[1.2, 1.3, 1.25], [1.8, 1.35, 1.5], [1.4, 1.75, 1.8]])
    F = np.array([[0, 1, 2]], np.int32)
    o = Oracle(V, F, 2, max_coarse=0, min_depth=2, box=[0, 0, 0, 4.0]).check().assemble()
    assert len(o.cells(2)) == 1 and o.count(2, "functions") == 8
    M, L = o.matrices(2)
    A = (M + 0.3 * L).toarray()
    rng = np.random.default_rng(1)
    b = rng.normal(size=(8, 2))
    for eps in (1e-6, 1e-3):
        x = o.block_sweep(2, 0.3, b, np.zeros((8, 2)), forward=True, eps=eps, omega=1.0)
        s = 1.0 / np.sqrt(np.diag(A))
        ref = s[:, None] * la.solve(A * np.outer(s, s) + eps * np.eye(8), s[:, None] * b, assume_a="pos")
        assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max(), eps



@pytest.mark.parametrize("mesh", ["sheets", "knot"])
def test_sweep_is_self_adjoint_and_contracts(mesh):
    if mesh == "sheets":
        V, F, _, _ = meshgen.two_sheets(16, 1.0 / 64)      # split supports: blocks of up to 16
        o = Oracle(V, F, 5, max_coarse=0, min_depth=4).check().assemble()
        d, t = 5, 1e-3
    else:
        V, F = meshgen.torus_knot(nu=256, nv=12, seed=3)
        o = Oracle(V, F, 6, max_coarse=0, min_depth=5).check().assemble()
        d, t = 6, 1e-4
    M, L = o.matrices(d)
    A = M + t * L
    n = A.shape[0]
    rng = np.random.default_rng(7)
    e, g = rng.normal(size=n), rng.normal(size=n)
    zero = np.zeros(n)
    Se = o.block_sweep(d, t, zero, e)[:, 0]     # e - W A e
    Sg = o.block_sweep(d, t, zero, g)[:, 0]
    lhs, rhs = (A @ Se) @ g, (A @ e) @ Sg
    assert abs(lhs - rhs) <= 1e-12 * (abs(A @ e) @ abs(g))
    # the sweep reduces the A-norm of any error (a contraction)
    for v in (e, g):
        assert (A @ o.block_sweep(d, t, zero, v)[:, 0]) @ o.block_sweep(d, t, zero, v)[:, 0] < (A @ v) @ v


def test_solution_is_a_fixed_point():
    V, F = meshgen.icosphere(2)
    o = Oracle(V, F, 4, max_coarse=0, min_depth=3).check().assemble()
    M, L = o.matrices(4)
    A = (M + 1e-2 * L).toarray()
    x = np.random.default_rng(3).normal(size=(A.shape[0], 2))
    b = A @ x
    y = o.block_sweep(4, 1e-2, b, x)
    assert np.abs(y - x).max() <= 1e-10 * np.abs(x).max()


def test_block_cycles_precondition_cg_to_the_dense_solution():
    V, F = meshgen.torus_knot(nu=512, nv=16, seed=3)
    o = Oracle(V, F, 6, max_coarse=256).check().assemble()
    f = V[:, 2] + 0.1 * V[:, 0] ** 2
    b = o.load_vector(f)
    M, L = o.matrices(6)
    A = M + 1e-4 * L
    xg, ig = o.solve(1e-4, b, rtol=1e-11, max_iter=500)
    xb, ib = o.solve(1e-4, b, rtol=1e-11, max_iter=500, smoother="block")
    assert ib["converged"] and ig["converged"]
    assert np.linalg.norm(b - A @ xb) <= 1e-11 * np.linalg.norm(b)
    # (the knot's matrix has rounding-sliver rows of zero mass, so compare the
    # two solutions where they mean something: at the mesh vertices)
    ub, ug = o.eval_vertices(xb), o.eval_vertices(xg)
    assert np.abs(ub - ug).max() <= 1e-8 * np.abs(ug).max()
    assert ib["cycles"] < 0.5 * ig["cycles"]
    # on a nonsingular system the dense solution itself
    Vs, Fs = meshgen.icosphere(2)
    os_ = Oracle(Vs, Fs, 4, max_coarse=64).check().assemble()
    bs = os_.load_vector(Vs[:, 2])
    Ms, Ls = os_.matrices(4)
    xd = la.solve((Ms + 1e-2 * Ls).toarray(), bs, assume_a="pos")
    xs, ist = os_.solve(1e-2, bs, rtol=1e-12, max_iter=300, smoother="block")
    assert np.abs(xs - xd).max() <= 1e-8 * np.abs(xd).max()
    # stationary block cycles converge
    _, iv = o.solve(1e-4, b, rtol=1e-30, max_iter=25, mode="vcycle", smoother="block")
    assert iv["history"][-1] < 1e-5 and iv["history"][-1] < 1e-2 * iv["history"][5]
    Vi, Fi = meshgen.icosphere(1)
    o2 = Oracle(Vi, Fi, 3, degree=2, max_coarse=64).check().assemble()
    with pytest.raises(RuntimeError, match="degree 1"):
        o2.solve(1e-3, np.ones(o2.count(3, "functions")), smoother="block")


def test_damping_scales_the_correction_and_applies_per_depth():
    V, F = meshgen.torus_knot(nu=256, nv=12, seed=3)
    o = Oracle(V, F, 6, max_coarse=0, min_depth=4).check().assemble()
    d, t = 6, 1e-4
    n = o.count(d, "functions")
    rng = np.random.default_rng(11)
    b, x = rng.normal(size=(n, 2)), rng.normal(size=(n, 2))
    full = o.block_sweep(d, t, b, x, omega=1.0) - x
    part = o.block_sweep(d, t, b, x, omega=0.37) - x
    assert np.abs(part - 0.37 * full).max() <= 1e-12 * np.abs(full).max()
    levels = d - o.coarsest + 1
    assert levels == 3
    f = V[:, 2:3] + 0.1 * V[:, 0:1] ** 2
    bb = o.load_vector(f)
    x1, _ = o.solve(t, bb, rtol=1e-30, max_iter=2, mode="vcycle", smoother="block", block_omega=0.5)
    x2, _ = o.solve(t, bb, rtol=1e-30, max_iter=2, mode="vcycle", smoother="block", block_omega=[0.5] * levels)
    assert np.array_equal(x1, x2)
    x3, _ = o.solve(t, bb, rtol=1e-30, max_iter=2, mode="vcycle", smoother="block",
                    block_omega=[0.5] * (levels - 1) + [0.3])
    assert not np.array_equal(x1, x3)
    with pytest.raises(ValueError):
        o.solve(t, bb, max_iter=1, smoother="block", block_omega=[0.5] * (levels + 1))
