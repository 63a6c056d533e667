"""Pins of the learned-smoother reference (oracle/learned.py).

Closed forms of damped Jacobi on eigenvectors of a circulant matrix (loss and
the one non-zero gradient entry), the contraction that the l1-Jacobi bound
guarantees for any network output, special networks that pass one feature
through (orientation of the packed weights), features of a synthetic chain
placed along one grid axis (offset indexing), invariants of the features of a
real hierarchy (centre entry 1, row sums = (M 1)_i / A_ii since L 1 = 0), and
central finite differences of the loss for the hand-derived gradient, for
both sweep types and for the two-grid loss; with unit weights the SOR sweep is
the oracle's own multicolour Gauss-Seidel sweep; the coarse correction with
the exact Galerkin inverse is an A-orthogonal projection and its adjoint is
its transpose.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Oracle
from oracle import learned as lr
from paper_1505_03615_amd import meshgen


def circulant_laplacian(n):
    A = sp.diags([np.full(n, 2.0), np.full(n - 1, -1.0), np.full(n - 1, -1.0)], [0, 1, -1], format="lil")
    A[0, n - 1] = -1.0
    A[n - 1, 0] = -1.0
    return A.tocsr()


def const_params(sg):
    p = np.zeros(lr.NP)
    p[lr.O_B3] = math.log((sg / 2.0) / (1.0 - sg / 2.0))   # 2 sigmoid(b3) = sg
    return p


def test_constant_omega_loss_and_gradient_closed_form():
    n, nu, sg = 32, 3, 1.4
    A = circulant_laplacian(n)
    ks = [3, 7]
    lam = np.array([2.0 - 2.0 * math.cos(2 * math.pi * k / n) for k in ks])
    E0 = np.stack([np.sin(2 * math.pi * k * np.arange(n) / n) for k in ks], axis=1)
    f = np.random.default_rng(0).normal(size=(n, lr.NF))
    act = np.ones(n, bool)
    c1 = np.full(n, 0.5)               # A_ii / sum_j |A_ij| = 2 / 4
    om = 0.5 * sg
    p = const_params(sg)
    assert np.allclose(lr.omega(p, f, act, c1), om, rtol=1e-15)
    # D^-1 A e = (lam / 2) e, so e_nu = (1 - om lam / 2)^nu e_0
    expect = np.mean([2 * nu * math.log(abs(1 - om * l / 2)) for l in lam])
    assert lr.loss(A, f, act, c1, p, E0, nu) == pytest.approx(expect, rel=1e-12)
    L, g = lr.loss_grad(A, f, act, c1, p, E0, nu)
    assert L == pytest.approx(expect, rel=1e-12)
    # only b3 moves omega when every weight is zero: dL/db3 = dL/dom * c s (1 - s / 2)
    dLdom = np.mean([2 * nu * (-l / 2) / (1 - om * l / 2) for l in lam])
    assert g[lr.O_B3] == pytest.approx(dLdom * 0.5 * sg * (1 - sg / 2), rel=1e-10)
    assert np.abs(np.delete(g, lr.O_B3)).max() == 0.0


def test_l1_bound_keeps_every_sweep_contracting():
    # any s in (0, 2): the sweep matrix I - W A has A-norm below 1 (W = diag(c s / A_ii))
    rng = np.random.default_rng(4)
    n = 40
    B = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.15)
    A = B @ B.T + 0.05 * np.eye(n)
    c1 = np.diag(A) / np.abs(A).sum(axis=1)
    for sg in (0.3, 1.0, 1.9, 1.999):
        W = np.diag(c1 * sg / np.diag(A))
        R = np.linalg.cholesky(A)
        T = R.T @ (np.eye(n) - W @ A) @ np.linalg.inv(R.T)   # similar in the A-inner product
        assert np.linalg.norm(T, 2) < 1.0
    # without the bound, omega = 1.9 plain Jacobi can expand the error
    W = np.diag(1.9 / np.diag(A))
    assert max(abs(np.linalg.eigvals(np.eye(n) - W @ A))) > 1.0


def test_network_orientation_passes_one_feature():
    rng = np.random.default_rng(1)
    f = rng.normal(size=(50, lr.NF))
    p = np.zeros(lr.NP)
    p[lr.O_W1 + 28 * lr.NH + 5] = 1.0     # feature 28 -> hidden 5
    p[lr.O_W2 + 5 * lr.NH + 9] = 2.0      # hidden 5 -> hidden 9
    p[lr.O_W3 + 9] = 0.5                  # hidden 9 -> z
    p[lr.O_B3] = -0.25
    z = lr.forward(p, f)[4]
    assert np.allclose(z, np.maximum(f[:, 28], 0) - 0.25, rtol=0, atol=1e-15)
    om = lr.omega(p, f, np.arange(50) % 7 != 0, np.ones(50))
    assert np.allclose(om[np.arange(50) % 7 != 0], 2 / (1 + np.exp(-(np.maximum(f[:, 28], 0) - 0.25)))[np.arange(50) % 7 != 0])
    assert np.all(om[np.arange(50) % 7 == 0] == 0)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.1415926, 0.0, 1e-30], dtype=np.float32)
    r = lr.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even mantissa
    assert r[2] == np.float32(1.0 + 4 * 2 ** -8)   # tie -> even (rounds up)
    assert r[3] == np.float32(-3.140625)
    assert r[4] == 0.0
    assert abs(r[5] - 1e-30) <= 2 ** -8 * 1e-30


def test_features_of_a_chain_along_y():
    # corners (0, j, 0), j = 0..5: neighbours at offsets (0, -1, 0) -> slot 10 and (0, 1, 0) -> slot 16
    n = 6
    keys = np.array([sum(((j >> b) & 1) << (3 * b + 1) for b in range(4)) for j in range(n)], dtype=np.uint64)
    assert np.array_equal(lr.demorton(keys)[:, 1], np.arange(n))
    Mm = sp.diags([np.full(n, 4.0), np.full(n - 1, 1.0), np.full(n - 1, 1.0)], [0, 1, -1], format="csr")
    Ll = sp.diags([np.full(n, 2.0), np.full(n - 1, -1.5), np.full(n - 1, -0.5)], [0, 1, -1], format="csr")
    A = (Mm + 0.1 * Ll).tocsr()
    f, act, c1 = lr.features(A, Mm, keys, 3, 5)
    assert act.all()
    a = A.toarray()
    for i in range(n):
        assert c1[i] == pytest.approx(a[i, i] / np.abs(a[i]).sum(), rel=1e-15)
        assert f[i, 13] == 1.0
        assert f[i, 10] == pytest.approx(a[i, i - 1] / a[i, i] if i > 0 else 0.0, abs=1e-15)
        assert f[i, 16] == pytest.approx(a[i, i + 1] / a[i, i] if i < n - 1 else 0.0, abs=1e-15)
        assert f[i, 28] == pytest.approx(4.0 / a[i, i], rel=1e-15)
        assert f[i, 29] == pytest.approx(0.2)
        others = np.delete(f[i, :27], [10, 13, 16])
        assert np.all(others == 0)
    assert f[:, 27].max() == 0.0


@pytest.fixture(scope="module")
def sphere():
    V, F = meshgen.icosphere(3)
    o = Oracle(V, F, 5, degree=1, max_coarse=0, min_depth=2).check().assemble()
    return o


def test_features_invariants_on_sphere(sphere):
    t = 1e-2
    for d in (sphere.depth, sphere.depth - 1):
        M, L = sphere.matrices(d)
        A = (M + t * L).tocsr()
        keys = sphere.functions(d)[0]
        f, act, c1 = lr.features(A, M, keys, d, sphere.depth)
        dg = A.diagonal()
        assert np.all(c1[act] > 0) and np.all(c1 <= 1) and np.all(c1[~act] == 0)
        assert np.all(f[act, 13] == 1.0)
        # L 1 = 0, so the entries of a row sum to (M 1)_i; none falls outside the 27 offsets
        rs = (M @ np.ones(M.shape[0]))[act] / dg[act]
        assert np.allclose(f[act, :27].sum(axis=1), rs, rtol=1e-12, atol=1e-12)
        assert np.all(f[act, 27] <= 0) and np.all(f[act, 27] >= -3)
        assert f[act, 27].max() == 0.0
        assert np.allclose(f[act, 28], M.diagonal()[act] / dg[act], rtol=1e-15)


def test_gradient_matches_central_differences(sphere):
    t, nu = 1e-2, 2
    d = sphere.depth
    M, L = sphere.matrices(d)
    A = (M + t * L).tocsr()
    f, act, c1 = lr.features(A, M, sphere.functions(d)[0], d, sphere.depth)
    rng = np.random.default_rng(7)
    p = rng.normal(size=lr.NP) * 0.3
    p[lr.O_B3] = -0.7
    E0 = rng.normal(size=(A.shape[0], 3))
    L0, g = lr.loss_grad(A, f, act, c1, p, E0, nu)
    assert L0 == pytest.approx(lr.loss(A, f, act, c1, p, E0, nu), rel=1e-14)
    assert L0 < 0
    idx = list(rng.choice(lr.O_B1, 6, replace=False)) + list(lr.O_B1 + rng.choice(lr.NH, 3, replace=False)) + \
        list(lr.O_W2 + rng.choice(lr.NH * lr.NH, 6, replace=False)) + \
        list(lr.O_B2 + rng.choice(lr.NH, 3, replace=False)) + list(lr.O_W3 + rng.choice(lr.NH, 3, replace=False)) + \
        [lr.O_B3]
    h = 1e-6
    checked = 0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (lr.loss(A, f, act, c1, pp, E0, nu) - lr.loss(A, f, act, c1, pm, E0, nu)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9 * max(1.0, abs(g).max())), i
        checked += abs(g[i]) > 1e-8
    assert checked >= 10      # most picked entries are live (ReLUs active)


def test_sor_with_unit_weights_is_the_oracle_gauss_seidel_sweep(sphere):
    t, d = 1e-2, sphere.depth
    M, L = sphere.matrices(d)
    A = (M + t * L).tocsr()
    keys = sphere.functions(d)[0]
    f, act, c1 = lr.features(A, M, keys, d, sphere.depth)
    col = lr.colours(keys)
    assert set(np.unique(col)) <= set(range(8))
    p = np.zeros(lr.NP)                     # z = 0: omega = 1/2 + sigmoid(0) = 1 on every row
    E0 = np.random.default_rng(3).normal(size=(A.shape[0], 2))
    E1 = lr.relax(A, f, act, c1, p, E0, 1, colour=col)
    G1 = sphere.gs_sweep(d, t, np.zeros_like(E0), E0, forward=True)
    assert np.abs(E1 - G1).max() <= 1e-12 * np.abs(E0).max()
    # two sweeps: the same sweep applied twice
    E2 = lr.relax(A, f, act, c1, p, E0, 2, colour=col)
    G2 = sphere.gs_sweep(d, t, np.zeros_like(E0), G1, forward=True)
    assert np.abs(E2 - G2).max() <= 1e-12 * np.abs(E0).max()


def test_sor_gradient_matches_central_differences(sphere):
    t, nu = 1e-2, 2
    d = sphere.depth
    M, L = sphere.matrices(d)
    A = (M + t * L).tocsr()
    keys = sphere.functions(d)[0]
    f, act, c1 = lr.features(A, M, keys, d, sphere.depth)
    col = lr.colours(keys)
    rng = np.random.default_rng(9)
    p = rng.normal(size=lr.NP) * 0.3
    p[lr.O_B3] = 0.3
    E0 = rng.normal(size=(A.shape[0], 2))
    L0, g = lr.loss_grad(A, f, act, c1, p, E0, nu, colour=col)
    assert L0 == pytest.approx(lr.loss(A, f, act, c1, p, E0, nu, colour=col), rel=1e-14)
    idx = list(rng.choice(lr.O_B1, 5, replace=False)) + list(lr.O_W2 + rng.choice(lr.NH * lr.NH, 5, replace=False)) + \
        list(lr.O_W3 + rng.choice(lr.NH, 3, replace=False)) + [lr.O_B3]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (lr.loss(A, f, act, c1, pp, E0, nu, colour=col) - lr.loss(A, f, act, c1, pm, E0, nu, colour=col)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9 * max(1.0, abs(g).max())), i


@pytest.fixture(scope="module")
def sphere_cc():
    """Sphere at depth 4 with a directly solved coarsest depth 3 (small enough
    for dense algebra)."""
    V, F = meshgen.icosphere(3)
    o = Oracle(V, F, 4, degree=1, max_coarse=512).check().assemble()
    assert o.coarsest == 3
    return o


def test_coarse_correction_is_a_projection_with_its_transpose_as_adjoint(sphere_cc):
    o, t = sphere_cc, 1e-2
    M, L = o.matrices(4)
    A = (M + t * L).tocsr()
    Mc, Lc = o.matrices(3)
    Ac = (Mc + t * Lc).tocsr()
    P = o.prolongation(4)
    assert abs(P.T @ A @ P - Ac).max() <= 1e-12 * abs(Ac).max()   # Galerkin
    B = np.linalg.pinv(Ac.toarray(), rcond=1e-13)
    fwd, adj = lr.coarse_correction(A, P, 0.5 * (B + B.T))     # symmetric as the cycle's coarse operator is
    rng = np.random.default_rng(2)
    X, Y = rng.normal(size=(A.shape[0], 3)), rng.normal(size=(A.shape[0], 3))
    C1 = fwd(X)
    assert np.abs(fwd(C1) - C1).max() <= 1e-8 * np.abs(C1).max()
    assert np.abs(P.T @ (A @ C1)).max() <= 1e-10 * np.abs(P.T @ (A @ X)).max()
    assert np.sum(fwd(X) * Y) == pytest.approx(np.sum(X * adj(Y)), rel=1e-10)


@pytest.mark.parametrize("sor", [False, True])
def test_two_grid_gradient_matches_central_differences(sphere_cc, sor):
    o, t, nu = sphere_cc, 1e-2, 2
    M, L = o.matrices(4)
    A = (M + t * L).tocsr()
    Mc, Lc = o.matrices(3)
    cc = lr.coarse_correction(A, o.prolongation(4), lr.coarse_inverse((Mc + t * Lc).tocsr(), 1e-6))
    keys = o.functions(4)[0]
    f, act, c1 = lr.features(A, M, keys, 4, 4)
    col = lr.colours(keys) if sor else None
    rng = np.random.default_rng(13)
    p = rng.normal(size=lr.NP) * 0.3
    p[lr.O_B3] = 0.2
    E0 = rng.normal(size=(A.shape[0], 2))
    L0, g = lr.loss_grad(A, f, act, c1, p, E0, nu, colour=col, cc=cc)
    assert L0 == pytest.approx(lr.loss(A, f, act, c1, p, E0, nu, colour=col, cc=cc), rel=1e-13)
    # the cycle reduces the residual much more than the sweeps alone
    assert L0 < lr.loss(A, f, act, c1, p, E0, nu, colour=col) - 1.0
    idx = list(rng.choice(lr.O_B1, 4, replace=False)) + list(lr.O_W2 + rng.choice(lr.NH * lr.NH, 4, replace=False)) + \
        list(lr.O_W3 + rng.choice(lr.NH, 3, replace=False)) + [lr.O_B3]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (lr.loss(A, f, act, c1, pp, E0, nu, colour=col, cc=cc) -
              lr.loss(A, f, act, c1, pm, E0, nu, colour=col, cc=cc)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9 * max(1.0, abs(g).max())), i
