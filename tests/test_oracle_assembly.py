"""Pins of the oracle's assembled matrices (Section 3.1 Eq. 2, Section 5.1).

Closed forms (partition of unity, monomial integrals over a triangle, linear
fields), invariants (symmetry, zero row sums of L, Galerkin identity of the
nested spaces, Section 4.1 Claim), the planar linear dependency of the
the Discussion closing Section 5, the split's block structure and the sphere spectrum.
"""
import math

import numpy as np
import pytest
import scipy.linalg as la

from oracle import Oracle
from paper_1505_03615_amd import meshgen


def tri_areas_normals(V, F):
    c = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    a = 0.5 * np.linalg.norm(c, axis=1)
    return a, c / np.linalg.norm(c, axis=1, keepdims=True)


@pytest.fixture(scope="module")
def sphere1():
    V, F = meshgen.icosphere(3)
    return V, F, Oracle(V, F, 5, degree=1, max_coarse=0, min_depth=2).check().assemble()


@pytest.fixture(scope="module")
def sphere2():
    V, F = meshgen.icosphere(2)
    return V, F, Oracle(V, F, 4, degree=2, max_coarse=0, min_depth=1).check().assemble()


@pytest.mark.parametrize("fx", ["sphere1", "sphere2"])
def test_partition_of_unity_symmetry_zero_rowsum(fx, request):
    V, F, o = request.getfixturevalue(fx)
    area = tri_areas_normals(V, F)[0].sum()
    for d in range(o.coarsest, o.depth + 1):
        M, L = o.matrices(d)
        assert abs(M.sum() - area) <= 1e-13 * area
        assert abs(M - M.T).max() <= 1e-14 * abs(M).max()
        assert abs(L - L.T).max() <= 1e-14 * abs(L).max()
        assert np.all(M @ np.ones(M.shape[0]) > 0)
        assert abs(L @ np.ones(L.shape[0])).max() <= 1e-12 * abs(L).max()
        # structure: degree 1 rows couple corners at most one apart per axis
        assert M.nnz == L.nnz


def _poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0.0) + ca * cb
    return out


def _lin(c):  # linear form sum_m c[m] lambda_m
    return {(1, 0, 0): c[0], (0, 1, 0): c[1], (0, 0, 1): c[2]}


def _integrate(p, area2):
    # int_T l1^a l2^b l3^c = 2A a! b! c! / (a+b+c+2)!  (area2 = 2A)
    return sum(c * area2 * math.factorial(a) * math.factorial(b) * math.factorial(g)
               / math.factorial(a + b + g + 2) for (a, b, g), c in p.items())


def _basis_poly(degree, j, comp_coeffs):
    """1D basis piece j on the unit cell as a polynomial in barycentrics, where
    the local coordinate is sum_m comp_coeffs[m] lambda_m."""
    l = _lin(comp_coeffs)
    one_minus = {e: -c for e, c in l.items()}
    for e in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):   # 1 = l1 + l2 + l3
        one_minus[e] = one_minus.get(e, 0.0) + 1.0
    if degree == 1:
        return l if j == 1 else one_minus
    if j == 0:
        return {e: 0.5 * c for e, c in _poly_mul(one_minus, one_minus).items()}
    if j == 2:
        return {e: 0.5 * c for e, c in _poly_mul(l, l).items()}
    # 3/4 - (l - 1/2)^2 = l (1 - l) + 1/2 with 1/2 = (l1+l2+l3)^2 / 2
    s = _lin((1.0, 1.0, 1.0))
    base = _poly_mul(l, one_minus)
    for e, c in _poly_mul(s, s).items():
        base[e] = base.get(e, 0.0) + 0.5 * c
    return base


def _dbasis_poly(degree, j, comp_coeffs):
    l = _lin(comp_coeffs)
    s = _lin((1.0, 1.0, 1.0))
    if degree == 1:
        return {e: (1.0 if j == 1 else -1.0) * c for e, c in s.items()}
    if j == 0:   # -(1 - l)
        return {e: -(s.get(e, 0) - l.get(e, 0)) for e in s}
    if j == 2:
        return l
    return {e: -2.0 * (l.get(e, 0) - 0.5 * s.get(e, 0)) for e in s}   # -2 (l - 1/2)


def _homog(p, deg):
    """Lift every monomial to total degree `deg` by multiplying with (l1+l2+l3)."""
    out = {}
    s = _lin((1.0, 1.0, 1.0))
    for e, c in p.items():
        q = {e: c}
        for _ in range(deg - sum(e)):
            q = _poly_mul(q, s)
        for ee, cc in q.items():
            out[ee] = out.get(ee, 0.0) + cc
    return out


@pytest.mark.parametrize("degree", [1, 2])
def test_single_triangle_matches_monomial_formula(degree):
    """One triangle inside one cell (grid units = world units): each entry of
    M and L equals the textbook integral of the product polynomial over the
    triangle, int l1^a l2^b l3^c = 2A a! b! c! / (a+b+c+2)!."""
    V, F = meshgen.single_triangle()
    o = Oracle(V, F, 1, degree=degree, box=[0, 0, 0, 2.0], max_coarse=0).check().assemble()
    M, L = o.matrices(1)
    fk, fc, fr = o.functions(1)
    W = 2 if degree == 1 else 3
    area, nrm = tri_areas_normals(V, F)
    n = nrm[0]
    # function key -> local index (jx, jy, jz): support coordinates minus the cell (0,0,0)
    def dec(k):
        c = [0, 0, 0]
        for b in range(21):
            for a in range(3):
                c[a] |= ((int(k) >> (3 * b + a)) & 1) << b
        return c
    loc = [dec(k) for k in fk]
    assert len(fk) == W ** 3
    vals, grads = [], []
    for j in loc:
        comps = [V[:, a] for a in range(3)]   # local coordinate at each vertex
        ph = [_basis_poly(degree, j[a], comps[a]) for a in range(3)]
        dph = [_dbasis_poly(degree, j[a], comps[a]) for a in range(3)]
        vals.append(_poly_mul(_poly_mul(ph[0], ph[1]), ph[2]))
        g = [_poly_mul(_poly_mul(dph[0], ph[1]), ph[2]), _poly_mul(_poly_mul(ph[0], dph[1]), ph[2]),
             _poly_mul(_poly_mul(ph[0], ph[1]), dph[2])]
        G = 2 * degree
        g = [_homog(q, G) for q in g]
        gn = {}
        for a in range(3):
            for e, c in g[a].items():
                gn[e] = gn.get(e, 0.0) + n[a] * c
        grads.append([{e: g[a].get(e, 0.0) - n[a] * gn.get(e, 0.0) for e in set(g[a]) | set(gn)}
                      for a in range(3)])
    Md, Ld = M.toarray(), L.toarray()
    for i in range(len(fk)):
        for j in range(len(fk)):
            m_ref = _integrate(_poly_mul(vals[i], vals[j]), 2 * area[0])
            l_ref = sum(_integrate(_poly_mul(grads[i][a], grads[j][a]), 2 * area[0]) for a in range(3))
            assert abs(Md[i, j] - m_ref) <= 1e-15 + 1e-12 * abs(m_ref)
            assert abs(Ld[i, j] - l_ref) <= 1e-14 + 1e-12 * abs(l_ref)


@pytest.mark.parametrize("fx", ["sphere1", "sphere2"])
def test_linear_field_closed_forms(fx, request):
    V, F, o = request.getfixturevalue(fx)
    M, L = o.matrices(o.depth)
    X0 = o.linear_coeffs()
    area, nrm = tri_areas_normals(V, F)
    rng = np.random.default_rng(5)
    for _ in range(3):
        a = rng.normal(size=3)
        x = X0 @ a
        g = V @ a
        gv = g[F]
        m_ref = (area / 6 * ((gv ** 2).sum(1) + gv[:, 0] * gv[:, 1] + gv[:, 1] * gv[:, 2]
                             + gv[:, 2] * gv[:, 0])).sum()
        l_ref = (area * (a @ a - (nrm @ a) ** 2)).sum()
        assert abs(x @ (M @ x) - m_ref) <= 1e-12 * abs(m_ref)
        assert abs(x @ (L @ x) - l_ref) <= 1e-12 * abs(l_ref)
    # the embedding is reproduced at the vertices
    assert np.allclose(o.eval_vertices(X0), V, rtol=0, atol=1e-12)


def sheet_fields_coeffs(X0, rep, nt_top, fields):
    """Coefficients a_s . node_i, s the sheet (0: triangles below nt_top) of
    each function's representative triangle."""
    s = (rep >= nt_top).astype(int)
    return np.einsum("ij,ij->i", X0, fields[s])


@pytest.mark.parametrize("degree", [1, 2])
def test_split_vertex_values_pick_the_vertex_component(degree):
    """Evaluation u(v) = sum_k x_(k, label_k(t_v)) b_k(v) (Section 4.2: a split
    function is one function per connected component) on two sheets closer
    than a cell, in split mode.  Every function gets the coefficient
    a_s . node, with a different linear field a_s for the sheet s of its
    representative triangle.  Linear reproduction of the B-splines then gives
    a_s . V_v at every vertex v of sheet s, exactly when each vertex reads the
    component of its own sheet.  Components of one support are numbered by
    smallest triangle and the top sheet's triangles come first, so a vertex
    of the bottom sheet that read component 0 (or any fixed component) would
    get the top sheet's field."""
    V, F, _, sheet = meshgen.two_sheets(16, 1.0 / 64)
    depth = 5 if degree == 1 else 4
    o = Oracle(V, F, depth, degree=degree, max_coarse=0, min_depth=depth - 1).check()
    keys, comp, rep = o.functions(depth)
    assert comp.max() >= 1 and (comp > 0).sum() > len(comp) // 4      # most supports split
    nt_top = len(F) // 2
    fields = np.array([[0.7, -1.3, 0.4], [-0.9, 0.5, 1.6]])
    x = sheet_fields_coeffs(o.linear_coeffs(), rep, nt_top, fields)
    want = np.einsum("ij,ij->i", V, fields[sheet])
    got = o.eval_vertices(x)[:, 0]
    assert np.abs(got - want).max() <= 1e-13
    # the two fields differ by O(1) at every vertex: a wrong pick cannot hide
    assert np.abs(V @ (fields[0] - fields[1])).min() > 1e-3


@pytest.mark.parametrize("fx", ["sphere1", "sphere2"])
def test_galerkin_identity_of_nested_spaces(fx, request):
    """Claim of Section 4.1: coarse functions are combinations of fine ones with
    the Eq. (4) coefficients, so M_{d-1} = P^T M_d P and L_{d-1} = P^T L_d P."""
    V, F, o = request.getfixturevalue(fx)
    for d in range(o.coarsest + 1, o.depth + 1):
        P = o.prolongation(d)
        Mf, Lf = o.matrices(d)
        Mc, Lc = o.matrices(d - 1)
        assert abs(P.T @ Mf @ P - Mc).max() <= 1e-12 * abs(Mc).max()
        assert abs(P.T @ Lf @ P - Lc).max() <= 1e-12 * abs(Lc).max()


def test_load_vector_constant_and_linear():
    V, F = meshgen.icosphere(2)
    o = Oracle(V, F, 4, max_coarse=0, min_depth=3).check().assemble()
    M, L = o.matrices(4)
    b = o.load_vector(np.stack([np.ones(len(V)), V[:, 0]], 1))
    assert np.allclose(b[:, 0], M @ np.ones(M.shape[0]), rtol=1e-12, atol=1e-16)
    assert np.allclose(b[:, 1], M @ o.linear_coeffs()[:, 0], rtol=1e-11, atol=1e-15)


def test_planar_sheet_linear_dependency():
    """Discussion closing Section 5: a planar component gives a singular system.  The
    corner samples of the linear function vanishing on the plane are an exact
    null vector of M and L (any orientation; axis-aligned planes give more)."""
    V, F, _, _ = meshgen.two_sheets(12, gap=0.2, rotate=True)
    V, F = V[: 13 * 13], F[: len(F) // 2]
    o = Oracle(V, F, 4, max_coarse=0).check().assemble()
    M, L = o.matrices(4)
    nrm = tri_areas_normals(V, F)[1][0]
    z = o.linear_coeffs() @ nrm - V[0] @ nrm
    assert abs(M @ z).max() <= 1e-13 * abs(M).max() * abs(z).max()
    assert abs(L @ z).max() <= 1e-12 * abs(L).max() * abs(z).max()
    # a curved surface has no such vector
    Vs, Fs = meshgen.icosphere(2)
    os_ = Oracle(Vs, Fs, 4, max_coarse=0).check().assemble()
    Ms, _ = os_.matrices(4)
    ev = la.eigvalsh(Ms.toarray() / np.sqrt(np.outer(Ms.diagonal(), Ms.diagonal())))
    assert ev[0] > 1e-8


def test_split_blocks_equal_single_sheets():
    """Two parallel sheets closer than a voxel: in split mode no function spans
    both, the matrices are block diagonal, and each block equals its sheet
    assembled alone in the same cube (Section 4.2; teaser coupling)."""
    n = 32
    V, F, xl, sheet = meshgen.two_sheets(n, gap=1.0 / n, rotate=True)
    o = Oracle(V, F, 5, max_coarse=0, min_depth=3).check().assemble()
    cube = o.cube()
    tri_sheet = sheet[F[:, 0]]
    nv1, nt1 = (n + 1) ** 2, len(F) // 2
    single = Oracle(V[:nv1], F[:nt1], 5, max_coarse=0, min_depth=3, box=cube).check().assemble()
    for d in range(3, 6):
        M, L = o.matrices(d)
        fk, fc, fr = o.functions(d)
        fs = tri_sheet[fr]
        Mc = M.tocoo()
        assert np.all(fs[Mc.row] == fs[Mc.col]), d
        top = np.where(fs == 0)[0]
        M1, L1 = single.matrices(d)
        assert np.array_equal(single.functions(d)[0], fk[top])
        assert abs(M[top][:, top] - M1).max() <= 1e-15 * abs(M1).max()
        assert abs(L[top][:, top] - L1).max() <= 1e-13 * abs(L1).max()
    # unsplit: functions span both sheets
    ou = Oracle(V, F, 5, split=0, max_coarse=0, min_depth=5).check().assemble()
    Mu, _ = ou.matrices(5)
    fku, _, _ = ou.functions(5)
    assert Mu.shape[0] < o.matrices(5)[0].shape[0]


def test_sphere_spectrum_approaches_l_l_plus_1():
    """Section 5.1: the generalised eigenvalues L x = lambda M x on the unit
    sphere approach l(l+1) = 0, 2, 6, 12 with multiplicities 1, 3, 5, 7."""
    V, F = meshgen.icosphere(4)
    o = Oracle(V, F, 4, max_coarse=0, min_depth=4).check().assemble()
    M, L = o.matrices(4)
    s = 1 / np.sqrt(M.diagonal())
    Ms = (M.toarray() * np.outer(s, s))
    Ls = (L.toarray() * np.outer(s, s))
    ev = la.eigh(Ls, Ms, eigvals_only=True, subset_by_index=[0, 15])
    ref = np.array([0] + [2] * 3 + [6] * 5 + [12] * 7, dtype=float)
    assert abs(ev[0]) < 1e-8
    assert np.all(np.abs(ev[1:] - ref[1:]) / ref[1:] < 0.03), ev
    # rotation stability of the spectrum
    R = meshgen.rodrigues((0.3, -1.0, 0.4), 0.7)
    o2 = Oracle(V @ R.T, F, 4, max_coarse=0, min_depth=4).check().assemble()
    M2, L2 = o2.matrices(4)
    s2 = 1 / np.sqrt(M2.diagonal())
    ev2 = la.eigh(L2.toarray() * np.outer(s2, s2), M2.toarray() * np.outer(s2, s2),
                  eigvals_only=True, subset_by_index=[0, 15])
    assert np.all(np.abs(ev2[1:] - ev[1:]) / ev[1:] < 0.02)
