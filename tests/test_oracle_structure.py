"""Pins of the oracle's discrete structure: pairs, octree, supports, split, chi.

Checked against the exact-rational brute force (different algorithms: clipped
area and parametric clipping instead of separating axes), hand cases and the
Observation of Section 4.1.
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle
from paper_1505_03615_amd import meshgen
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _in_grid_plane(V, F):
    for f in F:
        p = V[f]
        for a in range(3):
            if p[0, a] == p[1, a] == p[2, a] and float(p[0, a]).is_integer():
                return True
        if np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0])) == 0:
            return True
    return False


def dyadic_sheet(seed, n=4, D=2, denom=8):
    """A small bumpy sheet with dyadic coordinates inside [0, 2^D]^3, so every
    float operation of the predicates is exact (products of few-bit numbers)."""
    rng = np.random.default_rng(seed)
    N = 1 << D
    while True:
        xs = np.sort(rng.choice(np.arange(2, N * denom - 1), n, replace=False)) / denom
        ys = np.sort(rng.choice(np.arange(2, N * denom - 1), n, replace=False)) / denom
        Z = rng.integers(2, N * denom - 1, size=(n, n)) / denom
        V = np.array([[xs[i], ys[j], Z[i, j]] for i in range(n) for j in range(n)])
        F = []
        for i in range(n - 1):
            for j in range(n - 1):
                a, b, c, d = i * n + j, (i + 1) * n + j, (i + 1) * n + j + 1, i * n + j + 1
                F += [(a, b, c), (a, c, d)]
        F = np.array(F, np.int32)
        if not _in_grid_plane(V, F):
            return V, F


def dyadic_soup(seed, nt=6, D=2, denom=8):
    rng = np.random.default_rng(seed)
    N = 1 << D
    while True:
        V = rng.integers(1, N * denom, size=(3 * nt, 3)) / denom
        F = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
        if not _in_grid_plane(V, F):
            return V, F


def oracle_for(V, F, D, **kw):
    N = float(1 << D)
    return Oracle(V, F, D, box=[0.0, 0.0, 0.0, N], min_depth=0, max_coarse=0, **kw).check()


@pytest.mark.parametrize("seed", range(12))
def test_pairs_match_exact_clip(seed):
    V, F = dyadic_soup(seed) if seed % 2 else dyadic_sheet(seed)
    D = 2
    o = oracle_for(V, F, D)
    for d in range(D, -1, -1):
        Vd = V * (2.0 ** (d - D))
        exact = bf.pairs_exact([tuple(p) for p in Vd], F.tolist(), d)
        k, t = o.pairs(d)
        got = set(zip(k.tolist(), t.tolist()))
        assert got == exact, f"depth {d}"
        # pairs are sorted by (cell key, triangle)
        assert np.all(np.diff(k.astype(np.float64)) >= 0)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("degree", [1, 2])
def test_components_match_exact(seed, degree):
    V, F = dyadic_sheet(100 + seed, n=5)
    D = 2
    o = oracle_for(V, F, D, degree=degree)
    for d in range(D, -1, -1):
        Vd = [tuple(p) for p in V * (2.0 ** (d - D))]
        exact = bf.components_exact(Vd, F.tolist(), d, degree)
        key, tri, func = o.support_entries(d)
        fk, fc, fr = o.functions(d)
        got = {}
        for kk, tt, ff in zip(key.tolist(), tri.tolist(), func.tolist()):
            got.setdefault(kk, {}).setdefault(ff, []).append(tt)
        got = {kk: sorted(sorted(g) for g in v.values()) for kk, v in got.items()}
        assert got == exact, f"depth {d}"
        # functions in canonical order, components numbered by min triangle, rep = min
        assert np.all(np.diff(fk.astype(np.float64)) >= 0)
        for kk, groups in exact.items():
            idx = np.where(fk == kk)[0]
            assert list(fc[idx]) == list(range(len(groups)))
            assert list(fr[idx]) == [g[0] for g in groups]


def test_unsplit_has_one_function_per_support():
    V, F = dyadic_sheet(7, n=5)
    o = oracle_for(V, F, 2, split=0)
    for d in range(3):
        fk, fc, fr = o.functions(d)
        assert len(np.unique(fk)) == len(fk) and np.all(fc == 0)


def test_single_sheet_never_splits():
    V, F, _, _ = meshgen.two_sheets(16, gap=0.3, rotate=True)
    V = V[: 17 * 17]
    F = F[: len(F) // 2]
    o = Oracle(V, F, 5, max_coarse=0).check()
    for d in range(0, 6):
        fk, fc, fr = o.functions(d)
        assert np.all(fc == 0), d


def test_two_sheets_split_exactly_where_both_meet():
    """Two parallel sheets about 0.73 voxel apart at the finest depth: a support
    gets two functions iff its active triangles come from both sheets."""
    n = 32
    V, F, xl, sheet = meshgen.two_sheets(n, gap=1.0 / n, rotate=True)
    tri_sheet = sheet[F[:, 0]]
    o = Oracle(V, F, 5, max_coarse=0).check()
    for d in range(5, 1, -1):
        key, tri, func = o.support_entries(d)
        fk, fc, fr = o.functions(d)
        ncomp = {}
        sheets = {}
        for kk, tt, ff in zip(key.tolist(), tri.tolist(), func.tolist()):
            ncomp.setdefault(kk, set()).add(ff)
            sheets.setdefault(kk, set()).add(int(tri_sheet[tt]))
        for kk in ncomp:
            assert len(ncomp[kk]) == len(sheets[kk]), (d, kk)
        n_split = sum(len(v) == 2 for v in ncomp.values())
        assert n_split > 0


def test_observation_fine_component_inside_one_coarse_component():
    """Observation (Section 4.1): every triangle of a fine component carries
    the same coarse label at each parent support, so chi is well defined."""
    V, F = meshgen.torus_knot(nu=256, nv=8, seed=3)
    o = Oracle(V, F, 6, max_coarse=0).check()
    for d in range(6, 1, -1):
        key, tri, func = o.support_entries(d)
        ckey, ctri, cfunc = o.support_entries(d - 1)
        clook = {(k, t): f for k, t, f in zip(ckey.tolist(), ctri.tolist(), cfunc.tolist())}
        P = o.prolongation(d).tocsr()
        fk, fc, fr = o.functions(d)
        members = {}
        for kk, tt, ff in zip(key.tolist(), tri.tolist(), func.tolist()):
            members.setdefault(ff, []).append(tt)
        ckeys_of = {}
        cfk = o.functions(d - 1)[0]
        for f in range(0, len(fk), max(1, len(fk) // 300)):
            cols = P.indices[P.indptr[f]:P.indptr[f + 1]]
            for c in cols:
                K = int(cfk[c])
                labels = {clook[(K, t)] for t in members[f]}
                assert labels == {c}, (d, f)


def test_prolongation_stencils_match_printed():
    """Degree 2 uses the printed 1D stencil 1/4 (1 3 3 1) (Section 3.2, Eq. 3);
    degree 1 the hat refinement 1/2 (1 2 1).  Checked on the single coarse
    function of a tiny sheet and through P 1 = 1."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    printed = np.array(g["prolongation_stencil_1d"]["value"], dtype=float) / g["prolongation_stencil_1d"]["scale"]
    V, F = meshgen.icosphere(2)
    for degree, stencil in ((2, printed), (1, np.array([0.5, 1.0, 0.5]))):
        o = Oracle(V, F, 4, degree=degree, max_coarse=0).check()
        for d in range(4, 1, -1):
            P = o.prolongation(d)
            assert np.allclose(P @ np.ones(P.shape[1]), 1.0, atol=0, rtol=0)
            w = np.unique(np.round(P.data, 15))
            prods = np.unique(np.round(np.outer(np.outer(stencil, stencil), stencil).ravel(), 15))
            assert set(w.tolist()) <= set(prods.tolist())
            # rows have exactly 8 parents in degree 2 and 1/2/4/8 in degree 1
            nnz = np.diff(P.indptr)
            if degree == 2:
                assert np.all(nnz == 8)
            else:
                assert set(np.unique(nnz).tolist()) <= {1, 2, 4, 8}


def test_octree_parents_occupied_and_cells_shrink():
    V, F = meshgen.icosphere(3)
    o = Oracle(V, F, 6, max_coarse=0).check()
    for d in range(6, 0, -1):
        fine = o.cells(d)
        coarse = set(o.cells(d - 1).tolist())
        assert {int(k) >> 3 for k in fine} == coarse


def test_invalid_inputs_rejected():
    V = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5], [0.5, 1.5, 0.5]])
    F = np.array([[0, 1, 2]], np.int32)
    # lies in the grid plane z = 0.5 * (2^2 / 2) = 1 at depth 2 of a box of side 2
    o = Oracle(V, F, 2, box=[0, 0, 0, 2.0])
    assert not o.ok and "grid plane" in o.error
    o = Oracle(V, np.array([[0, 1, 1]], np.int32), 3)
    assert not o.ok
    o = Oracle(V, np.array([[0, 1, 5]], np.int32), 3)
    assert not o.ok
