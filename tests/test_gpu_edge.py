"""Edge cases of the HIP path against the oracle: a single triangle (degrees 1
and 2), many disconnected components, a hierarchy of one depth, invalid
inputs, and right-hand-side counts that do not fill the kernels' column
groups.  Calls go through the C ABI (the ctypes binding)."""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1505_03615_amd import meshgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    Vt, Ft = meshgen.single_triangle()
    Vc, Fc = meshgen.unit_cubes(n=3)
    V1, F1 = meshgen.icosphere(1)
    return {
        "triangle_deg1": dict(V=Vt, F=Ft, depth=4, degree=1, max_coarse=0),
        "triangle_deg2": dict(V=Vt, F=Ft, depth=3, degree=2, max_coarse=0),
        "cubes": dict(V=Vc, F=Fc, depth=6, degree=1, max_coarse=256),
        "one_depth": dict(V=V1, F=F1, depth=1, degree=1, max_coarse=4096),
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
        say(f"[gpu] edge: build {name} nt={len(c['F'])} depth={c['depth']} degree={c['degree']}")
        h = cf.camfe_hierarchy_build(ctx, c["V"], c["F"], depth=c["depth"], degree=c["degree"],
                                     max_coarse=c["max_coarse"])
        s = cf.camfe_assemble(h)
        o = Oracle(c["V"], c["F"], c["depth"], degree=c["degree"], max_coarse=c["max_coarse"]).check().assemble()
        _built[name] = (h, s, o)
    return _built[name]


@pytest.mark.parametrize("name", list(CASES))
def test_edge_hierarchy_and_matrices(cf, ctx, name):
    h, s, o = built(cf, ctx, name)
    D = CASES[name]["depth"]
    fin, d0 = cf.camfe_hierarchy_levels(h)
    assert (fin, d0) == (D, o.coarsest)
    for d in range(D, d0 - 1, -1):
        k, t = cf.camfe_export_pairs(h, d)
        ko, to = o.pairs(d)
        assert np.array_equal(k, ko) and np.array_equal(t, to), d
        for a, b in zip(cf.camfe_export_functions(h, d), o.functions(d)):
            assert np.array_equal(a, b), d
        if d > d0:
            P, Po = cf.camfe_export_prolongation(h, d), o.prolongation(d)
            assert np.array_equal(P.indices, Po.indices) and np.array_equal(P.data, Po.data), d
        Mo, Lo = o.matrices(d)
        M = cf.camfe_export_matrix(s, h, d, 0)
        L = cf.camfe_export_matrix(s, h, d, 1)
        assert abs(M - Mo).max() <= 1e-12 * abs(Mo).max(), d
        assert abs(L - Lo).max() <= 1e-12 * abs(Lo).max(), d


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_edge_solve(cf, ctx, name, precision):
    h, s, o = built(cf, ctx, name)
    c = CASES[name]
    rng = np.random.default_rng(5)
    f = rng.standard_normal(len(c["V"]))
    b = o.load_vector(f)
    t = 1e-3
    say(f"[gpu] edge: solve {name} precision={precision}")
    x, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=1500, precision=precision)
    Mo, Lo = o.matrices(c["depth"])
    A = Mo + t * Lo
    r = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
    assert st["converged"], st
    assert np.all(r <= 1e-6), r


@pytest.mark.parametrize("k", [2, 5, 9])
def test_right_hand_side_counts(cf, ctx, k):
    """k columns in one call (column groups of up to four in the kernels)
    and each column solved on its own both reach the tolerance.  The cubes'
    planar faces make M + t L nearly singular, so two converged solutions may
    differ along its near-null space: residuals are compared, not solutions."""
    h, s, o = built(cf, ctx, "cubes")
    c = CASES["cubes"]
    rng = np.random.default_rng(100 + k)
    F = rng.standard_normal((len(c["V"]), k))
    B = o.load_vector(F)
    say(f"[gpu] edge: {k} columns")
    X, st = cf.camfe_solve(s, B, t=1e-3, rtol=1e-9, max_iter=1500)
    assert st["converged"], st
    Mo, Lo = o.matrices(c["depth"])
    A = Mo + 1e-3 * Lo
    for j in range(k):
        xj, stj = cf.camfe_solve(s, B[:, j:j + 1], t=1e-3, rtol=1e-9, max_iter=1500)
        assert stj["converged"]
        rj = np.linalg.norm(B[:, j] - A @ X[:, j]) / np.linalg.norm(B[:, j])
        rs = np.linalg.norm(B[:, j] - A @ xj[:, 0]) / np.linalg.norm(B[:, j])
        assert rj <= 1e-8 and rs <= 1e-8, (j, rj, rs)


def test_invalid_meshes_are_rejected(cf, ctx):
    V, F = meshgen.icosphere(1)
    bad = {
        "empty mesh": (V, np.zeros((0, 3), np.int32), 3, 1),
        "repeated index": (V, np.array([[0, 0, 1]], np.int32), 3, 1),
        "index out of range": (V, np.array([[0, 1, len(V)]], np.int32), 3, 1),
        # exactly zero normal (binary-exact collinear points; coincident points)
        "collinear": (np.array([[0.0, 0.0, 0.0], [0.25, 0.5, 0.75], [0.5, 1.0, 1.5]]),
                      np.array([[0, 1, 2]], np.int32), 3, 1),
        "coincident": (np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [0.5, 0.7, 0.2]]),
                       np.array([[0, 1, 2]], np.int32), 3, 1),
        "nan vertex": (np.where(np.arange(V.size).reshape(V.shape) == 4, np.nan, V), F, 3, 1),
        "depth 0": (V, F, 0, 1),
        "depth 13": (V, F, 13, 1),
        "degree 3": (V, F, 3, 3),
    }
    for what, (Vb, Fb, depth, degree) in bad.items():
        say(f"[gpu] edge: reject {what}")
        with pytest.raises(cf.CamfeError, match="EINVAL"):
            cf.camfe_hierarchy_build(ctx, Vb, Fb, depth=depth, degree=degree)
