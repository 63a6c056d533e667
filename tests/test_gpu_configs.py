"""The small configuration at its stated size, against the oracle: the unit
icosphere subdivided three times (642 vertices, 1280 triangles), octree depth
5, degree-2 B-splines, connectivity-aware split, FP64, one right-hand side
b_i = int f b_i with f = z + N(0, 0.01^2) noise (seed 1), and the screened
Poisson system (M + 1e-3 L) x = b solved to 1e-10.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_1505_03615_amd import meshgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cf():
    import torch
    from paper_1505_03615_amd import camfe
    assert torch.cuda.is_available()
    return camfe


@pytest.fixture(scope="module")
def config1(cf):
    ctx = cf.camfe_ctx_create(0)
    V, F, f = meshgen.config_mesh("icosphere_l3")
    say("[gpu] config 1: icosphere L3, depth 5, degree 2")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=5, degree=2, split=1, max_coarse=2048)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 5, degree=2, split=1, max_coarse=2048).check().assemble()
    yield V, F, f, h, s, o
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)
    cf.camfe_ctx_destroy(ctx)


def test_config1_structure_and_matrices(cf, config1):
    V, F, f, h, s, o = config1
    fin, d0 = cf.camfe_hierarchy_levels(h)
    assert (fin, d0) == (5, o.coarsest)
    assert cf.camfe_hierarchy_info(h, 5)[2] == o.count(5, "functions") == 11448
    for d in range(5, -1, -1):
        assert np.array_equal(cf.camfe_export_cells(h, d), o.cells(d)), d
        k, t = cf.camfe_export_pairs(h, d)
        ko, to = o.pairs(d)
        assert np.array_equal(k, ko) and np.array_equal(t, to), d
        if d < d0:
            continue
        for a, b in zip(cf.camfe_export_functions(h, d), o.functions(d)):
            assert np.array_equal(a, b), d
        for a, b in zip(cf.camfe_export_support_entries(h, d), o.support_entries(d)):
            assert np.array_equal(a, b), d
        if d > d0:
            P, Po = cf.camfe_export_prolongation(h, d), o.prolongation(d)
            assert np.array_equal(P.indptr, Po.indptr) and np.array_equal(P.indices, Po.indices)
            assert np.array_equal(P.data, Po.data), d
        Mo, Lo = o.matrices(d)
        M, L = cf.camfe_export_matrix(s, h, d, 0), cf.camfe_export_matrix(s, h, d, 1)
        assert abs(M - Mo).max() <= 1e-12 * abs(Mo).max(), d
        assert abs(L - Lo).max() <= 1e-12 * abs(Lo).max(), d
    b = cf.camfe_load_vector(s, h, f)
    bo = o.load_vector(f)
    assert abs(b - bo).max() <= 1e-12 * abs(bo).max()


def test_config1_solve_to_1e10(cf, config1):
    """CG preconditioned by the FP64 V-cycle to 1e-10; the solution's residual
    in the oracle's matrices, and its values at the mesh vertices against the
    oracle's own solve (function-space agreement: coefficient vectors may
    differ along the near-null directions of the restricted quadratic space,
    which vanish on the surface)."""
    V, F, f, h, s, o = config1
    bo = o.load_vector(f)
    Mo, Lo = o.matrices(5)
    A = Mo + 1e-3 * Lo
    x, st = cf.camfe_solve(s, bo, t=1e-3, rtol=1e-10, max_iter=3000)
    r = np.linalg.norm(bo[:, 0] - A @ x[:, 0]) / np.linalg.norm(bo)
    say(f"[gpu] config 1: {st['cycles']} cycles, GPU residual {st['rel_residual']:.3e}, in the oracle's matrices {r:.3e}")
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert r <= 1e-9
    xo, io = o.solve(1e-3, bo, rtol=1e-10, max_iter=3000)
    assert io["converged"]
    uv, uo = cf.camfe_eval_vertices(s, len(V), x), o.eval_vertices(xo)
    ev = abs(uv - uo).max() / abs(uo).max()
    say(f"[gpu] config 1: oracle {io['cycles']} cycles; vertex values differ by {ev:.3e}")
    assert ev <= 1e-6
