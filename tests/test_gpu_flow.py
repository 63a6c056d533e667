"""Tracked cMCF steps (Section 5.3) on the GPU against the oracle's steps.

Each step re-weights the mass by area ratios, re-assembles M_t at every depth
and solves (M_t + delta/2 L_0) X' = M_t X from X; after every step the GPU's
M_t must match the oracle's within 1e-12, X' must solve the oracle's system
and the surface it gives must match the oracle's.
Also: a solve after re-assembly uses the new values (the cached solver state
is refreshed, not reused).
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from oracle.flow import flow_step
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
def ctx(cf):
    c = cf.camfe_ctx_create(0)
    yield c
    cf.camfe_ctx_destroy(c)


@pytest.mark.parametrize("name", ["sphere", "knot"])
def test_flow_steps_match_oracle(cf, ctx, name):
    if name == "sphere":
        V, F = meshgen.icosphere(4)
        depth, delta, steps = 6, 0.2, 3
    else:
        V, F = meshgen.torus_knot(nu=1024, nv=16, seed=3)
        depth, delta, steps = 7, 2e-4, 3
    say(f"[gpu] flow {name}: nt={len(F)} depth={depth}")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=depth, degree=1, max_coarse=512)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, depth, degree=1, max_coarse=512).check().assemble()
    X = cf.camfe_linear_coeffs(s, h)
    Xo = o.linear_coeffs()
    assert np.abs(X - Xo).max() <= 1e-13 * np.abs(Xo).max()
    fin, d0 = cf.camfe_hierarchy_levels(h)
    for k in range(steps):
        say(f"[gpu] flow {name}: step {k}")
        Xin = X.copy()                  # both sides step from the same coefficients
        X, st = cf.camfe_flow_step(s, X, delta, rtol=1e-11, max_iter=600)
        assert st["converged"], st
        Xo, info, w = flow_step(o, Xin, delta, rtol=1e-12, max_iter=600)
        for d in range(d0, fin + 1):
            Mo, _ = o.matrices(d)
            M = cf.camfe_export_matrix(s, h, d, 0)
            assert abs(M - Mo).max() <= 1e-12 * abs(Mo).max(), (k, d)
        # coefficients of functions with almost no mass are barely determined, so
        # compare what the step fixes: the residual in the oracle's system and the surface
        Mo, Lo = o.matrices(fin)
        b = Mo @ Xin
        rel = np.linalg.norm(b - (Mo + 0.5 * delta * Lo) @ X, axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(rel <= 1e-9), (k, rel)
        P, Po = cf.camfe_eval_vertices(s, len(V), X), o.eval_vertices(Xo)
        assert np.abs(P - Po).max() <= 1e-8 * np.abs(Po).max(), k
    if name == "sphere":
        r = np.linalg.norm(cf.camfe_eval_vertices(s, len(V), X), axis=1)
        assert np.median(r) < 0.6          # three steps of delta = 0.2 shrink the unit sphere
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_flow_mixed_precision_and_learned_smoother(cf, ctx):
    V, F = meshgen.torus_knot(nu=1024, nv=16, seed=3)
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=7, degree=1, max_coarse=512)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 7, degree=1, max_coarse=512).check().assemble()
    m = cf.camfe_model_create(None, levels=2, bf16=True)
    cf.camfe_smoother_attach(s, m)
    try:
        X = cf.camfe_linear_coeffs(s, h)
        for k in range(2):
            for precision, smoother in ((1, 0), (1, 2)):
                say(f"[gpu] flow knot mixed: step {k} smoother {smoother}")
                Xk, st = cf.camfe_flow_step(s, X.copy(), 2e-4, rtol=1e-8, max_iter=1500, precision=precision,
                                            smoother=smoother)
                assert st["converged"] and not st["fell_back"], st
                flow_step(o, X, 2e-4, rtol=1e-12)       # leaves the oracle's M_t for this input assembled
                Mo, Lo = o.matrices(7)
                A = Mo + 1e-4 * Lo
                b = Mo @ X
                rel = np.linalg.norm(b - A @ Xk, axis=0) / np.linalg.norm(b, axis=0)
                assert np.all(rel <= 1e-6), rel
            X = Xk
    finally:
        cf.camfe_smoother_attach(s, None)
        cf.camfe_model_destroy(m)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)


def test_solve_after_reassembly_uses_new_values(cf, ctx):
    V, F = meshgen.torus_knot(nu=1024, nv=16, seed=3)
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=6, degree=1, max_coarse=256)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 6, degree=1, max_coarse=256).check().assemble()
    b = o.load_vector(V[:, :1])
    x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-10, max_iter=400)   # builds the solver state
    assert st["converged"]
    w = np.random.default_rng(3).uniform(0.3, 3.0, len(F))
    cf.camfe_reassemble_mass(s, w)
    o.assemble(tri_weight=w)
    Mo, Lo = o.matrices(6)
    for precision in (0, 1):
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-10, max_iter=400, precision=precision)
        assert st["converged"], st
        r = np.linalg.norm(b - (Mo + 1e-3 * Lo) @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(r <= 1e-6), r
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)
