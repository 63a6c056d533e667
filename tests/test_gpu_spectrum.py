"""The spectrum L x = lambda M x on the GPU (Section 5.1), through the C ABI.

`camfe_eigs` (shift-invert subspace iteration with the multigrid solver)
against the oracle's dense generalised eigensolve: eigenvalues within 1e-8
relative (absolute for the zero ones), every returned vector an eigenvector
of the oracle's matrices to the requested tolerance, and the block
M-orthonormal.  Eigenvectors of repeated eigenvalues are not unique, so only
these properties are compared.  Cases: a sphere at both degrees, two nested
spheres split and unsplit, FP64 and mixed inner solves, and the argument
checks.
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
def ctx(cf):
    c = cf.camfe_ctx_create(0)
    yield c
    cf.camfe_ctx_destroy(c)


CASES = {
    "sphere_deg1": dict(mesh=lambda: meshgen.icosphere(3), depth=4, degree=1, split=1),
    "sphere_deg2": dict(mesh=lambda: meshgen.icosphere(3), depth=3, degree=2, split=1),
    "nested_split": dict(mesh=lambda: meshgen.nested_spheres(4, 0.02), depth=4, degree=1, split=1),
    "nested_unsplit": dict(mesh=lambda: meshgen.nested_spheres(4, 0.02), depth=4, degree=1, split=0),
}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_eigs_match_dense_oracle(cf, ctx, name, precision):
    c = CASES[name]
    V, F = c["mesh"]()
    say(f"[gpu] eigs {name} precision={precision}")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=c["depth"], degree=c["degree"], split=c["split"], max_coarse=512)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, c["depth"], degree=c["degree"], split=c["split"], max_coarse=512).check().assemble()
    nev, tol = 12, 1e-9
    ev, X, st = cf.camfe_eigs(s, h, nev, sigma=1.0, block=20, max_iter=300, tol=tol,
                              solve_rtol=1e-11 if precision == 0 else 1e-10, precision=precision, seed=7)
    say(f"[gpu] eigs {name}: {st}")
    assert st["converged"], st
    evo = o.eigenvalues(nev)
    assert np.all(np.abs(ev - evo) <= 1e-8 * np.maximum(1.0, np.abs(evo))), (ev, evo)
    M, L = o.matrices(c["depth"])
    R = L @ X - (M @ X) * ev[None, :]
    rel = np.linalg.norm(R, axis=0) / ((np.abs(ev) + 1.0) * np.linalg.norm(M @ X, axis=0))
    assert np.all(rel <= 10 * tol), rel
    G = X.T @ (M @ X)
    assert np.abs(G - np.eye(nev)).max() <= 1e-10
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_eigs_block_and_argument_checks(cf, ctx):
    V, F = meshgen.icosphere(2)
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=3, max_coarse=64)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 3, max_coarse=64).check().assemble()
    # the default block (nev + 8) and a block equal to nev give the same values
    ev1, _, s1 = cf.camfe_eigs(s, h, 4, sigma=2.0, tol=1e-10, solve_rtol=1e-12, vectors=False)
    ev2, _, s2 = cf.camfe_eigs(s, h, 4, sigma=2.0, block=4, max_iter=1000, tol=1e-10, solve_rtol=1e-12,
                               vectors=False)
    assert s1["converged"] and s2["converged"]
    evo = o.eigenvalues(4)
    assert np.all(np.abs(ev1 - evo) <= 1e-8 * np.maximum(1.0, evo))
    assert np.all(np.abs(ev2 - evo) <= 1e-8 * np.maximum(1.0, evo))
    assert s1["iterations"] < s2["iterations"]       # guard vectors speed the wanted pairs up
    for bad in (dict(nev=0), dict(nev=5, block=4), dict(nev=4, block=40), dict(nev=4, sigma=0.0),
                dict(nev=4, sigma=-1.0)):
        kw = dict(nev=4, sigma=1.0)
        kw.update(bad)
        with pytest.raises(cf.CamfeError):
            cf.camfe_eigs(s, h, kw.pop("nev"), **kw)
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_eigs_odd_block_and_solve_afterwards(cf, ctx):
    """An odd block (the round-robin Jacobi then idles one slot per round),
    and a solve with another t after the eigensolver set the solver up for
    t = 1/sigma."""
    V, F = meshgen.icosphere(3)
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=4, max_coarse=512)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 4, max_coarse=512).check().assemble()
    ev, X, st = cf.camfe_eigs(s, h, 5, sigma=0.5, block=9, tol=1e-9, solve_rtol=1e-11)
    assert st["converged"], st
    evo = o.eigenvalues(5)
    assert np.all(np.abs(ev - evo) <= 1e-8 * np.maximum(1.0, evo)), (ev, evo)
    M, L = o.matrices(4)
    assert np.abs(X.T @ (M @ X) - np.eye(5)).max() <= 1e-10
    b = o.load_vector(V[:, 2])
    x, sst = cf.camfe_solve(s, b, t=1e-3, rtol=1e-10, max_iter=400)
    r = np.linalg.norm(b - (M + 1e-3 * L) @ x) / np.linalg.norm(b)
    assert sst["converged"] and r <= 1e-9
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_nested_spheres_spectrum_at_depth_6_against_the_closed_form(cf, ctx):
    """Level-6 nested spheres at depth 6 (about 60k functions, beyond the
    dense oracle): the split spectrum is within 1e-3 of l(l+1) and
    l(l+1)/1.02^2 with two zero eigenvalues; the unsplit one has one."""
    gap = 0.02
    exact = []
    for l in range(6):
        exact += [l * (l + 1.0)] * (2 * l + 1) + [l * (l + 1.0) / (1 + gap) ** 2] * (2 * l + 1)
    exact = np.sort(exact)[:16]
    V, F = meshgen.nested_spheres(6, gap)
    zeros = {}
    for split in (1, 0):
        h = cf.camfe_hierarchy_build(ctx, V, F, depth=6, split=split, max_coarse=4096)
        s = cf.camfe_assemble(h)
        ev, _, st = cf.camfe_eigs(s, h, 16, sigma=1.0, tol=1e-9, solve_rtol=1e-10, precision=1, vectors=False)
        assert st["converged"], st
        zeros[split] = int((np.abs(ev) < 1e-6).sum())
        if split:
            nz = exact > 0
            assert np.all(np.abs(ev[nz] - exact[nz]) / exact[nz] < 1e-3), (ev, exact)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    assert zeros == {1: 2, 0: 1}
