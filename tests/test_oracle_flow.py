"""Pins of the tracked cMCF step reference (oracle/flow.py, Section 5.3).

On a round sphere the coordinate functions are eigenfunctions of the
Laplace-Beltrami operator, so the semi-implicit step shrinks the sphere by a
factor that follows from the step's form alone: 1 / (1 + delta lam / 2) for
the first step, where M_t = M_0, and rho^2 / (rho^2 + delta lam / 2) for the
second, where every triangle's area ratio is rho^2 and only the mass matrix
carries it.  lam is the discrete Rayleigh quotient of the coordinates.  Also:
the first step sees area ratios of exactly one (linear functions are
reproduced), and delta = 0 leaves the coefficients unchanged.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.flow import flow_step, triangle_areas
from paper_1505_03615_amd import meshgen


@pytest.fixture(scope="module")
def sphere():
    V, F = meshgen.icosphere(4)
    return Oracle(V, F, 6, degree=1, max_coarse=2048).check().assemble()


def _radius(o, X):
    return np.linalg.norm(o.eval_vertices(X), axis=1)


def test_first_step_weights_are_one_and_zero_step_is_identity(sphere):
    o = sphere
    X0 = o.linear_coeffs()
    assert np.allclose(o.eval_vertices(X0), o.V, rtol=0, atol=1e-13)
    X1, info, w = flow_step(o, X0, 0.0)
    assert np.abs(w - 1.0).max() <= 1e-12
    assert info["converged"]
    assert np.abs(X1 - X0).max() <= 1e-9 * np.abs(X0).max()


def test_sphere_shrinks_as_the_step_form_fixes(sphere):
    o = sphere
    o.assemble()
    X0 = o.linear_coeffs()
    M, L = o.matrices(o.depth)
    lam = np.mean([X0[:, a] @ (L @ X0[:, a]) / (X0[:, a] @ (M @ X0[:, a])) for a in range(3)])
    assert lam == pytest.approx(2.0, rel=0.02)          # l(l+1) with l = 1 on the unit sphere
    delta = 0.2
    X1, info, w = flow_step(o, X0, delta)
    rho1 = 1.0 / (1.0 + 0.5 * delta * lam)
    r1 = _radius(o, X1)
    assert np.median(r1) == pytest.approx(rho1, rel=3e-3)
    assert r1.std() <= 5e-3
    # second step: area ratios rho1^2 weight the mass only
    X2, info, w = flow_step(o, X1, delta)
    assert np.median(w) == pytest.approx(np.median(r1) ** 2, rel=2e-3)
    rho2 = rho1 ** 2 / (rho1 ** 2 + 0.5 * delta * lam)
    assert np.median(_radius(o, X2)) == pytest.approx(np.median(r1) * rho2, rel=3e-3)
    o.assemble()
