"""The synthetic inputs are what the documentation says they are.

Closed two-manifolds with the stated topology (every edge shared by exactly
two triangles; Euler characteristic 2 per sphere-like component), the stated
gaps and radii, and the checker colouring of the cubes model.
"""
import numpy as np

from paper_1505_03615_amd import meshgen


def _edges(F):
    E = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), 1)
    return np.unique(E, axis=0, return_counts=True)


def _components(nv, F):
    parent = np.arange(nv)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in np.concatenate([F[:, [0, 1]], F[:, [1, 2]]]):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return len({find(v) for v in range(nv)})


def test_u_tube_is_a_closed_genus_zero_surface_with_the_stated_gap():
    V, F = meshgen.u_tube(nv=32, ncap=6)
    u, c = _edges(F)
    assert np.all(c == 2)
    assert len(V) - len(u) + len(F) == 2
    arm_a = V[(V[:, 0] < 0) & (V[:, 1] > 0.1)]
    arm_b = V[(V[:, 0] > 0) & (V[:, 1] > 0.1)]
    assert abs((arm_b[:, 0].min() - arm_a[:, 0].max()) - 0.004) < 1e-12


def test_cubes_checker_has_216_closed_cubes_and_two_colours():
    V, F, col = meshgen.cubes_checker(n=6, subdiv=4)
    u, c = _edges(F)
    assert np.all(c == 2)
    assert _components(len(V), F) == 216
    assert len(V) - len(u) + len(F) == 2 * 216
    assert len(F) == 216 * 6 * 4 * 4 * 2
    assert len(np.unique(col, axis=0)) == 2
    # faces are parallel to the coordinate planes at the stated offset
    assert np.allclose(np.sort(np.unique(np.round(V[:, 0] - 0.1234, 9)))[[0, -1]], [0.0, 11.0])


def test_nested_spheres_radii_and_rotation():
    V, F = meshgen.nested_spheres(3, 0.02)
    r = np.linalg.norm(V, axis=1)
    n = len(V) // 2
    assert np.allclose(r[:n], 1.0) and np.allclose(r[n:], 1.02)
    R = meshgen.rodrigues((1.0, -2.0, 0.5), 0.9)
    Vr, Fr = meshgen.nested_spheres(3, 0.02, rotation=R)
    assert np.allclose(Vr, V @ R.T) and np.array_equal(Fr, F)
    u, c = _edges(F)
    assert np.all(c == 2) and _components(len(V), F) == 2


def test_stripe_knot_passes_through_itself():
    """The stripe knot's tube (radius 0.35) reaches across to other strands;
    the same sweep with the thin tube (radius 0.05) never does."""
    V, F, f, s = meshgen.stripe_knot(nu=512, nv=24)
    assert meshgen.near_other_strand(V, s, 0.05).sum() > 0.1 * len(V)
    assert np.allclose(f[:, 0], np.cos(40 * s))
    Vt, Ft = meshgen.torus_knot(nu=512, nv=24, radius=0.05, seed=5100)
    assert meshgen.near_other_strand(Vt, s, 0.05).sum() == 0
