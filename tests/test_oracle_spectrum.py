"""Pins of the spectrum (Section 5.1): L x = lambda M x.

Two concentric unit spheres 0.02 apart (closer than a cell at depth 4) have
the exact spectrum l(l+1) and l(l+1)/1.02^2, each with multiplicity 2l + 1.
The split space reproduces it within 1 % for l <= 2: two zero eigenvalues
(one constant per sphere) and both triplets.  The unsplit space ties the
spheres together: one zero eigenvalue and a single triplet between the two
exact ones.
"""
import numpy as np

from oracle import Oracle
from paper_1505_03615_amd import meshgen

GAP = 0.02


def _exact(k):
    ev = []
    for l in range(6):
        ev += [l * (l + 1.0)] * (2 * l + 1) + [l * (l + 1.0) / (1 + GAP) ** 2] * (2 * l + 1)
    return np.sort(ev)[:k]


def test_split_spectrum_of_nested_spheres_matches_the_closed_form():
    V, F = meshgen.nested_spheres(4, GAP)
    o = Oracle(V, F, 4, split=1, min_depth=4, max_coarse=0).check().assemble()
    ev = o.eigenvalues(18)
    ex = _exact(18)
    assert np.all(np.abs(ev[:2]) < 1e-9)
    assert np.all(np.abs(ev[2:] - ex[2:]) / ex[2:] < 0.01), (ev, ex)


def test_unsplit_space_merges_the_spheres():
    V, F = meshgen.nested_spheres(4, GAP)
    o = Oracle(V, F, 4, split=0, min_depth=4, max_coarse=0).check().assemble()
    ev = o.eigenvalues(6)
    assert abs(ev[0]) < 1e-9 and ev[1] > 1.5            # one constant only
    lo, hi = 2.0 / (1 + GAP) ** 2, 2.0
    assert np.all((ev[1:4] > lo) & (ev[1:4] < hi * 1.005))   # one triplet between the exact two
    assert ev[4] > 5.0
