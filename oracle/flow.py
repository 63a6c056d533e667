"""Reference for one tracked cMCF step (test infrastructure only).

Section 5.3: (M_t + delta/2 L_0) u_{t+delta} = M_t u_t.  Test functions are
tracked (the hierarchy of the original surface is kept), so L_0 is the
original stiffness matrix and M_t the original mass integral with every
triangle weighted by its current area over its original area; the current
surface is the mesh with its vertices moved to u_t = sum_i X_i b_i.  Written
as the plain composition of the oracle's own steps (vertex evaluation,
weighted assembly, matrix product, solve); the HIP library is never imported.
"""
from __future__ import annotations

import numpy as np


def triangle_areas(V, F):
    c = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    return 0.5 * np.linalg.norm(c, axis=1)


def flow_step(o, X, delta, rtol=1e-12, max_iter=400):
    """(X', solve info, triangle weights) for the coefficients X (n x 3) of u_t."""
    P = o.eval_vertices(X)
    w = triangle_areas(P, o.F) / triangle_areas(o.V, o.F)
    o.assemble(tri_weight=w)
    M, _ = o.matrices(o.depth)
    b = M @ np.asarray(X)
    Xn, info = o.solve(0.5 * delta, b, rtol=rtol, max_iter=max_iter, x0=X)
    return Xn, info, w
