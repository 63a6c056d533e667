"""Exact-rational brute force for the discrete structure (tiny inputs only).

Independent of the oracle's separating-axis predicates: a triangle meets an
open cell iff its exact clip against the closed cell has positive area (the
mesh is in general position: no triangle lies in a grid plane), a segment
meets an open box iff its exact parametric clip (Liang-Barsky) leaves an open
parameter interval, and components of supp(b_k) restricted to the mesh are
found by walking shared edges/vertices that reach into the open support
(Section 4.2).  All arithmetic is on fractions.Fraction.
"""
from fractions import Fraction as Fr
from itertools import product


def morton3(x, y, z):
    k = 0
    for b in range(21):
        k |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return k


def _clip_closed(poly, a, v, ge):
    out = []
    n = len(poly)
    for i in range(n):
        P, Q = poly[i], poly[(i + 1) % n]
        inP = P[a] >= v if ge else P[a] <= v
        inQ = Q[a] >= v if ge else Q[a] <= v
        if inP:
            out.append(P)
        if inP != inQ:
            lam = (v - P[a]) / (Q[a] - P[a])
            out.append(tuple(P[b] + lam * (Q[b] - P[b]) for b in range(3)))
    return out


def clipped_area2(tri, lo, hi):
    """Squared norm of twice the vector area of tri clipped to box [lo, hi]."""
    poly = [tuple(Fr(c) for c in p) for p in tri]
    for a in range(3):
        if len(poly) >= 3:
            poly = _clip_closed(poly, a, Fr(lo[a]), True)
        if len(poly) >= 3:
            poly = _clip_closed(poly, a, Fr(hi[a]), False)
    if len(poly) < 3:
        return Fr(0)
    s = [Fr(0)] * 3
    p0 = poly[0]
    for i in range(1, len(poly) - 1):
        u = [poly[i][c] - p0[c] for c in range(3)]
        w = [poly[i + 1][c] - p0[c] for c in range(3)]
        cr = [u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]]
        s = [s[c] + cr[c] for c in range(3)]
    return s[0] ** 2 + s[1] ** 2 + s[2] ** 2


def segment_meets_open_box(p, q, lo, hi):
    """Liang-Barsky on the open box: is {t in [0,1] : lo < p + t (q-p) < hi} non-empty?"""
    t0, t1 = Fr(0), Fr(1)
    open0, open1 = False, False  # whether the bound is strict
    for a in range(3):
        pa, da = Fr(p[a]), Fr(q[a]) - Fr(p[a])
        if da == 0:
            if not (Fr(lo[a]) < pa < Fr(hi[a])):
                return False
            continue
        ta, tb = (Fr(lo[a]) - pa) / da, (Fr(hi[a]) - pa) / da
        if ta > tb:
            ta, tb = tb, ta
        if ta > t0 or (ta == t0 and not open0):
            t0, open0 = ta, True
        if tb < t1 or (tb == t1 and not open1):
            t1, open1 = tb, True
    if t0 < t1:
        return True
    return t0 == t1 and not open0 and not open1


def pairs_exact(V, F, d):
    """{(Morton(cell), tri)} with positive-area overlap at depth d; V already in
    depth-d grid units (Fractions or exact floats)."""
    out = set()
    n = 1 << d
    for t, f in enumerate(F):
        tri = [V[i] for i in f]
        lo = [max(0, min(n - 1, int(min(p[a] for p in tri) // 1))) for a in range(3)]
        hi = [max(0, min(n - 1, int(max(p[a] for p in tri) // 1))) for a in range(3)]
        for z in range(lo[2], hi[2] + 1):
            for y in range(lo[1], hi[1] + 1):
                for x in range(lo[0], hi[0] + 1):
                    if clipped_area2(tri, (x, y, z), (x + 1, y + 1, z + 1)) > 0:
                        out.add((morton3(x, y, z), t))
    return out


def components_exact(V, F, d, degree=1):
    """{support key: [sorted list of triangle groups]} at depth d for the
    connectivity-aware split.  V in depth-d grid units."""
    W = 2 if degree == 1 else 3
    pairs = pairs_exact(V, F, d)
    act = {}
    for key, t in pairs:
        c = [0, 0, 0]
        for b in range(21):
            for a in range(3):
                c[a] |= ((key >> (3 * b + a)) & 1) << b
        for j in product(range(W), repeat=3):
            s = (c[0] + j[0], c[1] + j[1], c[2] + j[2])
            act.setdefault(s, set()).add(t)
    edges = {}
    verts = {}
    for t, f in enumerate(F):
        for j in range(3):
            a, b = sorted((f[j], f[(j + 1) % 3]))
            edges.setdefault((a, b), set()).add(t)
            verts.setdefault(f[j], set()).add(t)
    out = {}
    for s, tris in act.items():
        if degree == 1:
            lo, hi = [s[a] - 1 for a in range(3)], [s[a] + 1 for a in range(3)]
        else:
            lo, hi = [s[a] - 2 for a in range(3)], [s[a] + 1 for a in range(3)]
        parent = {t: t for t in tris}

        def find(x):
            while parent[x] != x:
                x = parent[x]
            return x

        def unite(a, b):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)

        for (a, b), ts in edges.items():
            ts = [t for t in ts if t in tris]
            if len(ts) > 1 and segment_meets_open_box(V[a], V[b], lo, hi):
                for t in ts[1:]:
                    unite(ts[0], t)
        for v, ts in verts.items():
            ts = [t for t in ts if t in tris]
            if len(ts) > 1 and all(Fr(lo[a]) < Fr(V[v][a]) < Fr(hi[a]) for a in range(3)):
                for t in ts[1:]:
                    unite(ts[0], t)
        groups = {}
        for t in tris:
            groups.setdefault(find(t), []).append(t)
        out[morton3(*s)] = sorted(sorted(g) for g in groups.values())
    return out
