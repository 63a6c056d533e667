"""Seeded synthetic inputs: triangle meshes and right-hand-side values.

This module holds no part of the method's arithmetic.  It only produces
vertex/triangle arrays and per-vertex values, each from a fixed recipe and a
numpy ``default_rng(seed)`` (PCG64) stream, so that the HIP path and the CPU
oracle are fed byte-identical inputs.

None of the paper's models (pulley, armadillo, brain, knot) ships here; the
meshes below are synthetic stand-ins with the shapes and sizes of the paper's
workloads (Section 5: a closed genus-0 surface, a thin tube knotted close to
itself, two nearly touching sheets that couple values across a gap).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "icosphere", "octasphere", "two_sheets", "torus", "torus_knot",
    "noisy_sphere", "unit_cubes", "cubes_checker", "u_tube", "nested_spheres", "single_triangle", "config_mesh",
    "config4_batch", "stripe_knot", "near_other_strand",
]


def _midpoint_subdivide(V, F, project):
    """One 1->4 midpoint subdivision; new vertices optionally pushed to the unit sphere."""
    F = np.asarray(F, dtype=np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    uniq, inv = np.unique(e, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    mid = 0.5 * (V[uniq[:, 0]] + V[uniq[:, 1]])
    if project:
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    nv = V.shape[0]
    m = nv + inv.reshape(3, -1).T  # midpoint of edges (01, 12, 20) per face
    a, b, c = F[:, 0], F[:, 1], F[:, 2]
    m01, m12, m20 = m[:, 0], m[:, 1], m[:, 2]
    NF = np.concatenate([
        np.stack([a, m01, m20], 1), np.stack([b, m12, m01], 1),
        np.stack([c, m20, m12], 1), np.stack([m01, m12, m20], 1)], axis=0)
    return np.concatenate([V, mid], axis=0), NF


_ICO_CACHE = {}


def icosphere(level: int):
    """Unit icosphere: icosahedron (cyclic (0, +-1, +-phi) family), `level` midpoint
    subdivisions, new vertices projected to the sphere.  Level 3: 642 V / 1280 F.
    (Built once per level and process; callers get copies.)"""
    if level not in _ICO_CACHE:
        _ICO_CACHE[level] = _icosphere(level)
    V, F = _ICO_CACHE[level]
    return V.copy(), F.copy()


def _icosphere(level: int):
    p = (1.0 + 5.0 ** 0.5) / 2.0
    V = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            V += [(0.0, s1, s2 * p), (s1, s2 * p, 0.0), (s2 * p, 0.0, s1)]
    V = np.array(V, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # faces: all triples of mutually adjacent vertices (edge length = min distance)
    D = np.linalg.norm(V[:, None] - V[None], axis=2)
    emin = D[D > 0].min()
    adj = np.abs(D - emin) < 1e-9
    F = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                if adj[i, j] and adj[j, k] and adj[i, k]:
                    n = np.cross(V[j] - V[i], V[k] - V[i])
                    F.append((i, j, k) if n @ V[i] > 0 else (i, k, j))
    F = np.array(F, dtype=np.int64)
    for _ in range(level):
        V, F = _midpoint_subdivide(V, F, True)
    return V, F.astype(np.int32)


def octasphere(level: int):
    """Unit sphere from an octahedron with `level` projected midpoint subdivisions
    (8 * 4**level triangles)."""
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    F = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int64)
    for _ in range(level):
        V, F = _midpoint_subdivide(V, F, True)
    return V, F.astype(np.int32)


def _grid_sheet(n):
    """Unit square [-1/2, 1/2]^2 as an n x n quad grid, each quad split on its
    (i,j)-(i+1,j+1) diagonal.  Returns (V with z = 0, F)."""
    t = np.linspace(-0.5, 0.5, n + 1)
    X, Y = np.meshgrid(t, t, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a = idx[:-1, :-1].ravel(); b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel(); d = idx[:-1, 1:].ravel()
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], axis=0)
    return V, F


def rodrigues(axis, angle):
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def two_sheets(n: int = 256, gap: float = 1.0 / 256, rotate: bool = True):
    """Two parallel unit squares `gap` apart (z = +-gap/2), each an n x n grid of
    split quads.  With `rotate`, both are turned by Rodrigues((1,2,3), 0.3 rad) so
    that no triangle lies in a grid plane.  Returns V, F, x_local (pre-rotation
    x coordinate) and sheet id (0 = top, 1 = bottom) per vertex."""
    V1, F1 = _grid_sheet(n)
    top = V1.copy(); top[:, 2] = gap / 2
    bot = V1.copy(); bot[:, 2] = -gap / 2
    V = np.concatenate([top, bot], axis=0)
    F = np.concatenate([F1, F1 + V1.shape[0]], axis=0)
    xloc = V[:, 0].copy()
    sheet = np.concatenate([np.zeros(len(V1), np.int32), np.ones(len(V1), np.int32)])
    if rotate:
        V = V @ rodrigues((1.0, 2.0, 3.0), 0.3).T
    return V, F.astype(np.int32), xloc, sheet


def _periodic_grid_faces(nu, nv):
    i = np.arange(nu)[:, None]; j = np.arange(nv)[None, :]
    a = (i * nv + j); b = (((i + 1) % nu) * nv + j)
    c = (((i + 1) % nu) * nv + (j + 1) % nv); d = (i * nv + (j + 1) % nv)
    a, b, c, d = (x.ravel() for x in (a, b, c, d))
    return np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], axis=0)


def torus(R: float, r: float, nu: int, nv: int):
    u = 2 * np.pi * np.arange(nu) / nu
    v = 2 * np.pi * np.arange(nv) / nv
    U, W = np.meshgrid(u, v, indexing="ij")
    V = np.stack([(R + r * np.cos(W)) * np.cos(U), (R + r * np.cos(W)) * np.sin(U),
                  r * np.sin(W)], axis=-1).reshape(-1, 3)
    return V, _periodic_grid_faces(nu, nv).astype(np.int32)


def torus_knot(p: int = 3, q: int = 5, nu: int = 16384, nv: int = 64, R: float = 1.0,
               a: float = 0.4, radius: float = 0.05, jitter: float = 1e-4, seed: int = 3):
    """Tube of `radius` swept along the (p,q) torus knot
    c(s) = ((R + a cos qs) cos ps, (R + a cos qs) sin ps, a sin qs) with the Frenet
    frame; nu x nv periodic grid of split quads; each coordinate jittered by
    N(0, jitter^2) from default_rng(seed)."""
    s = 2 * np.pi * np.arange(nu) / nu
    cq, sq, cp, sp = np.cos(q * s), np.sin(q * s), np.cos(p * s), np.sin(p * s)
    rr = R + a * cq
    c = np.stack([rr * cp, rr * sp, a * sq], 1)
    # first and second derivatives of the centre line
    drr = -a * q * sq
    d1 = np.stack([drr * cp - rr * p * sp, drr * sp + rr * p * cp, a * q * cq], 1)
    ddrr = -a * q * q * cq
    d2 = np.stack([ddrr * cp - 2 * drr * p * sp - rr * p * p * cp,
                   ddrr * sp + 2 * drr * p * cp - rr * p * p * sp,
                   -a * q * q * sq], 1)
    T = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    Nn = d2 - (d2 * T).sum(1, keepdims=True) * T
    Nn /= np.linalg.norm(Nn, axis=1, keepdims=True)
    B = np.cross(T, Nn)
    th = 2 * np.pi * np.arange(nv) / nv
    V = (c[:, None, :] + radius * (np.cos(th)[None, :, None] * Nn[:, None, :]
                                   + np.sin(th)[None, :, None] * B[:, None, :]))
    V = V.reshape(-1, 3)
    if jitter > 0:
        V = V + np.random.default_rng(seed).normal(0.0, jitter, size=V.shape)
    return V, _periodic_grid_faces(nu, nv).astype(np.int32)


def noisy_sphere(level: int, seed: int, bumps: int = 16, amp: float = 0.05, base: str = "ico"):
    """Sphere with radius 1 + amp * sum of `bumps` seeded Gaussian bumps."""
    V, F = icosphere(level) if base == "ico" else octasphere(level)
    rng = np.random.default_rng(seed)
    cen = rng.normal(size=(bumps, 3)); cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    wid = rng.uniform(0.2, 0.6, size=bumps)
    sgn = rng.choice([-1.0, 1.0], size=bumps)
    d2 = ((V[:, None, :] - cen[None]) ** 2).sum(-1)
    rad = 1.0 + amp * (sgn[None] * np.exp(-d2 / (2 * wid[None] ** 2))).sum(1)
    return V * rad[:, None], F


def unit_cubes(n: int = 6, pitch: float = 2.0, rotate: bool = True):
    """n x n x n equidistant unit cubes (12 triangles each), centre pitch `pitch`,
    turned into general position like `two_sheets`."""
    cv = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=np.float64)
    cf = np.array([[0, 2, 1], [1, 2, 3], [4, 5, 6], [5, 7, 6], [0, 1, 4], [1, 5, 4],
                   [2, 6, 3], [3, 6, 7], [0, 4, 2], [2, 4, 6], [1, 3, 5], [3, 7, 5]])
    Vs, Fs = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                Fs.append(cf + 8 * len(Vs))
                Vs.append(cv + pitch * np.array([i, j, k], dtype=np.float64))
    V = np.concatenate(Vs); F = np.concatenate(Fs)
    if rotate:
        V = V @ rodrigues((1.0, 2.0, 3.0), 0.3).T
    return V, F.astype(np.int32)


def u_tube(radius: float = 0.2, gap: float = 0.004, arm: float = 1.0, nv: int = 64, ncap: int = 12):
    """A genus-0 two-lobe surface: a tube of `radius` swept along a U (two
    parallel arms of length `arm` along y joined by a half circle of radius
    radius + gap/2, so the arms' facing walls are `gap` apart), closed by
    hemispherical caps.  nv vertices per ring; body rings about a quad's
    width apart; ncap rings per cap plus a pole; split quads and pole fans."""
    rb = radius + 0.5 * gap
    ltot = 2.0 * arm + np.pi * rb
    nb = max(2, int(round(ltot / (2.0 * np.pi * radius / nv)))) + 1
    s = np.linspace(0.0, ltot, nb)

    def centre(s):
        c = np.zeros((len(s), 3)); t = np.zeros((len(s), 3))
        a = s < arm                                   # arm A, down along -y at x = -rb
        c[a] = np.stack([np.full(a.sum(), -rb), arm - s[a], np.zeros(a.sum())], 1)
        t[a] = [0.0, -1.0, 0.0]
        b = (s >= arm) & (s <= arm + np.pi * rb)      # half circle under the origin
        ph = np.pi + (s[b] - arm) / rb
        c[b] = np.stack([rb * np.cos(ph), rb * np.sin(ph), np.zeros(b.sum())], 1)
        t[b] = np.stack([-np.sin(ph), np.cos(ph), np.zeros(b.sum())], 1)
        e = s > arm + np.pi * rb                      # arm B, up along +y at x = +rb
        c[e] = np.stack([np.full(e.sum(), rb), s[e] - arm - np.pi * rb, np.zeros(e.sum())], 1)
        t[e] = [0.0, 1.0, 0.0]
        return c, t

    c, t = centre(s)
    # cap rings beyond each end: angle psi from the pole, distance r cos psi past the end
    psi = np.pi / 2 * np.arange(1, ncap) / ncap
    caps_a = [(c[0] - t[0] * radius * np.cos(p), t[0], radius * np.sin(p)) for p in psi]
    caps_b = [(c[-1] + t[-1] * radius * np.cos(p), t[-1], radius * np.sin(p)) for p in psi[::-1]]
    rings = caps_a + [(c[i], t[i], radius) for i in range(nb)] + caps_b
    th = 2.0 * np.pi * np.arange(nv) / nv
    z = np.array([0.0, 0.0, 1.0])
    Vr = []
    for cc, tt, rr in rings:
        n = np.cross(z, tt)                           # in-plane normal
        Vr.append(cc[None, :] + rr * (np.cos(th)[:, None] * n[None, :] + np.sin(th)[:, None] * z[None, :]))
    Vr = np.concatenate(Vr)
    nr = len(rings)
    pole_a = c[0] - t[0] * radius
    pole_b = c[-1] + t[-1] * radius
    V = np.concatenate([Vr, pole_a[None, :], pole_b[None, :]])
    ia, ib = nr * nv, nr * nv + 1
    i = np.arange(nr - 1)[:, None]; j = np.arange(nv)[None, :]
    a = i * nv + j; b = (i + 1) * nv + j; cq = (i + 1) * nv + (j + 1) % nv; d = i * nv + (j + 1) % nv
    a, b, cq, d = (x.ravel() for x in (a, b, cq, d))
    F = [np.stack([a, b, cq], 1), np.stack([a, cq, d], 1)]
    jj = np.arange(nv)
    F.append(np.stack([np.full(nv, ia), jj, (jj + 1) % nv], 1))
    last = (nr - 1) * nv
    F.append(np.stack([np.full(nv, ib), last + (jj + 1) % nv, last + jj], 1))
    return V, np.concatenate(F).astype(np.int32)


def nested_spheres(level: int = 4, gap: float = 0.02, rotation=None):
    """Two concentric icospheres (radii 1 and 1 + gap), optionally turned by
    a rotation matrix: a closed surface pair closer than a cell, whose exact
    Laplace-Beltrami spectrum is l(l + 1) and l(l + 1) / (1 + gap)^2, each
    with multiplicity 2l + 1."""
    V1, F1 = icosphere(level)
    V = np.concatenate([V1, V1 * (1.0 + gap)])
    if rotation is not None:
        V = V @ np.asarray(rotation, dtype=np.float64).T
    return V, np.concatenate([F1, F1 + len(V1)]).astype(np.int32)


def _cube_lattice(s: int):
    """Surface of [0, s]^3 as split unit quads on the integer lattice, one
    vertex per lattice point (faces share the vertices of the cube's edges)."""
    quads = []
    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3
        for side in (0, s):
            a, b = np.meshgrid(np.arange(s), np.arange(s), indexing="ij")
            a, b = a.ravel(), b.ravel()
            corners = []
            for da, db in ((0, 0), (1, 0), (1, 1), (0, 1)):
                p = np.zeros((a.size, 3), np.int64)
                p[:, ax] = side; p[:, u] = a + da; p[:, v] = b + db
                corners.append(p)
            quads.append(np.stack(corners, 1))
    q = np.concatenate(quads)                                  # (6 s^2, 4, 3)
    pts, inv = np.unique(q.reshape(-1, 3), axis=0, return_inverse=True)
    qi = inv.reshape(-1, 4)
    F = np.concatenate([qi[:, [0, 1, 2]], qi[:, [0, 2, 3]]])
    return pts.astype(np.float64) / s, F


def cubes_checker(n: int = 6, pitch: float = 2.0, subdiv: int = 4, size: float = 0.5,
                  offset: float = 0.1234):
    """n x n x n equidistant unit cubes (centre pitch `pitch`), each face an
    subdiv x subdiv grid of split quads, shifted by `offset` along every axis
    (faces parallel to the grid planes but off them), with a solid 3D checker
    of cell `size` as a per-vertex colour: (0.9, 0.2, 0.2) where
    floor(x/size) + floor(y/size) + floor(z/size) is even, else
    (0.2, 0.3, 0.9), taken in the cubes' unshifted frame.  Returns V, F and
    the colours (nv x 3)."""
    cv, cf = _cube_lattice(subdiv)
    Vs, Fs = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                Fs.append(cf + len(cv) * len(Vs))
                Vs.append(cv + pitch * np.array([i, j, k], dtype=np.float64))
    V = np.concatenate(Vs)
    par = np.floor(V / size).astype(np.int64).sum(1) % 2
    col = np.where(par[:, None] == 0, np.array([0.9, 0.2, 0.2]), np.array([0.2, 0.3, 0.9]))
    return V + offset, np.concatenate(Fs).astype(np.int32), col


def single_triangle():
    """One generic triangle (used with an explicit box so it sits inside one cell)."""
    V = np.array([[0.31, 0.27, 0.43], [0.71, 0.36, 0.52], [0.42, 0.69, 0.61]])
    return V, np.array([[0, 1, 2]], dtype=np.int32)


def stripe_knot(nu: int = 8192, nv: int = 64, radius: float = 0.35, stripes: int = 40, seed: int = 5100):
    """A self-intersecting (3,5) torus-knot tube: radius 0.35 exceeds half the
    smallest distance between distinct strands of the centre line (0.567), and
    stays below its smallest radius of curvature (0.73), so the tube passes
    through itself where strands come close but never folds.  The colour is a
    stripe texture along the knot, f = cos(stripes * s) at the vertices of
    centre-line parameter s.  Returns V, F, f (nv x 1) and s per vertex."""
    V, F = torus_knot(nu=nu, nv=nv, radius=radius, seed=seed)
    s = np.repeat(2 * np.pi * np.arange(nu) / nu, nv)
    return V, F, np.cos(stripes * s)[:, None], s


def near_other_strand(V, s, dist: float, min_ds: float = 0.6):
    """Vertices within `dist` of a vertex whose centre-line parameter differs by
    more than min_ds (circularly): where the self-intersecting tube passes
    through or near another part of itself."""
    from scipy.spatial import cKDTree
    pairs = cKDTree(V).query_pairs(dist, output_type="ndarray")
    ds = np.abs(s[pairs[:, 0]] - s[pairs[:, 1]])
    ds = np.minimum(ds, 2 * np.pi - ds)
    far = pairs[ds > min_ds]
    mask = np.zeros(len(V), dtype=bool)
    mask[far.ravel()] = True
    return mask


def config4_batch(count: int = 64, seed: int = 4000):
    """The batch of uneven meshes, member i from seed + i: i % 3 == 0 an
    icosphere of level 3..7, 1 a torus with R/r ~ U[2, 6] and log-uniform
    1k..1.3M triangles (quad grid nu x nv with nu / nv = R / r), 2 a
    noise-displaced icosphere of level 3..8 (16 Gaussian bumps, amplitude
    0.05).  Each gets the depth clamp(round(log2(side / mean edge)), 6, 10) and
    k ~ U{1..16} right-hand-side columns of per-vertex N(0, 1) values.
    Returns a list of dicts (kind, V, F, depth, fv)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        kind = i % 3
        if kind == 0:
            V, F = icosphere(3 + (i // 3) % 5)
            name = f"icosphere L{3 + (i // 3) % 5}"
        elif kind == 1:
            ratio = float(rng.uniform(2.0, 6.0))
            tris = float(np.exp(rng.uniform(np.log(1e3), np.log(1.3e6))))
            nv = max(4, int(round(np.sqrt(tris / (2.0 * ratio)))))
            nu = max(8, int(round(tris / (2.0 * nv))))
            V, F = torus(ratio, 1.0, nu, nv)
            name = f"torus R/r={ratio:.2f} {nu}x{nv}"
        else:
            lev = 3 + (i // 3) % 6
            V, F = noisy_sphere(lev, seed=seed + i)
            name = f"noisy icosphere L{lev}"
        e = np.linalg.norm(V[F[:, 1]] - V[F[:, 0]], axis=1).mean()
        side = 1.125 * (V.max(0) - V.min(0)).max()
        depth = int(np.clip(np.round(np.log2(side / e)), 6, 10))
        k = int(rng.integers(1, 17))
        fv = np.asfortranarray(rng.normal(size=(len(V), k)))
        out.append(dict(kind=name, V=V, F=F, depth=depth, fv=fv))
    return out


def config_mesh(name: str, **kw):
    """Workload meshes by name, with their right-hand sides:
    'icosphere_l3'  : 642 V / 1280 F unit icosphere; f = z + N(0, 0.01^2), seed 1.
    'two_sheets_256': 2 x 131,072 tris, 1/256 apart, rotated; f = +-sin(40 pi x_local).
    'knot_2m'       : (3,5) knot tube, 16384 x 64 -> 2,097,152 tris, jitter seed 3;
                      f = vertex coordinates (3 columns)."""
    if name == "icosphere_l3":
        V, F = icosphere(3)
        f = V[:, 2] + np.random.default_rng(1).normal(0.0, 0.01, size=V.shape[0])
        return V, F, f[:, None]
    if name.startswith("two_sheets"):
        n = kw.get("n", 256)
        V, F, xl, sh = two_sheets(n, kw.get("gap", 1.0 / 256), kw.get("rotate", True))
        f = np.where(sh == 0, 1.0, -1.0) * np.sin(40 * np.pi * xl)
        return V, F, f[:, None]
    if name.startswith("knot"):
        V, F = torus_knot(nu=kw.get("nu", 16384), nv=kw.get("nv", 64), seed=kw.get("seed", 3))
        return V, F, V.copy()
    raise KeyError(name)
