"""Reference for the learned Jacobi smoother (test infrastructure only).

Plain FP64 numpy, written from the definitions: the per-row features, the
30-32-32-1 ReLU network with s = 2 sigmoid(z), and two sweep types: damped
Jacobi with omega = c s, c the l1-Jacobi bound A_ii / sum_j |A_ij|
(e <- e - omega D^-1 A e on all rows at once), and multicolour SOR with
omega = 1/2 + sigmoid(z) (the same update applied to the rows of colour 0, then colour 1,
..., colour = parity of the corner coordinates); the training loss
L = mean_s log(|A e_nu^s|^2 / |A e_0^s|^2), with its gradient obtained by
the chain rule written out by hand (adjoint sweeps, then back-propagation
through the network).  Nothing here comes from the paper: its smoother is
Gauss-Seidel (Section 5.2); this smoother is an optional replacement for it.
The HIP library is never imported.

Parameter packing of one network (2081 floats): W1[30][32], b1[32],
W2[32][32], b2[32], w3[32], b3, with W[i][j] mapping input i to output j.
"""
from __future__ import annotations

import numpy as np

NF, NH = 30, 32
O_W1 = 0
O_B1 = O_W1 + NF * NH
O_W2 = O_B1 + NH
O_B2 = O_W2 + NH * NH
O_W3 = O_B2 + NH
O_B3 = O_W3 + NH
NP = O_B3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64).reshape(-1)
    assert p.size == NP
    return (p[O_W1:O_B1].reshape(NF, NH), p[O_B1:O_W2], p[O_W2:O_B2].reshape(NH, NH), p[O_B2:O_W3],
            p[O_W3:O_B3], p[O_B3])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]])


def bf16_round(p):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    u = np.asarray(p, dtype=np.float32).view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = np.where(finite, u + 0x7FFF + ((u >> 16) & 1), u)
    return ((r >> 16) << 16).astype(np.uint32).view(np.float32)


def demorton(keys):
    """(n, 3) grid coordinates of Morton keys (bit b of x at 3b, y at 3b+1, z at 3b+2)."""
    keys = np.asarray(keys, dtype=np.uint64)
    c = np.zeros((len(keys), 3), dtype=np.int64)
    for b in range(21):
        for a in range(3):
            c[:, a] |= ((keys >> np.uint64(3 * b + a)) & np.uint64(1)).astype(np.int64) << b
    return c


def features(A, M, keys, d, D):
    """Row features (n, 30), the active mask and the l1-Jacobi bound
    c_i = A_ii / sum_j |A_ij| for A = M + t L at depth d.

    [0..27): entries of row i summed per grid offset delta in {-1,0,1}^3 of the
    column's corner from the row's corner, over A_ii, at index
    (dx+1) + 3 (dy+1) + 9 (dz+1); [27] clamp(log10(A_ii / max_j A_jj), -30, 0)/10;
    [28] M_ii / A_ii; [29] (D - d) / 10.  Rows with A_ii <= 0 (no computed
    mass) are inactive and all zero."""
    A = A.tocsr()
    M = M.tocsr()
    n = A.shape[0]
    diag = A.diagonal()
    mdiag = M.diagonal()
    c = demorton(keys)
    act = diag > 0
    dmax = diag[act].max() if act.any() else 1.0
    f = np.zeros((n, NF))
    c1 = np.zeros(n)
    for i in range(n):
        if not act[i]:
            continue
        c1[i] = diag[i] / np.abs(A.data[A.indptr[i]:A.indptr[i + 1]]).sum()
        for e in range(A.indptr[i], A.indptr[i + 1]):
            j = A.indices[e]
            dx, dy, dz = c[j] - c[i]
            if max(abs(dx), abs(dy), abs(dz)) <= 1:
                f[i, (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] += A.data[e] / diag[i]
        f[i, 27] = min(0.0, max(-30.0, np.log10(diag[i] / dmax))) / 10.0
        f[i, 28] = mdiag[i] / diag[i]
        f[i, 29] = (D - d) / 10.0
    return f, act, c1


def colours(keys):
    """Colour of each degree-1 function: (x & 1) + 2 (y & 1) + 4 (z & 1) of its corner."""
    c = demorton(keys)
    return (c[:, 0] & 1) + 2 * (c[:, 1] & 1) + 4 * (c[:, 2] & 1)


def _masks(n, colour, forward=True):
    """Rows relaxed by each step of one sweep: all rows (Jacobi) or one colour
    at a time (colours 0..7, or 7..0 when not forward)."""
    if colour is None:
        return [np.ones(n, bool)]
    order = range(8) if forward else range(7, -1, -1)
    return [colour == c for c in order]


def coarse_inverse(Ac, eps):
    """D^-1/2 (D^-1/2 Ac D^-1/2 + eps I)^-1 D^-1/2, dense; a row of zero
    diagonal gets a unit diagonal in the scaled matrix and a zero row and
    column in the result (the coarsest solve of the multigrid cycle)."""
    A = Ac.toarray()
    d = np.diag(A).copy()
    pos = d > 0
    s = np.where(pos, 1.0 / np.sqrt(np.where(pos, d, 1.0)), 0.0)
    As = s[:, None] * A * s[None, :]
    idx = np.where(~pos)[0]
    As[idx, idx] = 1.0
    As += eps * np.eye(len(d))
    return s[:, None] * np.linalg.inv(As) * s[None, :]


def coarse_correction(A, P, Bc):
    """(e -> e - P Bc P^T A e, its transpose g -> g - A P Bc P^T g) for a
    symmetric coarse operator Bc (a dense matrix or a function)."""
    A = A.tocsr()
    P = P.tocsr()
    apply_bc = Bc if callable(Bc) else (lambda x: Bc @ x)
    def fwd(E):
        return E - P @ apply_bc(P.T @ (A @ E))
    def adj(G):
        return G - A @ (P @ apply_bc(P.T @ G))
    return fwd, adj


def _ops(n, nu, colour, cc):
    """The cycle as a list of steps: ('relax', rows) or ('cc',).  Without cc:
    nu sweeps; with cc: nu sweeps, the coarse correction, nu sweeps with the
    colours reversed."""
    ops = [("relax", m) for _ in range(nu) for m in _masks(n, colour, True)]
    if cc is not None:
        ops.append(("cc",))
        ops += [("relax", m) for _ in range(nu) for m in _masks(n, colour, False)]
    return ops


def forward(params, f):
    """Hidden pre-activations and z of every row."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    a1 = f @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return a1, h1, a2, h2, z


def _two_sigmoid(z):
    """2 / (1 + exp(-z)) without overflow for large |z|."""
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 2.0 / (1.0 + e), 2.0 * e / (1.0 + e))


def omega(params, f, act, c1, sor=False):
    """Jacobi: omega_i = c_i s_i with s_i = 2 sigmoid(z_i); SOR: omega_i =
    1/2 + sigmoid(z_i); 0 on inactive rows."""
    z = forward(params, f)[4]
    w = 0.5 + 0.5 * _two_sigmoid(z) if sor else c1 * _two_sigmoid(z)
    return np.where(act, w, 0.0)


def _invdiag(A):
    dg = A.diagonal()
    return np.where(dg > 0, 1.0 / np.where(dg > 0, dg, 1.0), 0.0)


def relax(A, f, act, c1, params, E0, nu, colour=None, cc=None):
    """The error after nu sweeps (Jacobi when colour is None, omega = c s;
    multicolour SOR otherwise, omega = 1/2 + sigmoid(z)), or after a two-grid
    cycle when cc = (forward, adjoint) of the coarse correction is given."""
    A = A.tocsr()
    n = A.shape[0]
    om = omega(params, f, act, c1, sor=colour is not None)
    dinv = _invdiag(A)
    E = np.array(E0, dtype=np.float64, ndmin=2).reshape(n, -1)
    for op in _ops(n, nu, colour, cc):
        if op[0] == "cc":
            E = cc[0](E)
        else:
            E = E - np.where(op[1], om * dinv, 0.0)[:, None] * (A @ E)
    return E


def loss(A, f, act, c1, params, E0, nu, colour=None, cc=None):
    """Mean over the columns of E0 of log(|A e_end|^2 / |A e_0|^2)."""
    A = A.tocsr()
    E0 = np.array(E0, dtype=np.float64, ndmin=2).reshape(A.shape[0], -1)
    r0 = A @ E0
    r = A @ relax(A, f, act, c1, params, E0, nu, colour, cc)
    return float(np.mean(np.log(np.sum(r * r, axis=0) / np.sum(r0 * r0, axis=0))))


def loss_grad(A, f, act, c1, params, E0, nu, colour=None, cc=None):
    """(loss, gradient over the packed parameters)."""
    A = A.tocsr()
    n = A.shape[0]
    a1, h1, a2, h2, z = forward(params, f)
    sg = _two_sigmoid(z)
    om = omega(params, f, act, c1, sor=colour is not None)
    dinv = _invdiag(A)
    E = np.array(E0, dtype=np.float64, ndmin=2).reshape(n, -1)
    S = E.shape[1]
    r0 = A @ E
    ops = _ops(n, nu, colour, cc)
    U = []
    for op in ops:
        if op[0] == "cc":
            U.append(None)
            E = cc[0](E)
            continue
        u = np.where(op[1][:, None], dinv[:, None] * (A @ E), 0.0)     # D^-1 A e_k on the relaxed rows
        U.append(u)
        E = E - om[:, None] * u
    r = A @ E
    n0 = np.sum(r0 * r0, axis=0)
    n1 = np.sum(r * r, axis=0)
    L = float(np.mean(np.log(n1 / n0)))
    # dL/de_nu = (2 / S) A r / |r|^2 per column (A symmetric)
    G = (A @ r) * (2.0 / S / n1)[None, :]
    gom = np.zeros(n)
    for k in range(len(ops) - 1, -1, -1):
        if ops[k][0] == "cc":
            G = cc[1](G)
            continue
        # e_{k+1} = e_k - omega * u_k,  u_k = (D^-1 A e_k) on the step's rows
        gom -= np.sum(G * U[k], axis=1)
        G = G - A @ (np.where(ops[k][1], om * dinv, 0.0)[:, None] * G)
    if colour is None:
        dz = np.where(act, gom * c1 * sg * (1.0 - 0.5 * sg), 0.0)      # d omega / dz = c s (1 - s / 2)
    else:
        sig = 0.5 * sg
        dz = np.where(act, gom * sig * (1.0 - sig), 0.0)                # d omega / dz = sigma (1 - sigma)
    W1, b1, W2, b2, w3, b3 = unpack(params)
    d2 = (dz[:, None] * w3[None, :]) * (a2 > 0)
    d1 = (d2 @ W2.T) * (a1 > 0)
    grad = pack(f.T @ d1, d1.sum(axis=0), h1.T @ d2, d2.sum(axis=0), h2.T @ dz, dz.sum())
    return L, grad
