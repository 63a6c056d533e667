"""Reference for the learned Jacobi smoother (test infrastructure only).

Plain FP64 numpy, written from the definitions: the per-row features, the
30-32-32-1 ReLU network with s = 2 sigmoid(z) and omega = c s, c the l1-Jacobi
bound A_ii / sum_j |A_ij|, the damped Jacobi error
sweeps e <- e - omega D^-1 A e and the training loss
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


def forward(params, f):
    """Hidden pre-activations and z of every row."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    a1 = f @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return a1, h1, a2, h2, z


def omega(params, f, act, c1):
    """omega_i = c_i s_i with s_i = 2 sigmoid(z_i); 0 on inactive rows."""
    z = forward(params, f)[4]
    return np.where(act, c1 * 2.0 / (1.0 + np.exp(-z)), 0.0)


def _invdiag(A):
    dg = A.diagonal()
    return np.where(dg > 0, 1.0 / np.where(dg > 0, dg, 1.0), 0.0)


def loss(A, f, act, c1, params, E0, nu):
    """Mean over the columns of E0 of log(|A e_nu|^2 / |A e_0|^2)."""
    A = A.tocsr()
    om = omega(params, f, act, c1)
    dinv = _invdiag(A)
    E = np.array(E0, dtype=np.float64, ndmin=2).reshape(A.shape[0], -1)
    r0 = A @ E
    for _ in range(nu):
        E = E - (om * dinv)[:, None] * (A @ E)
    r = A @ E
    return float(np.mean(np.log(np.sum(r * r, axis=0) / np.sum(r0 * r0, axis=0))))


def loss_grad(A, f, act, c1, params, E0, nu):
    """(loss, gradient over the packed parameters)."""
    A = A.tocsr()
    n = A.shape[0]
    a1, h1, a2, h2, z = forward(params, f)
    sg = 2.0 / (1.0 + np.exp(-z))
    om = np.where(act, c1 * sg, 0.0)
    dinv = _invdiag(A)
    E = np.array(E0, dtype=np.float64, ndmin=2).reshape(n, -1)
    S = E.shape[1]
    r0 = A @ E
    U = []
    for _ in range(nu):
        u = dinv[:, None] * (A @ E)          # D^-1 A e_k
        U.append(u)
        E = E - om[:, None] * u
    r = A @ E
    n0 = np.sum(r0 * r0, axis=0)
    n1 = np.sum(r * r, axis=0)
    L = float(np.mean(np.log(n1 / n0)))
    # dL/de_nu = (2 / S) A r / |r|^2 per column (A symmetric)
    G = (A @ r) * (2.0 / S / n1)[None, :]
    gom = np.zeros(n)
    for k in range(nu - 1, -1, -1):
        # e_{k+1} = e_k - omega * u_k,  u_k = D^-1 A e_k
        gom -= np.sum(G * U[k], axis=1)
        G = G - A @ ((om * dinv)[:, None] * G)
    dz = np.where(act, gom * c1 * sg * (1.0 - 0.5 * sg), 0.0)   # d omega / dz = c s (1 - s / 2)
    W1, b1, W2, b2, w3, b3 = unpack(params)
    d2 = (dz[:, None] * w3[None, :]) * (a2 > 0)
    d1 = (d2 @ W2.T) * (a1 > 0)
    grad = pack(f.T @ d1, d1.sum(axis=0), h1.T @ d2, d2.sum(axis=0), h2.T @ dz, dz.sum())
    return L, grad
