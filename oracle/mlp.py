"""FP64 reference of the learned gradient screen: feature rows, the 3-layer
MLP forward and backward with the same BF16 quantisation points as the GPU
kernels, Adam, and the screen's selection rule.

TEST INFRASTRUCTURE.  The screen is not in the paper; it ranks the operator
pool so that ADAPT-VQE's exact pool gradients ("Numerical performance": the
gradient over the whole pool is the bottleneck) are computed only for a
top-K plus an audit sample.  Every definition below is written from its
statement: features, MLP y = W3 relu(W2 relu(W1 f + b1) + b2) + b3, MSE
loss, Adam.  BF16 rounding happens at the points the GPU rounds: the feature
rows, W1, W2, the first layer's activations, and the two backward error
signals that enter matrix products (dZ2, dZ1); everything else is FP64 here.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 32
HID = 256
N_PARAM = HID * N_FEAT + HID + HID * HID + HID + HID + 1


def bf16(x):
    """Round to FP32 (RNE), then to BF16 (RNE); returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + HID * N_FEAT].reshape(HID, N_FEAT); o += HID * N_FEAT
    b1 = p[o:o + HID]; o += HID
    W2 = p[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = p[o:o + HID]; o += HID
    W3 = p[o:o + HID]; o += HID
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, np.atleast_1d(b3)])


def forward(p, X, quant=True):
    q = bf16 if quant else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Xq = q(X)
    Z1 = Xq @ q(W1).T + b1
    H1 = q(np.maximum(Z1, 0.0))
    Z2 = H1 @ q(W2).T + b2
    y = np.maximum(Z2, 0.0) @ W3 + b3[0]
    return y, (Xq, Z1, H1, Z2)


def loss_grad(p, X, t, quant=True):
    """MSE loss mean((y - t)^2) and its parameter gradient (backward pass)."""
    q = bf16 if quant else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (Xq, Z1, H1, Z2) = forward(p, X, quant)
    B = X.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    A2 = np.maximum(Z2, 0.0)
    dW3 = A2.T @ dy
    db3 = np.array([dy.sum()])
    dZ2 = np.outer(dy, W3) * (Z2 > 0)
    db2 = dZ2.sum(axis=0)
    dZ2q = q(dZ2)
    dW2 = dZ2q.T @ H1
    dH1 = dZ2q @ q(W2)
    dZ1 = dH1 * (Z1 > 0)
    db1 = dZ1.sum(axis=0)
    dW1 = q(dZ1).T @ Xq
    return loss, y, pack(dW1, db1, dW2, db2, dW3, db3)


class Adam:
    def __init__(self, p, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.p = np.asarray(p, dtype=np.float64).copy()
        self.m = np.zeros_like(self.p)
        self.v = np.zeros_like(self.p)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        self.p = self.p - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.p


# ---------------------------------------------------------------- features

def static_features(n_orb, cre, ann, cls, h, g):
    """Per operator: class one-hot (0..4), spatial orbital indices / (M-1)
    of (c1, c2, a1, a2) with -1 padding (5..8), log10(|integral| + 1e-12)
    (9..10: h_ca for singles, (c1 a1|c2 a2) and (c1 a2|c2 a1) for doubles),
    M/16 (17); the qubit indices of (c1, c2, a1, a2) (-1 padding)."""
    M = n_orb
    n = len(cre)
    F = np.zeros((n, N_FEAT))
    Q = -np.ones((n, 4), dtype=np.int64)
    den = max(M - 1, 1)
    for k in range(n):
        cq = [q for q in range(2 * M) if (int(cre[k]) >> q) & 1]
        aq = [q for q in range(2 * M) if (int(ann[k]) >> q) & 1]
        F[k, int(cls[k])] = 1.0
        sp = [q % M for q in cq] + [-1] * (2 - len(cq)) + [q % M for q in aq] + [-1] * (2 - len(aq))
        qs = cq + [-1] * (2 - len(cq)) + aq + [-1] * (2 - len(aq))
        for i in range(4):
            F[k, 5 + i] = sp[i] / den if sp[i] >= 0 else -1.0
            Q[k, i] = qs[i]
        if len(cq) == 1:
            F[k, 9] = math.log10(abs(h[cq[0] % M, aq[0] % M]) + 1e-12)
        else:
            c1, c2 = cq[0] % M, cq[1] % M
            a1, a2 = aq[0] % M, aq[1] % M
            F[k, 9] = math.log10(abs(g[c1, a1, c2, a2]) + 1e-12)
            F[k, 10] = math.log10(abs(g[c1, a2, c2, a1]) + 1e-12)
        F[k, 17] = M / 16.0
    # a 4-qubit list for singles: (c, -1, a, -1) -> keep (c, a, -1, -1) order
    for k in range(n):
        if int(cls[k]) <= 1:
            Q[k] = [Q[k, 0], Q[k, 2], -1, -1]
            F[k, 5:9] = [F[k, 5], F[k, 7], -1.0, -1.0]
    return F, Q


def features(F_static, Q, occ, gprev, age, n_orb=None, last=None, last_g=0.0):
    """Full feature rows (FP64; the GPU rounds FP32 values to BF16).  With
    the last selected operator's four qubit indices `last` (qidx layout):
    slot 18 marks that operator, 19 and 20 count the spin-orbitals and the
    spatial orbitals it shares with each operator (/ 4), 21 is
    log10(|last_g| + 1e-12); all four are 0 when there is no selection."""
    X = np.array(F_static, dtype=np.float64)
    for i in range(4):
        X[:, 11 + i] = np.where(Q[:, i] >= 0, occ[np.maximum(Q[:, i], 0)], 0.0)
    X[:, 15] = np.log10(np.abs(gprev) + 1e-12)
    X[:, 16] = np.minimum(age, 50) / 10.0
    if last is not None and any(int(q) >= 0 for q in last):
        M = int(n_orb)
        lq = set(int(q) for q in last if int(q) >= 0)
        ls = set(q % M for q in lq)
        for k in range(X.shape[0]):
            kq = set(int(q) for q in Q[k] if int(q) >= 0)
            X[k, 18] = 1.0 if [int(q) for q in Q[k]] == [int(q) for q in last] else 0.0
            X[k, 19] = len(kq & lq) / 4.0
            X[k, 20] = len(set(q % M for q in kq) & ls) / 4.0
            X[k, 21] = math.log10(abs(last_g) + 1e-12)
    return X


def select(scores, K, audit_ranks):
    """Top-K operators by score (stable: ties keep the lower index), plus the
    operators at the given ranks among the rest (the audit sample)."""
    order = np.argsort(-np.asarray(scores, dtype=np.float32), kind="stable")
    top = order[:K]
    rest = order[K:]
    aud = rest[np.asarray(audit_ranks, dtype=np.int64)]
    return top, aud
