"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only *produces inputs*: one- and two-electron integrals drawn
from a seed, their Jordan-Wigner Pauli-string form (x_mask, z_mask, coeff),
the canonical spin-orbital singles+doubles operator pool, the Hartree-Fock
occupation, and random sector states.  It holds none of the arithmetic of
the state-vector hot path (H*psi, energies, gradients, rotations); both the
oracle and the HIP library consume what it returns.

Conventions (stated once, used by every consumer):

* M spatial orbitals, n = 2M qubits.  Qubit q < M is orbital q with spin
  alpha, qubit q >= M is orbital q-M with spin beta ("blocked" order).
* A computational basis state b is an n-bit integer; bit q set = spin-orbital
  q occupied.  alpha string = b & (2^M - 1), beta string = b >> M.
* Jordan-Wigner (paper, "Sparse State-Vector Emulation": spin-orbitals are
  mapped to qubits by Jordan-Wigner): a_q = (prod_{q'<q} Z_q') (X_q + iY_q)/2
  with |1> = occupied.
* Pauli string P(x, z) = tensor over qubits of I (0,0), X (1,0), Z (0,1),
  Y (1,1) for bits (x_q, z_q).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

N_CHOLESKY = 8  # rank of the synthetic two-body factorisation


# ---------------------------------------------------------------------------
# integrals
# ---------------------------------------------------------------------------

def integrals(n_orb: int, seed: int):
    """Synthetic molecular integrals (h, g) in chemist's notation, FP64.

    h_pq = h_qp ~ N(0,1) * exp(-|p-q|/2) sampled for p <= q in row-major
    order, then h_pp += -2 - 0.5 p.  For t = 0..7 a symmetric L^t with
    entries 0.3 * N(0,1) (upper triangle incl. diagonal, row-major), and
    g_pqrs = sum_t L^t_pq L^t_rs, which is positive semidefinite as a
    (pq),(rs) supermatrix and has exact 8-fold permutational symmetry: every
    element is computed once for the upper triangle of the supermatrix, with
    t summed in order 0..7, then mirrored.
    """
    M = int(n_orb)
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    for p in range(M):
        for q in range(p, M):
            v = rng.standard_normal() * math.exp(-abs(p - q) / 2.0)
            h[p, q] = v
            h[q, p] = v
    for p in range(M):
        h[p, p] += -2.0 - 0.5 * p
    npair = M * (M + 1) // 2
    pairs = [(p, q) for p in range(M) for q in range(p, M)]
    L = np.zeros((N_CHOLESKY, npair))
    for t in range(N_CHOLESKY):
        for k in range(npair):
            L[t, k] = 0.3 * rng.standard_normal()
    # sum over t in fixed order; elementwise products are commutative so the
    # (P,R) and (R,P) entries are bit-identical.
    G = np.zeros((npair, npair))
    for t in range(N_CHOLESKY):
        G += np.multiply.outer(L[t], L[t])
    g = np.zeros((M, M, M, M))
    for a, (p, q) in enumerate(pairs):
        for b, (r, s) in enumerate(pairs):
            v = G[a, b]
            g[p, q, r, s] = v
            g[q, p, r, s] = v
            g[p, q, s, r] = v
            g[q, p, s, r] = v
    return h, g


# ---------------------------------------------------------------------------
# Jordan-Wigner Pauli list
# ---------------------------------------------------------------------------

_POPC8 = np.array([bin(i).count("1") for i in range(256)], dtype=np.int64)


def _popcount64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return _POPC8[a.view(np.uint8).reshape(a.shape + (8,))].sum(axis=-1)


def _products(ops, coeff):
    """Expand sum_i coeff[i] * prod_k ops[k][i] where ops[k][i] = (q, dagger)
    columns, into X^x Z^z terms.  Returns (x, z, c) arrays (unmerged)."""
    nops = len(ops)
    n = coeff.shape[0]
    xs, zs, cs = [], [], []
    for combo in range(1 << nops):
        x = np.zeros(n, dtype=np.uint64)
        z = np.zeros(n, dtype=np.uint64)
        c = coeff.copy()
        for k in range(nops):
            q, dag = ops[k]
            pick = (combo >> k) & 1
            e = np.left_shift(np.uint64(1), q.astype(np.uint64))
            m = e - np.uint64(1)
            xk = e
            zk = m | e if pick else m
            ck = 0.5 if (not pick or dag) else -0.5
            # (X^x Z^z)(X^xk Z^zk) = (-1)^{popc(z & xk)} X^(x^xk) Z^(z^zk)
            sgn = 1 - 2 * (_popcount64(z & xk) & 1)
            c = c * ck * sgn
            x = x ^ xk
            z = z ^ zk
        xs.append(x)
        zs.append(z)
        cs.append(c)
    return np.concatenate(xs), np.concatenate(zs), np.concatenate(cs)


def jw_pauli_list(h: np.ndarray, g: np.ndarray):
    """Pauli-string form of the second-quantised Hamiltonian

        H = sum_{pq,s} h_pq a+_{ps} a_{qs}
          + 1/2 sum_{pqrs,st} g_pqrs a+_{ps} a+_{rt} a_{st} a_{qs}

    under Jordan-Wigner with blocked spin order.  Returns (x, z, c) with
    x, z uint32 masks and c float64 real coefficients of P(x, z).  Equal
    (x, z) are merged with an exactly rounded sum (math.fsum) so that terms
    which cancel in exact arithmetic (every odd-n_Y term of a real H) become
    exactly 0.0; only exact zeros are dropped.  Sorted by (x, z).
    """
    M = h.shape[0]
    n = 2 * M
    if n > 32:
        raise ValueError("at most 32 qubits")
    # one-body: spin-orbital indices P = p + s*M
    p, q, s = np.meshgrid(np.arange(M), np.arange(M), np.arange(2), indexing="ij")
    p, q, s = p.ravel(), q.ravel(), s.ravel()
    c1 = h[p, q]
    P = p + s * M
    Q = q + s * M
    keep = c1 != 0.0
    x1, z1, k1 = _products([(P[keep], True), (Q[keep], False)], c1[keep])
    # two-body
    idx = np.indices((M, M, M, M, 2, 2)).reshape(6, -1)
    p, q, r, t_, s, u = idx
    c2 = 0.5 * g[p, q, r, t_]
    Pp = p + s * M
    Qq = q + s * M
    Rr = r + u * M
    Ss = t_ + u * M
    keep = (c2 != 0.0) & (Pp != Rr) & (Qq != Ss)
    x2, z2, k2 = _products(
        [(Pp[keep], True), (Rr[keep], True), (Ss[keep], False), (Qq[keep], False)],
        c2[keep],
    )
    x = np.concatenate([x1, x2])
    z = np.concatenate([z1, z2])
    c = np.concatenate([k1, k2])
    key = (x << np.uint64(32)) | z
    order = np.argsort(key, kind="stable")
    key = key[order]
    c = c[order]
    uniq, start = np.unique(key, return_index=True)
    bounds = list(start) + [len(key)]
    cl = c.tolist()
    out_c = np.array([math.fsum(cl[bounds[i]:bounds[i + 1]]) for i in range(len(uniq))])
    ux = (uniq >> np.uint64(32)).astype(np.uint64)
    uz = (uniq & np.uint64(0xFFFFFFFF)).astype(np.uint64)
    # X^x Z^z = (-i)^{n_Y} P(x,z): a real coefficient needs even n_Y and
    # picks up (-1)^{n_Y/2}; odd-n_Y sums must vanish exactly.
    ny = _popcount64(ux & uz)
    odd = (ny & 1) == 1
    if np.any(out_c[odd] != 0.0):
        raise ArithmeticError("odd-n_Y Pauli term with nonzero coefficient")
    out_c = out_c * (1 - 2 * ((ny // 2) & 1))
    keep = (out_c != 0.0) & (~odd)
    return (ux[keep].astype(np.uint32), uz[keep].astype(np.uint32), out_c[keep].astype(np.float64))


# ---------------------------------------------------------------------------
# operator pool
# ---------------------------------------------------------------------------

POOL_CLASSES = ("a", "b", "aa", "bb", "ab")


def canonical_pool(n_orb: int):
    """Generalised spin-orbital singles and doubles conserving N_alpha and
    N_beta, one representative per generator A = tau - tau^dagger (the one
    whose annihilation mask is numerically smaller than its creation mask).

    Returned as (cre_mask, ann_mask, cls) arrays in canonical order: class
    (alpha singles, beta singles, alpha-alpha, beta-beta, alpha-beta), then
    (ann_mask, cre_mask) ascending.  Counts: 2 C(M,2) + 6 C(M,4)
    + (M(M-1))^2 / 2.
    """
    M = int(n_orb)
    out = {k: [] for k in range(5)}
    for spin, cls in ((0, 0), (1, 1)):
        off = spin * M
        for a in range(M):
            for c in range(a + 1, M):
                out[cls].append((1 << (c + off), 1 << (a + off)))
    for spin, cls in ((0, 2), (1, 3)):
        off = spin * M
        for quad in _combinations(M, 4):
            bits = [1 << (o + off) for o in quad]
            full = sum(bits)
            seen = set()
            for i in range(4):
                for j in range(i + 1, 4):
                    m1 = bits[i] | bits[j]
                    m2 = full ^ m1
                    ann, cre = min(m1, m2), max(m1, m2)
                    if (ann, cre) not in seen:
                        seen.add((ann, cre))
                        out[cls].append((cre, ann))
    for a1 in range(M):
        for c1 in range(M):
            if a1 == c1:
                continue
            for a2 in range(M):
                for c2 in range(a2 + 1, M):
                    # beta part decides the numeric order: ann beta bit < cre beta bit
                    ann = (1 << a1) | (1 << (a2 + M))
                    cre = (1 << c1) | (1 << (c2 + M))
                    out[4].append((cre, ann))
    cre_l, ann_l, cls_l = [], [], []
    for k in range(5):
        lst = sorted(out[k], key=lambda ca: (ca[1], ca[0]))
        for cre, ann in lst:
            cre_l.append(cre)
            ann_l.append(ann)
            cls_l.append(k)
    return (np.array(cre_l, dtype=np.uint32), np.array(ann_l, dtype=np.uint32),
            np.array(cls_l, dtype=np.uint8))


def _combinations(m, k):
    import itertools
    return itertools.combinations(range(m), k)


def pool_size(n_orb: int) -> int:
    M = n_orb
    return 2 * math.comb(M, 2) + 6 * math.comb(M, 4) + (M * (M - 1)) ** 2 // 2


# ---------------------------------------------------------------------------
# states
# ---------------------------------------------------------------------------

def hf_bits(n_orb: int, n_alpha: int, n_beta: int) -> int:
    """Hartree-Fock determinant: lowest-index alpha and beta orbitals."""
    return ((1 << n_alpha) - 1) | (((1 << n_beta) - 1) << n_orb)


def near_hf_bits(n_orb: int, n_alpha: int, n_beta: int, n_exc: int = 24, seed: int = 3) -> np.ndarray:
    """Bitstrings of an early-ADAPT support: the Hartree-Fock determinant and
    n_exc determinants reached from it by one pool excitation (occupied
    orbitals annihilated, empty ones created), drawn at random (seeded)."""
    cre, ann, _ = canonical_pool(n_orb)
    hf = hf_bits(n_orb, n_alpha, n_beta)
    ok = [i for i in range(cre.size) if (int(ann[i]) & hf) == int(ann[i]) and (int(cre[i]) & hf) == 0]
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(ok), size=min(n_exc, len(ok)), replace=False)
    bits = [hf] + [(hf & ~int(ann[ok[i]])) | int(cre[ok[i]]) for i in pick]
    return np.array(bits, dtype=np.uint32)


def sparse_state(dim: int, d_alpha: int, n_random: int = 64, seed: int = 21):
    """Sparse sector vector as (sorted indices, values), norm 1: the 16
    lowest alpha ranks with the lowest beta string, the 16 lowest beta ranks
    with the lowest alpha string (Hartree-Fock and the strings next to it in
    colex order), and n_random uniform indices; N(0,1) values."""
    rng = np.random.default_rng(seed)
    near = [i for i in range(min(16, d_alpha))] + [j * d_alpha for j in range(1, min(16, dim // d_alpha))]
    idx = np.unique(np.concatenate([np.array(near, dtype=np.int64),
                                    rng.choice(dim, size=min(n_random, dim), replace=False).astype(np.int64)]))
    val = rng.standard_normal(idx.size)
    val /= math.sqrt(float(np.dot(val, val)))
    return idx, val


def random_state(dim: int, seed: int = 7, dtype=np.float64) -> np.ndarray:
    """Dense N(0,1) sector vector normalised to 1 (FP64 norm)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(dim)
    v /= math.sqrt(float(np.dot(v, v)))
    return v.astype(dtype)


def sector_dim(n_orb: int, n_alpha: int, n_beta: int) -> int:
    return math.comb(n_orb, n_alpha) * math.comb(n_orb, n_beta)


# ---------------------------------------------------------------------------
# screen network initialisation
# ---------------------------------------------------------------------------

def mlp_init(seed: int, n_feat: int = 32, hidden: int = 256):
    """Seeded initial parameters of the 32-256-256-1 screen network, float32,
    layout W1[256][32], b1, W2[256][256], b2, W3[256], b3: He-uniform weights,
    zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (hidden, n_feat)) * math.sqrt(6.0 / n_feat)
    W2 = rng.uniform(-1, 1, (hidden, hidden)) * math.sqrt(6.0 / hidden)
    W3 = rng.uniform(-1, 1, hidden) * math.sqrt(6.0 / hidden)
    return np.concatenate([W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), W3,
                           np.zeros(1)]).astype(np.float32)


# ---------------------------------------------------------------------------
# workload configurations
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n_orb: int
    n_alpha: int
    n_beta: int
    seed: int = 42
    iterations: int = 0
    note: str = ""

    @property
    def n_qubits(self) -> int:
        return 2 * self.n_orb

    @property
    def dim(self) -> int:
        return sector_dim(self.n_orb, self.n_alpha, self.n_beta)


WORKLOADS = {
    "h4_8q": Workload("h4_8q", 4, 2, 2, 42, 10, "8 qubits, plain FP64, dense-FCI check"),
    "h8_16q": Workload("h8_16q", 8, 4, 4, 42, 30, "16 qubits, first parity run"),
    "h12_24q": Workload("h12_24q", 12, 6, 6, 42, 0, "24 qubits, batching"),
    "h14_28q": Workload("h14_28q", 14, 7, 7, 42, 50, "28 qubits, FP32 study"),
    "h16_32q": Workload("h16_32q", 16, 8, 8, 42, 0, "32 qubits, FP32 + screen"),
}

# eight uneven co-launched instances (orbital counts 8..12, seeds 42+i)
INSTANCES = tuple(
    Workload(f"inst{i}_M{m}", m, (m + 1) // 2, m // 2, 42 + i)
    for i, m in enumerate((8, 9, 10, 10, 11, 11, 12, 12))
)


def hamiltonian(w: Workload):
    """(x, z, c) Pauli list and integrals for a workload."""
    h, g = integrals(w.n_orb, w.seed)
    x, z, c = jw_pauli_list(h, g)
    return x, z, c, h, g
