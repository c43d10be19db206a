"""Jordan-Wigner Pauli list of the second-quantised molecular Hamiltonian.

TEST INFRASTRUCTURE (see the package docstring): the reference for the
device-side Hamiltonian assembly.  The paper builds H by summing the
contributions of the individual fermionic operators after mapping them to
qubits ("Sparse State-Vector Emulation"); the mapping is Jordan-Wigner with
spin orbital P = p + s M on qubit P (blocked spin order).

Definitions used, written out:
  * Pauli string P(x, z) = prod_q sigma(x_q, z_q), sigma(0,0) = I,
    sigma(1,0) = X, sigma(0,1) = Z, sigma(1,1) = Y.  Since Y = i X Z,
    P(x, z) = i^{|x & z|} X^x Z^z, and the product of two strings is
    P(x1,z1) P(x2,z2) = i^k P(x1^x2, z1^z2) with
    k = |x1&z1| + |x2&z2| + 2|z1&x2| - |(x1^x2)&(z1^z2)|  (mod 4).
  * a_P = Z_0 ... Z_{P-1} (X_P + i Y_P) / 2 and a+_P = Z_0 ... Z_{P-1} (X_P - i Y_P) / 2,
    i.e. a_P = (P(e, m) + i P(e, m|e)) / 2 with e = 2^P, m = 2^P - 1, and
    a+_P = (P(e, m) - i P(e, m|e)) / 2.
  * H = sum_{pq s} h_pq a+_{ps} a_{qs}
      + 1/2 sum_{pqrs, s t} g_pqrs a+_{ps} a+_{rt} a_{st} a_{qs}  (chemist's notation),
    terms with a+_P a+_P or a_Q a_Q (zero operators) omitted.
Every product of ladder operators is expanded into its 2^k Pauli strings with
complex coefficients; equal strings are merged with exactly rounded sums
(math.fsum) of the real and the imaginary parts.  A real H has all imaginary
parts cancel exactly; the function checks that.

Parity: pinned against the dense second-quantised matrix built from explicit
ladder-operator matrices (brute.fermion_hamiltonian) in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import math

import numpy as np

_POPC16 = np.array([bin(i).count("1") for i in range(1 << 16)], dtype=np.int64)


def _popc(a):
    a = np.asarray(a, dtype=np.uint64)
    return (_POPC16[(a & np.uint64(0xFFFF)).astype(np.int64)] + _POPC16[((a >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)]
            + _POPC16[((a >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.int64)]
            + _POPC16[((a >> np.uint64(48)) & np.uint64(0xFFFF)).astype(np.int64)])


_IPOW = np.array([1.0 + 0j, 1j, -1.0 + 0j, -1j])


def _expand(positions, coeff):
    """sum_i coeff[i] * prod_k L_k(i) for ladder operators given per position
    k as (qubit array, dagger flag), left to right.  Returns the unmerged
    (x, z, complex c) of all 2^k Pauli strings per term."""
    n = coeff.shape[0]
    xs, zs, cs = [], [], []
    for choice in range(1 << len(positions)):
        x = np.zeros(n, dtype=np.uint64)
        z = np.zeros(n, dtype=np.uint64)
        c = coeff.astype(complex)
        for k, (q, dag) in enumerate(positions):
            e = np.left_shift(np.uint64(1), q.astype(np.uint64))
            m = e - np.uint64(1)
            if (choice >> k) & 1:   # the Y part: +-(i/2) P(e, m|e)
                x2, z2, f = e, m | e, (-0.5j if dag else 0.5j)
            else:                   # the X part: (1/2) P(e, m)
                x2, z2, f = e, m, 0.5
            kexp = (_popc(x & z) + _popc(x2 & z2) + 2 * _popc(z & x2) - _popc((x ^ x2) & (z ^ z2))) % 4
            c = c * f * _IPOW[kexp]
            x = x ^ x2
            z = z ^ z2
        xs.append(x)
        zs.append(z)
        cs.append(c)
    return np.concatenate(xs), np.concatenate(zs), np.concatenate(cs)


def jw_pauli_list(h: np.ndarray, g: np.ndarray, e_core: float = 0.0):
    """(x, z, c): H = e_core + the one- and two-body operator as sum_t c_t P(x_t, z_t),
    sorted by (x, z), exact zeros dropped; uint32 masks, FP64 coefficients."""
    M = h.shape[0]
    if 2 * M > 32:
        raise ValueError("at most 32 qubits")
    parts = []
    p, q, s = (a.ravel() for a in np.meshgrid(np.arange(M), np.arange(M), np.arange(2), indexing="ij"))
    c1 = h[p, q].astype(float)
    keep = c1 != 0.0
    parts.append(_expand([((p + s * M)[keep], True), ((q + s * M)[keep], False)], c1[keep]))
    p, q, r, u, s, t = np.indices((M, M, M, M, 2, 2)).reshape(6, -1)
    c2 = 0.5 * g[p, q, r, u]
    P, Q, R, U = p + s * M, q + s * M, r + t * M, u + t * M
    keep = (c2 != 0.0) & (P != R) & (Q != U)
    parts.append(_expand([(P[keep], True), (R[keep], True), (U[keep], False), (Q[keep], False)], c2[keep]))
    x = np.concatenate([a[0] for a in parts])
    z = np.concatenate([a[1] for a in parts])
    c = np.concatenate([a[2] for a in parts])
    if e_core != 0.0:
        x = np.concatenate([x, np.zeros(1, np.uint64)])
        z = np.concatenate([z, np.zeros(1, np.uint64)])
        c = np.concatenate([c, np.array([complex(e_core)])])
    key = (x << np.uint64(32)) | z
    order = np.argsort(key, kind="stable")
    key, c = key[order], c[order]
    uniq, start = np.unique(key, return_index=True)
    bounds = list(start) + [key.size]
    re, im = c.real.tolist(), c.imag.tolist()
    cr = np.array([math.fsum(re[bounds[i]:bounds[i + 1]]) for i in range(uniq.size)])
    ci = np.array([math.fsum(im[bounds[i]:bounds[i + 1]]) for i in range(uniq.size)])
    if np.any(ci != 0.0):
        raise ArithmeticError("imaginary Pauli coefficient: the integrals do not define a real Hamiltonian")
    keep = cr != 0.0
    return ((uniq[keep] >> np.uint64(32)).astype(np.uint32), (uniq[keep] & np.uint64(0xFFFFFFFF)).astype(np.uint32),
            cr[keep])
