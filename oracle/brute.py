"""Dense brute force over the full 2^n Fock space (small n only).

TEST INFRASTRUCTURE.  Independent constructions used to pin the sector
oracle and the Pauli-string inputs:

* ladder operators built two ways: from the Jordan-Wigner sign rule on basis
  states, and as Kronecker products Z x ... x Z x sigma^- x I x ... x I;
* the second-quantised molecular Hamiltonian (paper, "General Framework for
  Variational Algorithms": a real H in R^{2^n x 2^n}) from explicit ladder
  matrix products;
* Pauli strings as Kronecker products of 2x2 Pauli matrices;
* the symmetry-restricted basis Omega_CIk by enumerating all 2^n bitstrings
  ("Sparse State-Vector Emulation", Table 1) and FCI by dense
  diagonalisation.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

I2 = np.eye(2, dtype=complex)
X2 = np.array([[0, 1], [1, 0]], dtype=complex)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z2 = np.array([[1, 0], [0, -1]], dtype=complex)
SM = np.array([[0, 1], [0, 0]], dtype=complex)  # |0><1| : annihilates |1> = occupied


def _kron_list(mats):
    """kron(mats[n-1], ..., mats[0]): mats[q] acts on qubit q (bit q of b)."""
    out = sp.csr_matrix(np.ones((1, 1), dtype=complex))
    for m in reversed(mats):
        out = sp.kron(out, sp.csr_matrix(m), format="csr")
    return out


def ladder_kron(q: int, n: int, dagger: bool = False):
    """a_q = (prod_{q'<q} Z_q') sigma^-_q, as a Kronecker product."""
    mats = [Z2] * q + [SM.T.conj() if dagger else SM] + [I2] * (n - q - 1)
    return _kron_list(mats)


def ladder_sign(q: int, n: int, dagger: bool = False):
    """a_q from its action on basis states:
    a_q|b> = (-1)^{#occupied modes below q} |b - e_q>  if bit q is set."""
    N = 1 << n
    rows, cols, vals = [], [], []
    for b in range(N):
        occ = (b >> q) & 1
        if occ == (0 if dagger else 1):
            sgn = -1.0 if bin(b & ((1 << q) - 1)).count("1") % 2 else 1.0
            rows.append(b ^ (1 << q))
            cols.append(b)
            vals.append(sgn)
    return sp.csr_matrix((np.array(vals, dtype=complex), (rows, cols)), shape=(N, N))


def fermion_hamiltonian(h: np.ndarray, g: np.ndarray):
    """H = sum h_pq a+_{ps} a_{qs} + 1/2 sum g_pqrs a+_{ps} a+_{rt} a_{st} a_{qs}
    (chemist's notation, blocked spin order), as a sparse 2^n matrix."""
    M = h.shape[0]
    n = 2 * M
    a = [ladder_sign(q, n) for q in range(n)]
    ad = [ladder_sign(q, n, True) for q in range(n)]
    N = 1 << n
    H = sp.csr_matrix((N, N), dtype=complex)
    for s in range(2):
        for p in range(M):
            for q in range(M):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * (ad[p + s * M] @ a[q + s * M])
    for s in range(2):
        for t in range(2):
            for p in range(M):
                for r in range(M):
                    P, R = p + s * M, r + t * M
                    if P == R:
                        continue
                    pr = ad[P] @ ad[R]
                    for q in range(M):
                        for u in range(M):
                            Q, U = q + s * M, u + t * M
                            if Q == U or g[p, q, r, u] == 0.0:
                                continue
                            H = H + (0.5 * g[p, q, r, u]) * (pr @ a[U] @ a[Q])
    return H


def pauli_kron(x: int, z: int, n: int):
    mats = []
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        mats.append(Y2 if (xb and zb) else X2 if xb else Z2 if zb else I2)
    return _kron_list(mats)


def pauli_sum(x, z, c, n):
    N = 1 << n
    H = sp.csr_matrix((N, N), dtype=complex)
    for xi, zi, ci in zip(x, z, c):
        H = H + complex(ci) * pauli_kron(int(xi), int(zi), n)
    return H


def number_op(n: int, qubits):
    N = 1 << n
    d = np.zeros(N)
    for b in range(N):
        d[b] = sum((b >> q) & 1 for q in qubits)
    return sp.diags(d.astype(complex))


def sector_basis(M: int, na: int, nb: int):
    """All bitstrings with popcount(alpha) = na, popcount(beta) = nb, in
    ascending numeric order (the enumeration that the rank must reproduce)."""
    n = 2 * M
    am = (1 << M) - 1
    return np.array([b for b in range(1 << n)
                     if bin(b & am).count("1") == na and bin(b >> M).count("1") == nb],
                    dtype=np.int64)


def sector_matrix(Hfull, basis):
    """Dense P_S H P_S restricted to the sector basis."""
    return Hfull[basis][:, basis].toarray()


def fci(Hsec):
    """Lowest eigenvalue of the real symmetric sector matrix."""
    return float(np.linalg.eigvalsh(np.real(Hsec))[0])


def generator_matrix(cre: int, ann: int, n: int):
    """A = tau - tau^dagger, tau = a+_{c1} a+_{c2} a_{a2} a_{a1} (c1<c2, a1<a2)
    or a+_c a_a, from Kronecker-product ladder operators."""
    cq = [q for q in range(n) if (cre >> q) & 1]
    aq = [q for q in range(n) if (ann >> q) & 1]
    if len(cq) == 1:
        tau = ladder_kron(cq[0], n, True) @ ladder_kron(aq[0], n)
    else:
        tau = (ladder_kron(cq[0], n, True) @ ladder_kron(cq[1], n, True)
               @ ladder_kron(aq[1], n) @ ladder_kron(aq[0], n))
    return tau - tau.conj().T


def qubit_generator_matrix(cre: int, ann: int, n: int):
    """A = tau - tau^dagger for a qubit excitation (the QEB pool):
    tau = prod_c sigma^+_c prod_a sigma^-_a with no Jordan-Wigner strings,
    sigma^- = |0><1| on the qubit (empties an occupied orbital)."""
    mats = []
    for q in range(n):
        if (cre >> q) & 1:
            mats.append(SM.T.copy())
        elif (ann >> q) & 1:
            mats.append(SM)
        else:
            mats.append(I2)
    tau = _kron_list(mats)
    return tau - tau.conj().T


# ---------------------------------------------------------------------------
# sector-level twins (NumPy, vectorised over determinants)
# ---------------------------------------------------------------------------

def _popc(a):
    a = np.asarray(a, dtype=np.int64)
    c = np.zeros(a.shape, dtype=np.int64)
    for q in range(40):
        c += (a >> q) & 1
    return c


def _colex_rank(s, k):
    """colex rank sum_i C(o_i, i) of k-subsets given as integer masks."""
    from math import comb
    s = np.asarray(s, dtype=np.int64)
    r = np.zeros(s.shape, dtype=np.int64)
    i = np.zeros(s.shape, dtype=np.int64)
    for o in range(32):
        bit = (s >> o) & 1
        i = i + bit
        r = r + bit * np.array([comb(o, int(v)) for v in range(k + 2)])[np.minimum(i, k + 1)]
    return r


def sector_index(M, na, nb, bits):
    """idx = rank(beta) * C(M, na) + rank(alpha), vectorised."""
    from math import comb
    bits = np.asarray(bits, dtype=np.int64)
    am = (1 << M) - 1
    return _colex_rank(bits >> M, nb) * comb(M, na) + _colex_rank(bits & am, na)


def sector_matrix_from_paulis(M, na, nb, x, z, c):
    """Dense P_S H P_S from a Pauli list: for each term, every sector
    determinant d couples to b = d xor x with <d|P|b> = i^{n_Y} (-1)^{popc(z&b)}."""
    basis = sector_basis(M, na, nb)
    dim = basis.size
    am = (1 << M) - 1
    H = np.zeros((dim, dim), dtype=complex)
    for xi, zi, ci in zip(x.tolist(), z.tolist(), c.tolist()):
        b = basis ^ xi
        ok = (_popc(b & am) == na) & (_popc(b >> M) == nb)
        ny = bin(xi & zi).count("1")
        ph = (1j ** ny) * (1 - 2 * (_popc(zi & b[ok]) & 1))
        cols = np.searchsorted(basis, b[ok])
        np.add.at(H, (np.nonzero(ok)[0], cols), ci * ph)
    return H


def sigma_second_quantised(M, na, nb, h, g, psi):
    """sigma = H psi applying every one- and two-body fermionic term directly
    to the determinants (ladder-operator signs), with no Pauli strings."""
    basis = sector_basis(M, na, nb)
    sig = np.zeros(psi.shape, dtype=np.float64)

    def lad(bits, amp, q, dag):
        occ = (bits >> q) & 1
        ok = occ == (0 if dag else 1)
        sg = 1 - 2 * (_popc(bits & ((1 << q) - 1)) & 1)
        return (bits ^ (1 << q))[ok], (amp * sg)[ok]

    def add(bits, amp):
        if bits.size:
            np.add.at(sig, np.searchsorted(basis, bits), amp)

    for s in range(2):
        for p in range(M):
            for q in range(M):
                if h[p, q] == 0.0:
                    continue
                b, a = lad(basis, psi, q + s * M, False)
                b, a = lad(b, a, p + s * M, True)
                add(b, h[p, q] * a)
    for s in range(2):
        for t in range(2):
            for q in range(M):
                b1, a1 = lad(basis, psi, q + s * M, False)
                for u in range(M):
                    if u + t * M == q + s * M:
                        continue
                    b2, a2 = lad(b1, a1, u + t * M, False)
                    for r in range(M):
                        if b2.size == 0:
                            break
                        b3, a3 = lad(b2, a2, r + t * M, True)
                        for p in range(M):
                            if p + s * M == r + t * M or g[p, q, r, u] == 0.0:
                                continue
                            b4, a4 = lad(b3, a3, p + s * M, True)
                            add(b4, 0.5 * g[p, q, r, u] * a4)
    return sig


def hf_energy_slater_condon(h, g, na, nb):
    """E_HF = sum_{i s} h_ii + 1/2 sum_{i s, j t} [(ii|jj) - delta_st (ij|ji)]
    over the occupied spin-orbitals of the lowest-index determinant."""
    occ = [(i, 0) for i in range(na)] + [(i, 1) for i in range(nb)]
    e = sum(h[i, i] for i, _ in occ)
    for i, s in occ:
        for j, t in occ:
            e += 0.5 * g[i, i, j, j]
            if s == t:
                e -= 0.5 * g[i, j, j, i]
    return e
