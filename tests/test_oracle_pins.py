"""Pins of the CPU oracle (and of the shared synthetic inputs) against values
fixed by the paper and by the mathematics: Table 1 dimensions, brute-force
enumeration, independent operator constructions, closed forms, invariants."""
import math
import os

import numpy as np
import scipy.sparse as sp
import pytest
import scipy.linalg as sla

import oracle
from oracle import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- Table 1

def test_table1_sector_dims():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_sector_dims.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for name, ne, nq, nci, ncik in rows:
        ne, nq, nci, ncik = int(ne), int(nq), int(nci), int(ncik)
        M = nq // 2
        assert math.comb(nq, ne) == nci
        assert oracle.sector_dim(M, ne // 2, ne // 2) == ncik
        assert oracle.binom(M, ne // 2) ** 2 == ncik


# ----------------------------------------------------------------- ranking

@pytest.mark.parametrize("M,na,nb", [(3, 1, 2), (4, 2, 2), (5, 3, 2), (6, 3, 3), (6, 1, 4), (7, 4, 3)])
def test_rank_is_sorted_enumeration(M, na, nb):
    basis = brute.sector_basis(M, na, nb)
    assert basis.size == oracle.sector_dim(M, na, nb)
    idx = oracle.rank(M, na, nb, basis)
    assert np.array_equal(idx, np.arange(basis.size))
    back = oracle.unrank(M, na, nb, np.arange(basis.size))
    assert np.array_equal(back.astype(np.int64), basis)
    assert np.array_equal(brute.sector_index(M, na, nb, basis), np.arange(basis.size))


def test_rank_out_of_sector_and_large():
    assert oracle.rank(4, 2, 2, np.array([0b0111_0011]))[0] == -1
    rng = np.random.default_rng(0)
    dim = oracle.sector_dim(16, 8, 8)
    idx = rng.integers(0, dim, 4096)
    bits = oracle.unrank(16, 8, 8, idx)
    assert np.all([bin(int(b) & 0xFFFF).count("1") == 8 and bin(int(b) >> 16).count("1") == 8
                   for b in bits])
    assert np.array_equal(oracle.rank(16, 8, 8, bits), idx)
    # ascending index <=> ascending bitstring
    o = np.argsort(idx)
    assert np.all(np.diff(bits[o].astype(np.int64)) > 0)


# ------------------------------------------------- ladder operators / JW

def test_ladder_sign_equals_kron_and_car():
    n = 5
    for q in range(n):
        for dag in (False, True):
            d = brute.ladder_sign(q, n, dag) - brute.ladder_kron(q, n, dag)
            assert abs(d).max() == 0
    a = [brute.ladder_sign(q, n) for q in range(n)]
    for p in range(n):
        for q in range(n):
            ac = a[p] @ a[q].conj().T + a[q].conj().T @ a[p]
            exp = np.eye(1 << n) if p == q else np.zeros((1 << n, 1 << n))
            assert np.allclose(ac.toarray(), exp)
            assert abs(a[p] @ a[q] + a[q] @ a[p]).max() == 0


def test_pauli_algebra():
    rng = np.random.default_rng(1)
    n = 5
    for _ in range(20):
        x, z = (int(v) for v in rng.integers(0, 1 << n, 2))
        P = brute.pauli_kron(x, z, n)
        assert np.allclose((P @ P).toarray(), np.eye(1 << n))
        x2, z2 = (int(v) for v in rng.integers(0, 1 << n, 2))
        Q = brute.pauli_kron(x2, z2, n)
        # commute iff symplectic product is even
        sym = bin(x & z2).count("1") + bin(z & x2).count("1")
        comm = (P @ Q - (1 if sym % 2 == 0 else -1) * (Q @ P))
        assert abs(comm).max() < 1e-14


@pytest.mark.parametrize("M", [2, 3, 4])
def test_pauli_list_equals_fermionic_hamiltonian(M):
    h, g = synth.integrals(M, 42 + M)
    x, z, c = synth.jw_pauli_list(h, g)
    n = 2 * M
    Hf = brute.fermion_hamiltonian(h, g)
    Hp = brute.pauli_sum(x, z, c, n)
    assert abs(Hf - Hp).max() < 1e-13
    # real symmetric
    assert abs(Hf.imag).max() == 0 and abs(Hf - Hf.T).max() < 1e-13


@pytest.mark.parametrize("M", [1, 2, 3])
def test_oracle_jw_equals_fermionic_hamiltonian(M):
    """The oracle's own Jordan-Wigner expansion (complex Pauli algebra) gives
    the dense second-quantised matrix built from explicit ladder matrices,
    including the constant."""
    from oracle import jw
    h, g = synth.integrals(M, 77 + M)
    x, z, c = jw.jw_pauli_list(h, g, e_core=-0.75)
    n = 2 * M
    Hf = brute.fermion_hamiltonian(h, g) + (-0.75) * sp.identity(1 << n)
    Hp = brute.pauli_sum(x, z, c, n)
    assert abs(Hf - Hp).max() < 1e-13


def test_oracle_jw_nonreal_and_trivial():
    from oracle import jw
    h, g = synth.integrals(2, 3)
    h2 = h.copy()
    h2[0, 1] += 0.25  # h not symmetric: imaginary strings survive
    with pytest.raises(ArithmeticError):
        jw.jw_pauli_list(h2, g)
    x, z, c = jw.jw_pauli_list(np.zeros((2, 2)), np.zeros((2, 2, 2, 2)), e_core=1.5)
    assert list(x) == [0] and list(z) == [0] and list(c) == [1.5]


@pytest.mark.parametrize("M", [3, 4, 5, 6, 8, 12])
def test_pauli_term_count_closed_form(M):
    h, g = synth.integrals(M, 42)
    x, z, c = synth.jw_pauli_list(h, g)
    n = 2 * M
    T = (1 + n + math.comb(n, 2)) + 2 * math.comb(M, 2) * 2 * (n - 1) \
        + 12 * math.comb(M, 4) + 4 * math.comb(M, 2) ** 2
    assert len(c) == T
    assert np.all(np.array([bin(int(a) & int(b)).count("1") % 2 for a, b in zip(x, z)]) == 0)


def test_integrals_symmetry():
    h, g = synth.integrals(6, 42)
    assert np.array_equal(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(g, g.transpose(perm))
    sup = g.reshape(36, 36)
    assert np.linalg.eigvalsh(sup).min() > -1e-12
    h2, g2 = synth.integrals(6, 42)
    assert np.array_equal(h, h2) and np.array_equal(g, g2)


def test_number_and_sz_conservation():
    M = 3
    h, g = synth.integrals(M, 5)
    x, z, c = synth.jw_pauli_list(h, g)
    n = 2 * M
    H = brute.pauli_sum(x, z, c, n)
    Na = brute.number_op(n, range(M))
    Nb = brute.number_op(n, range(M, n))
    assert abs(H @ Na - Na @ H).max() < 1e-12
    assert abs(H @ Nb - Nb @ H).max() < 1e-12


# ---------------------------------------------------------------- H psi

def test_single_pauli_phase_formula():
    """sigma = P_S P P_S psi for single (even n_Y) Pauli strings, including
    ones that do not conserve particle number, against Kronecker matrices."""
    M, na, nb = 3, 1, 2
    n = 2 * M
    basis = brute.sector_basis(M, na, nb)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(basis.size)
    tested = 0
    for _ in range(200):
        x, z = (int(v) for v in rng.integers(0, 1 << n, 2))
        if bin(x & z).count("1") % 2:
            continue
        P = brute.pauli_kron(x, z, n)[basis][:, basis].toarray()
        assert abs(P.imag).max() == 0
        s = oracle.apply_h(M, na, nb, np.array([x]), np.array([z]), np.array([0.7]), psi)
        assert np.allclose(s, 0.7 * P.real @ psi, atol=1e-14)
        tested += 1
    assert tested > 50
    with pytest.raises(ValueError):
        oracle.apply_h(M, na, nb, np.array([1]), np.array([1]), np.array([1.0]), psi)


@pytest.mark.parametrize("M,na,nb", [(3, 2, 1), (4, 2, 2), (4, 3, 1), (5, 2, 3)])
def test_apply_h_equals_dense_fermionic(M, na, nb):
    h, g = synth.integrals(M, 11)
    x, z, c = synth.jw_pauli_list(h, g)
    basis = brute.sector_basis(M, na, nb)
    Hs = brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis).real
    psi = synth.random_state(basis.size, 9)
    s = oracle.apply_h(M, na, nb, x, z, c, psi)
    ref = Hs @ psi
    assert np.linalg.norm(s - ref) / np.linalg.norm(ref) < 1e-12
    Hp = brute.sector_matrix_from_paulis(M, na, nb, x, z, c)
    assert abs(Hp - Hs).max() < 1e-12


def test_apply_h_16q_second_quantised_route():
    w = synth.WORKLOADS["h8_16q"]
    x, z, c, h, g = synth.hamiltonian(w)
    psi = synth.random_state(w.dim, 7)
    s = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi)
    ref = brute.sigma_second_quantised(w.n_orb, w.n_alpha, w.n_beta, h, g, psi)
    assert np.linalg.norm(s - ref) / np.linalg.norm(ref) < 1e-12
    # Hermiticity on the sector: <phi|H psi> = <H phi|psi>
    phi = synth.random_state(w.dim, 8)
    sp_ = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, phi)
    assert abs(oracle.dot(phi, s) - oracle.dot(sp_, psi)) < 1e-13 * abs(oracle.dot(phi, s)) + 1e-14


def test_sampled_rows_match_full():
    w = synth.WORKLOADS["h8_16q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    psi = synth.random_state(w.dim, 7)
    full = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi)
    idx = np.array([0, 5, 77, 4899, 1234])
    part = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi, out_idx=idx)
    assert np.array_equal(part, full[idx])


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 2, 3)])
def test_apply_h_sparse_input_equals_dense_fermionic(M, na, nb):
    """The input-side (push) sum for a sparse psi against the dense
    second-quantised sector matrix, and empty / single-state inputs."""
    h, g = synth.integrals(M, 12)
    x, z, c = synth.jw_pauli_list(h, g)
    basis = brute.sector_basis(M, na, nb)
    Hs = brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis).real
    rng = np.random.default_rng(3)
    idx = rng.choice(basis.size, 4, replace=False)
    val = rng.standard_normal(4)
    psi = np.zeros(basis.size)
    psi[idx] = val
    s = oracle.apply_h_sparse(M, na, nb, x, z, c, idx, val)
    assert np.abs(s - Hs @ psi).max() < 1e-12 * np.abs(Hs @ psi).max()
    assert np.array_equal(oracle.apply_h_sparse(M, na, nb, x, z, c, idx[:0], val[:0]), np.zeros(basis.size))
    one = oracle.apply_h_sparse(M, na, nb, x, z, c, idx[:1], np.ones(1))
    assert np.abs(one - Hs[:, idx[0]]).max() < 1e-12
    with pytest.raises(ValueError):
        oracle.apply_h_sparse(M, na, nb, np.array([1]), np.array([1]), np.array([1.0]), idx, val)


# ---------------------------------------------------------------- energy

@pytest.mark.parametrize("name", ["h4_8q", "h8_16q", "h12_24q", "h14_28q", "h16_32q"])
def test_hf_energy_slater_condon(name):
    w = synth.WORKLOADS[name]
    x, z, c, h, g = synth.hamiltonian(w)
    bits_hf = synth.hf_bits(w.n_orb, w.n_alpha, w.n_beta)
    assert oracle.rank(w.n_orb, w.n_alpha, w.n_beta, np.array([bits_hf]))[0] == 0
    # diagonal element via the Pauli list: terms with x = 0
    diag = c[x == 0]
    zd = z[x == 0]
    ph = np.array([1 - 2 * (bin(int(zz) & bits_hf).count("1") & 1) for zz in zd])
    e_pauli = math.fsum((diag * ph).tolist())
    e_sc = brute.hf_energy_slater_condon(h, g, w.n_alpha, w.n_beta)
    assert abs(e_pauli - e_sc) < 1e-10
    if w.dim <= 5_000:
        psi = np.zeros(w.dim)
        psi[0] = 1.0
        assert abs(oracle.energy(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi) - e_sc) < 1e-10
    elif w.dim <= 20_000_000:
        psi = np.zeros(w.dim)
        psi[0] = 1.0
        s0 = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi, out_idx=np.array([0]))
        assert abs(s0[0] - e_sc) < 1e-10


def test_fci_and_variational_bound():
    w = synth.WORKLOADS["h4_8q"]
    x, z, c, h, g = synth.hamiltonian(w)
    basis = brute.sector_basis(w.n_orb, w.n_alpha, w.n_beta)
    Hs = brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis).real
    efci = brute.fci(Hs)
    rng = np.random.default_rng(0)
    for _ in range(20):
        psi = rng.standard_normal(w.dim)
        assert oracle.energy(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi) >= efci - 1e-12
    evals, evecs = np.linalg.eigh(Hs)
    assert abs(oracle.energy(w.n_orb, w.n_alpha, w.n_beta, x, z, c, evecs[:, 0]) - efci) < 1e-12


# ---------------------------------------------------------------- pool

@pytest.mark.parametrize("M,count", [(4, 90), (8, 2044), (12, 11814), (14, 22750), (16, 39960)])
def test_pool_counts(M, count):
    assert synth.pool_size(M) == count
    if M <= 12:
        cre, ann, cls = synth.canonical_pool(M)
        assert len(cre) == count
        assert np.all(ann < cre) and np.all((cre & ann) == 0)
        assert len(set(zip(cre.tolist(), ann.tolist()))) == count


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 3, 2), (8, 4, 4)])
def test_pair_count_identity(M, na, nb):
    """sum_k |P_k| = (nnz_struct - dim)/2, nnz per row = 1 + s_a + s_b + d_a + d_b + s_a s_b."""
    cre, ann, _ = synth.canonical_pool(M)
    tot = sum(oracle.pair_count(M, na, nb, a, b) for a, b in zip(cre, ann))
    sa, sb = na * (M - na), nb * (M - nb)
    da = math.comb(na, 2) * math.comb(M - na, 2)
    db = math.comb(nb, 2) * math.comb(M - nb, 2)
    dim = oracle.sector_dim(M, na, nb)
    nnz = dim * (1 + sa + sb + da + db + sa * sb)
    assert tot == (nnz - dim) // 2


def test_tau_matches_ladder_products():
    M = 3
    n = 2 * M
    cre, ann, _ = synth.canonical_pool(M)
    for cr, an in zip(cre.tolist(), ann.tolist()):
        A = brute.generator_matrix(cr, an, n).real.toarray()
        for b in range(1 << n):
            s, bp = oracle.apply_tau(cr, an, b)
            if s:
                assert A[bp, b] == s and A[b, bp] == -s


# ---------------------------------------------------------------- rotations

def test_rotation_equals_expm():
    M, na, nb = 3, 2, 1
    n = 2 * M
    basis = brute.sector_basis(M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    psi = synth.random_state(basis.size, 4)
    full = np.zeros(1 << n)
    full[basis] = psi
    for k in range(len(cre)):
        A = brute.generator_matrix(int(cre[k]), int(ann[k]), n).real.toarray()
        th = 0.3 + 0.1 * k
        ref = sla.expm(th * A) @ full
        out = oracle.rotate(M, na, nb, cre[k], ann[k], th, psi)
        assert np.abs(out - ref[basis]).max() < 1e-14
        assert np.abs(np.delete(ref, basis)).max() < 1e-14
        assert abs(np.linalg.norm(out) - 1.0) < 1e-14
        back = oracle.rotate(M, na, nb, cre[k], ann[k], -th, out)
        assert np.abs(back - psi).max() < 1e-14
        two = oracle.rotate(M, na, nb, cre[k], ann[k], 0.2, oracle.rotate(M, na, nb, cre[k], ann[k], 0.5, psi))
        assert np.abs(two - oracle.rotate(M, na, nb, cre[k], ann[k], 0.7, psi)).max() < 1e-14
        gen = oracle.apply_generator(M, na, nb, cre[k], ann[k], psi)
        assert np.abs(gen - (A @ full)[basis]).max() < 1e-14


# ---------------------------------------------------------------- gradients

def test_gradients_finite_difference_and_shift_rule():
    w = synth.WORKLOADS["h4_8q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(M)
    psi = synth.random_state(w.dim, 12)
    sig = oracle.apply_h(M, na, nb, x, z, c, psi)
    grad = oracle.pool_gradients(M, na, nb, cre, ann, psi, sig)

    def E(k, th):
        v = oracle.rotate(M, na, nb, cre[k], ann[k], th, psi)
        return oracle.dot(v, oracle.apply_h(M, na, nb, x, z, c, v))

    r = math.sqrt(2.0)
    for k in range(len(cre)):
        fd = (E(k, 1e-4) - E(k, -1e-4)) / 2e-4
        assert abs(fd - grad[k]) < 1e-7
        shift = (E(k, math.pi / 4) - E(k, -math.pi / 4)) - (r - 1) / 2 * (E(k, math.pi / 2) - E(k, -math.pi / 2))
        assert abs(shift - grad[k]) < 1e-11
    # dense commutator form g = psi^T [H, A] psi
    basis = brute.sector_basis(M, na, nb)
    Hs = brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis).real
    for k in range(0, len(cre), 7):
        A = brute.generator_matrix(int(cre[k]), int(ann[k]), 2 * M).real.toarray()[np.ix_(basis, basis)]
        assert abs(psi @ (Hs @ A - A @ Hs) @ psi - grad[k]) < 1e-12


def test_gradient_at_hf_is_slater_condon_element():
    w = synth.WORKLOADS["h4_8q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(M)
    basis = brute.sector_basis(M, na, nb)
    Hs = brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis).real
    psi = np.zeros(w.dim)
    psi[0] = 1.0
    sig = oracle.apply_h(M, na, nb, x, z, c, psi)
    grad = oracle.pool_gradients(M, na, nb, cre, ann, psi, sig)
    hf = int(basis[0])
    for k in range(len(cre)):
        s, bp = oracle.apply_tau(int(cre[k]), int(ann[k]), hf)
        s2, bp2 = oracle.apply_tau(int(ann[k]), int(cre[k]), hf)
        if s:
            j = int(np.searchsorted(basis, bp))
            assert abs(grad[k] - 2 * s * Hs[j, 0]) < 1e-12
        elif s2:  # A = tau - tau^dag acts on HF through -tau^dag
            j = int(np.searchsorted(basis, bp2))
            assert abs(grad[k] + 2 * s2 * Hs[j, 0]) < 1e-12
        else:
            assert grad[k] == 0.0


def test_dense_sector_problem_equals_plain():
    """The dense/sparse ADAPT helper equals the term-by-term oracle."""
    from oracle.adapt import DenseSectorProblem, SectorProblem, run_adapt
    w = synth.WORKLOADS["h4_8q"]
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    p1 = SectorProblem(w.n_orb, w.n_alpha, w.n_beta, x, z, c, cre, ann)
    p2 = DenseSectorProblem(w.n_orb, w.n_alpha, w.n_beta, x, z, c, cre, ann)
    ops, th = [5, 80, 3], np.array([0.1, -0.2, 0.3])
    e1, g1 = p1.energy_grad(ops, th)
    e2, g2 = p2.energy_grad(ops, th)
    assert abs(e1 - e2) < 1e-13 and np.abs(g1 - g2).max() < 1e-13
    psi = p1.state(ops, th)
    sig = p1.hpsi(psi)
    ref = oracle.pool_gradients(w.n_orb, w.n_alpha, w.n_beta, cre, ann, psi, sig)
    assert np.abs(p2.gradients(psi, sig) - ref).max() < 1e-13
    l1, l2 = run_adapt(p1, 4), run_adapt(p2, 4)
    assert l1.selected == l2.selected
    assert np.abs(np.array(l1.energies) - np.array(l2.energies)).max() < 1e-10
    # ADAPT energies: non-increasing, above FCI
    basis = brute.sector_basis(w.n_orb, w.n_alpha, w.n_beta)
    efci = brute.fci(brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis))
    assert np.all(np.diff(l2.energies) <= 1e-12) and min(l2.energies) >= efci - 1e-10


@pytest.mark.parametrize("M,na,nb", [(3, 1, 2), (4, 2, 2)])
def test_qubit_excitations_equal_kron_matrices(M, na, nb):
    """Qubit-excitation (QEB) generators of the oracle, pair by pair, equal the
    sector block of the Kronecker-product matrix prod sigma^+ prod sigma^- -
    h.c.; the fermionic generators differ from them only in signs."""
    n = 2 * M
    basis = brute.sector_basis(M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    rng = np.random.default_rng(M)
    pick = rng.choice(cre.size, size=min(24, cre.size), replace=False)
    dim = len(basis)
    for k in pick:
        Aq = brute.sector_matrix(brute.qubit_generator_matrix(int(cre[k]), int(ann[k]), n), basis).real
        Af = brute.sector_matrix(brute.generator_matrix(int(cre[k]), int(ann[k]), n), basis).real
        with oracle.qubit_excitations():
            cols = np.stack([oracle.apply_generator(M, na, nb, cre[k], ann[k], np.eye(dim)[j]) for j in range(dim)], 1)
        assert np.array_equal(cols, Aq), k
        assert np.array_equal(np.abs(Aq), np.abs(Af)), k
    # the context restores the fermionic kind
    e = np.eye(dim)[0]
    k = int(pick[0])
    assert np.array_equal(oracle.apply_generator(M, na, nb, cre[k], ann[k], e),
                          brute.sector_matrix(brute.generator_matrix(int(cre[k]), int(ann[k]), n), basis).real[:, 0])


def test_qubit_single_pauli_form():
    """A QEB single on qubits (a, c) is (i/2)(X_a Y_c - Y_a X_c) up to the
    orientation sign of the generator (the textbook form of the qubit single
    excitation, a real antisymmetric matrix): checked densely on four qubits."""
    n = 4
    for a, c in [(0, 1), (0, 3), (1, 2)]:
        A = brute.qubit_generator_matrix(1 << c, 1 << a, n).toarray()
        x = (1 << a) | (1 << c)
        P1 = brute.pauli_kron(x, 1 << c, n).toarray()  # X_a Y_c
        P2 = brute.pauli_kron(x, 1 << a, n).toarray()  # Y_a X_c
        B = 0.5j * (P1 - P2)
        assert np.allclose(A, B, atol=1e-15) or np.allclose(A, -B, atol=1e-15)
        assert np.allclose(A, -A.T.conj())
