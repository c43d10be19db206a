"""Pins of the oracle's multi-parameter ansatz gradient, of its ADAPT loop's
first step and of the sparse-support pool-gradient sum (no GPU).

The ansatz is U(theta)|psi_0> = U_j...U_1|HF>, U_i = exp(theta_i A_{k_i}),
newest factor applied last (the state-preparation operator of "General
Framework for Variational Algorithms"); E(theta) = <psi|H|psi> (the energy
equation there).  dE/dtheta_i is pinned against central differences of the
oracle's own energy and against the exact four-point shift rule, which holds
for every parameter because each generator's spectrum lies in {0, +-i}
(A^3 = -A), so E restricted to one coordinate is a trigonometric polynomial
of degree 2.  A planted mistake (the generator inserted one factor too late)
must fail both pins.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle.adapt import DenseSectorProblem, SectorProblem, run_adapt
import synth


def _problem(name, dense=False):
    w = synth.WORKLOADS[name]
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    cls_ = DenseSectorProblem if dense else SectorProblem
    return w, cls_(w.n_orb, w.n_alpha, w.n_beta, x, z, c, cre, ann)


def _ansatz(prob, n_ops, seed):
    rng = np.random.default_rng(seed)
    ops = [int(k) for k in rng.integers(0, len(prob.cre), n_ops)]
    ops[-1] = ops[1]  # a repeated operator is allowed in ADAPT
    th = rng.uniform(-0.6, 0.6, n_ops)
    return ops, th


def _energy(prob, ops, th):
    psi = prob.state(ops, th)
    return float(psi @ prob.hpsi(psi))


def _fd_error(prob, ops, th, h=1e-4):
    """max_i |central difference - analytic dE/dtheta_i|."""
    _, grad = prob.energy_grad(ops, th)
    err = 0.0
    for i in range(len(ops)):
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (_energy(prob, ops, tp) - _energy(prob, ops, tm)) / (2 * h)
        err = max(err, abs(fd - grad[i]))
    return err


def _shift_error(prob, ops, th):
    """max_i |four-point shift rule - analytic dE/dtheta_i| (exact for A^3 = -A)."""
    _, grad = prob.energy_grad(ops, th)
    r = math.sqrt(2.0)
    err = 0.0
    for i in range(len(ops)):
        def E(d):
            t = th.copy()
            t[i] += d
            return _energy(prob, ops, t)
        sh = (E(math.pi / 4) - E(-math.pi / 4)) - (r - 1) / 2 * (E(math.pi / 2) - E(-math.pi / 2))
        err = max(err, abs(sh - grad[i]))
    return err


class _LateInsertion(SectorProblem):
    """Planted mistake: A_i inserted after U_{i+1} instead of after U_i."""

    def energy_grad(self, ops, thetas):
        psi = self.state(ops, thetas)
        sig = self.hpsi(psi)
        E = oracle.dot(psi, sig)
        grad = np.zeros(len(ops))
        for i in range(len(ops)):
            stop = min(i + 2, len(ops))
            v = self.state(ops[:stop], thetas[:stop])
            k = ops[i]
            v = oracle.apply_generator(self.M, self.na, self.nb, self.cre[k], self.ann[k], v)
            for kk, t in zip(ops[stop:], thetas[stop:]):
                v = oracle.rotate(self.M, self.na, self.nb, self.cre[kk], self.ann[kk], t, v)
            grad[i] = 2.0 * oracle.dot(sig, v)
        return E, grad


@pytest.mark.parametrize("name", ["h4_8q", "h8_16q"])
def test_energy_grad_finite_differences(name):
    _, prob = _problem(name)
    ops, th = _ansatz(prob, 5, 21)
    assert _fd_error(prob, ops, th) <= 1e-7


@pytest.mark.parametrize("name", ["h4_8q", "h8_16q"])
def test_energy_grad_shift_rule(name):
    _, prob = _problem(name)
    ops, th = _ansatz(prob, 5, 22)
    assert _shift_error(prob, ops, th) <= 1e-11


@pytest.mark.parametrize("name", ["h4_8q", "h8_16q"])
def test_dense_energy_grad_pins(name):
    """The dense helper used beside the GPU runs, pinned the same way."""
    _, prob = _problem(name, dense=True)
    ops, th = _ansatz(prob, 5, 23)
    assert _fd_error(prob, ops, th) <= 1e-7
    assert _shift_error(prob, ops, th) <= 1e-11


def test_planted_late_insertion_fails_the_pins():
    w, prob = _problem("h4_8q")
    bad = _LateInsertion(w.n_orb, w.n_alpha, w.n_beta, prob.x, prob.z, prob.c, prob.cre, prob.ann)
    ops, th = _ansatz(prob, 5, 21)
    assert _fd_error(prob, ops, th) <= 1e-7
    assert _fd_error(bad, ops, th) > 1e-4
    assert _shift_error(bad, ops, th) > 1e-4


def test_run_adapt_first_step_closed_form():
    """run_adapt's first iteration from HF: exp(theta A)|HF> stays in
    span{HF, D'}, so its optimum is the lower eigenvalue of the 2x2 block."""
    w, prob = _problem("h4_8q")
    log = run_adapt(prob, 1)
    k = log.selected[0]
    basis = brute.sector_basis(w.n_orb, w.n_alpha, w.n_beta)
    Hs = brute.sector_matrix_from_paulis(w.n_orb, w.n_alpha, w.n_beta, prob.x, prob.z, prob.c).real
    s, bp = oracle.apply_tau(int(prob.cre[k]), int(prob.ann[k]), int(basis[0]))
    if not s:
        s, bp = oracle.apply_tau(int(prob.ann[k]), int(prob.cre[k]), int(basis[0]))
    assert s != 0
    j = int(np.searchsorted(basis, bp))
    blk = np.array([[Hs[0, 0], Hs[0, j]], [Hs[j, 0], Hs[j, j]]])
    assert abs(log.energies[0] - np.linalg.eigvalsh(blk)[0]) < 1e-10
    # the selection is the argmax of |2 H[D', HF]| over the pool (tie rule)
    assert abs(abs(log.grads[0][k]) - 2 * abs(Hs[j, 0])) < 1e-12
    assert abs(log.grads[0][k]) >= np.abs(log.grads[0]).max() * (1 - 1e-9)


# ------------------------------------------------- sparse-support pool gradients

def _sparse_state(dim, n_nz, seed):
    rng = np.random.default_rng(seed)
    nz = np.sort(rng.choice(dim, size=min(n_nz, dim), replace=False)).astype(np.int64)
    psi = np.zeros(dim)
    psi[nz] = rng.standard_normal(nz.size)
    psi /= np.linalg.norm(psi)
    return nz, psi


@pytest.mark.parametrize("name,n_nz", [("h4_8q", 5), ("h4_8q", 36), ("h8_16q", 17), ("h8_16q", 400)])
def test_pool_gradients_sparse_equals_full_pair_sum(name, n_nz):
    w = synth.WORKLOADS[name]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, _, _ = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(M)
    nz, psi = _sparse_state(w.dim, n_nz, 5 + n_nz)
    sig = oracle.apply_h(M, na, nb, x, z, c, psi)
    full = oracle.pool_gradients(M, na, nb, cre, ann, psi, sig)
    sp_ = oracle.pool_gradients_sparse(M, na, nb, cre, ann, nz, psi, sig)
    assert np.abs(sp_ - full).max() <= 1e-13 * max(1.0, np.abs(full).max())
    assert np.count_nonzero(full) > 0


def test_pool_gradients_sparse_commutator_and_edges():
    """Against the dense commutator form g = psi^T [H, A] psi with Kronecker
    ladder matrices; the empty support gives 0; a dense psi listed whole
    gives the full pair sum."""
    w = synth.WORKLOADS["h4_8q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(M)
    basis = brute.sector_basis(M, na, nb)
    Hs = brute.sector_matrix(brute.fermion_hamiltonian(h, g), basis).real
    nz, psi = _sparse_state(w.dim, 4, 9)
    sig = Hs @ psi
    got = oracle.pool_gradients_sparse(M, na, nb, cre, ann, nz, psi, sig)
    for k in range(len(cre)):
        A = brute.generator_matrix(int(cre[k]), int(ann[k]), 2 * M).real.toarray()[np.ix_(basis, basis)]
        assert abs(psi @ (Hs @ A - A @ Hs) @ psi - got[k]) < 1e-12
    zero = oracle.pool_gradients_sparse(M, na, nb, cre, ann, np.zeros(0, np.int64), np.zeros(w.dim),
                                        np.zeros(w.dim))
    assert np.all(zero == 0.0)
    dense = synth.random_state(w.dim, 3)
    sd = oracle.apply_h(M, na, nb, x, z, c, dense)
    a = oracle.pool_gradients_sparse(M, na, nb, cre, ann, np.arange(w.dim), dense, sd)
    b = oracle.pool_gradients(M, na, nb, cre, ann, dense, sd)
    assert np.abs(a - b).max() <= 1e-13 * max(1.0, np.abs(b).max())
