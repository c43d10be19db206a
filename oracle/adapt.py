"""ADAPT-VQE reference loop on the plain sector oracle.

TEST INFRASTRUCTURE.  Follows the paper's description of ADAPT-VQE
("Numerical performance"): grow the ansatz one pool operator at a time,
choosing the operator with the largest energy gradient, then re-optimise all
parameters, starting from the Hartree-Fock determinant.  The state is
U(theta)|psi_0> with U = prod_i exp(theta_i A_{k_i}), newest factor applied
last (the state-preparation operator of "General Framework for Variational
Algorithms").

Readings where the paper is silent (each listed in the design notes):
  * selection: argmax |g_k|, ties (|g_k| >= max|g| (1 - tol)) resolved to
    the lowest canonical pool index;
  * inner optimiser: BFGS (scipy), gradient-norm (inf) tolerance gtol,
    warm-started from the previous parameters with the new one at 0;
  * stop early when max |g| < 1e-10.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.optimize import minimize

from . import apply_generator, apply_h, dot, pool_gradients, rotate


@dataclass
class AdaptLog:
    energies: list = field(default_factory=list)     # energy after each iteration's optimisation
    selected: list = field(default_factory=list)     # pool index appended each iteration
    tie_sets: list = field(default_factory=list)     # candidate set of each selection
    gmax: list = field(default_factory=list)         # max |g| at selection time
    grads: list = field(default_factory=list)        # full gradient vector at selection time
    thetas: list = field(default_factory=list)       # parameters after optimisation
    n_evals: list = field(default_factory=list)      # energy evaluations per iteration
    forced: int = 0                                   # teacher-forced selections
    e_hf: float = 0.0


class SectorProblem:
    def __init__(self, M, na, nb, x, z, c, cre, ann):
        self.M, self.na, self.nb = M, na, nb
        self.x, self.z, self.c = x, z, c
        self.cre, self.ann = np.asarray(cre), np.asarray(ann)
        from . import sector_dim
        self.dim = sector_dim(M, na, nb)

    def hf(self):
        v = np.zeros(self.dim)
        v[0] = 1.0  # the lowest-index determinant has sector index 0
        return v

    def hpsi(self, psi):
        return apply_h(self.M, self.na, self.nb, self.x, self.z, self.c, psi)

    def state(self, ops, thetas):
        psi = self.hf()
        for k, th in zip(ops, thetas):
            psi = rotate(self.M, self.na, self.nb, self.cre[k], self.ann[k], th, psi)
        return psi

    def energy_grad(self, ops, thetas):
        """E(theta) and dE/dtheta_i = 2 <H psi | d psi / d theta_i>, with
        d psi / d theta_i = U_j..U_{i+1} A_i U_i..U_1 |psi_0> built directly."""
        psi = self.state(ops, thetas)
        sig = self.hpsi(psi)
        E = dot(psi, sig)
        grad = np.zeros(len(ops))
        for i in range(len(ops)):
            v = self.state(ops[: i + 1], thetas[: i + 1])
            k = ops[i]
            v = apply_generator(self.M, self.na, self.nb, self.cre[k], self.ann[k], v)
            for kk, th in zip(ops[i + 1:], thetas[i + 1:]):
                v = rotate(self.M, self.na, self.nb, self.cre[kk], self.ann[kk], th, v)
            grad[i] = 2.0 * dot(sig, v)
        return E, grad


class DenseSectorProblem(SectorProblem):
    """The same definitions on small sectors with faster linear algebra: H as
    the dense sector matrix of the Pauli sum (element by element from the
    Pauli strings), each generator A as a sparse matrix of its literal pairs,
    exp(theta A) = 1 + sin(theta) A + (1 - cos(theta)) A^2 (A^3 = -A), and
    g_k = 2 sigma^T A_k psi.  For dim <= ~5,000."""

    def __init__(self, M, na, nb, x, z, c, cre, ann):
        super().__init__(M, na, nb, x, z, c, cre, ann)
        import scipy.sparse as sp
        from . import brute, pair_list
        self.H = brute.sector_matrix_from_paulis(M, na, nb, x, z, c).real
        self._sp = sp
        self._pair_list = pair_list
        self._A = {}

    def A(self, k):
        if k not in self._A:
            src, dst, sg = self._pair_list(self.M, self.na, self.nb, self.cre[k], self.ann[k])
            s = sg.astype(np.float64)
            # A|D> = s|D'>, A|D'> = -s|D>
            rows = np.concatenate([dst, src])
            cols = np.concatenate([src, dst])
            vals = np.concatenate([s, -s])
            self._A[k] = self._sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))
        return self._A[k]

    def hpsi(self, psi):
        return self.H @ psi

    def rot(self, k, th, v):
        Av = self.A(k) @ v
        return v + np.sin(th) * Av + (1.0 - np.cos(th)) * (self.A(k) @ Av)

    def state(self, ops, thetas):
        psi = self.hf()
        for k, th in zip(ops, thetas):
            psi = self.rot(k, th, psi)
        return psi

    def energy_grad(self, ops, thetas):
        psi = self.state(ops, thetas)
        sig = self.hpsi(psi)
        E = float(psi @ sig)
        grad = np.zeros(len(ops))
        for i in range(len(ops)):
            v = self.state(ops[: i + 1], thetas[: i + 1])
            v = self.A(ops[i]) @ v
            for kk, th in zip(ops[i + 1:], thetas[i + 1:]):
                v = self.rot(kk, th, v)
            grad[i] = 2.0 * float(sig @ v)
        return E, grad

    def gradients(self, psi, sig):
        return np.array([2.0 * float(sig @ (self.A(k) @ psi)) for k in range(len(self.cre))])


def run_adapt(prob: SectorProblem, n_iter: int, tie_tol: float = 1e-9, gtol: float = 1e-9,
              force=None) -> AdaptLog:
    """force(iteration, gradients, own_choice) -> index lets a caller
    teacher-force the selection (the caller validates it against gradients)."""
    log = AdaptLog()
    ops: list = []
    thetas = np.zeros(0)
    psi = prob.hf()
    log.e_hf = dot(psi, prob.hpsi(psi))
    for it in range(n_iter):
        sig = prob.hpsi(psi)
        if isinstance(prob, DenseSectorProblem):
            g = prob.gradients(psi, sig)
        else:
            g = pool_gradients(prob.M, prob.na, prob.nb, prob.cre, prob.ann, psi, sig)
        ag = np.abs(g)
        gm = float(ag.max())
        if gm < 1e-10:
            break
        ties = np.nonzero(ag >= gm * (1.0 - tie_tol))[0]
        k = int(ties.min())
        if force is not None:
            # the caller checks the forced index against g (near-ties it
            # accepts are its decision) and the oracle follows it
            fk = int(force(it, g, k))
            if fk != k:
                log.forced += 1
                k = fk
        ops.append(k)
        thetas = np.append(thetas, 0.0)
        nev = [0]

        def fun(t):
            nev[0] += 1
            return prob.energy_grad(ops, t)

        res = minimize(fun, thetas, jac=True, method="BFGS",
                       options={"gtol": gtol, "maxiter": 1000})
        thetas = np.array(res.x)
        psi = prob.state(ops, thetas)
        log.energies.append(float(res.fun))
        log.selected.append(k)
        log.tie_sets.append(ties.tolist())
        log.gmax.append(gm)
        log.grads.append(g)
        log.thetas.append(thetas.copy())
        log.n_evals.append(nev[0])
    return log
