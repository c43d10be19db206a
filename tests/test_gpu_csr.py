"""GPU parity of the materialised CSR Hamiltonian (the paper's storage,
kept as a comparison for the matrix-free product): the exported matrix
against the oracle's sector matrix (columns of oracle.apply_h), its SpMV
against the oracle, the 24-qubit SpMV against the matrix-free product, and
the refusals (28 qubits does not fit, generic Hamiltonians)."""
import math
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hyp():
    import paper_2604_01176_amd as hyp
    return hyp


def _ham(hyp, M, na, nb, seed):
    h, g = synth.integrals(M, seed)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    return S, hyp.Hamiltonian(S, x, z, c), (x, z, c)


def _row_length(M, na, nb):
    s = lambda n: n * (M - n)
    d = lambda n: math.comb(n, 2) * math.comb(M - n, 2)
    return 1 + s(na) + d(na) + s(nb) + d(nb) + s(na) * s(nb)


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 3, 2), (6, 3, 3), (7, 2, 5), (3, 0, 2), (4, 4, 1), (2, 1, 1)])
def test_csr_matrix_equals_oracle(hyp, M, na, nb):
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 900 + M)
    A = hyp.CsrMatrix(H)
    L = _row_length(M, na, nb)
    assert A.nnz == S.dim * L
    rp, col, val = A.export()
    assert np.array_equal(rp, np.arange(S.dim + 1, dtype=np.int64) * L)
    dense = np.zeros((S.dim, S.dim))
    for d in range(S.dim):
        cols = col[d * L:(d + 1) * L]
        assert np.unique(cols).size == L  # each column once
        assert cols.min() >= 0 and cols.max() < S.dim
        dense[d, cols] = val[d * L:(d + 1) * L]
    ref = np.stack([oracle.apply_h(M, na, nb, x, z, c, np.eye(S.dim)[j]) for j in range(S.dim)], 1)
    assert np.abs(dense - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.all(dense[ref != 0.0] != 0.0) or np.abs(ref[dense == 0.0]).max() <= 1e-13


@pytest.mark.parametrize("M,na,nb", [(6, 3, 3), (8, 4, 4), (9, 5, 4), (10, 5, 5)])
def test_csr_spmv(hyp, M, na, nb):
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 950 + M)
    A = hyp.CsrMatrix(H)
    psi = synth.random_state(S.dim, 29)
    ref = oracle.apply_h(M, na, nb, x, z, c, psi)
    out = A.apply(torch.from_numpy(psi).cuda()).cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
    p32 = psi.astype(np.float32)
    ref32 = oracle.apply_h(M, na, nb, x, z, c, p32.astype(np.float64))
    out32 = A.apply(torch.from_numpy(p32).cuda()).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(out32 - ref32) <= 2e-6 * np.linalg.norm(ref32)


def test_csr_24q_against_matrix_free(hyp):
    w = synth.WORKLOADS["h12_24q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    t0 = time.perf_counter()
    A = hyp.CsrMatrix(H)
    t_build = time.perf_counter() - t0
    psi = torch.from_numpy(synth.random_state(S.dim, 7)).cuda()
    mf = H.apply(psi)
    cs = A.apply(psi)
    torch.cuda.synchronize()
    times = {}
    for name, fn in (("csr", lambda: A.apply(psi, cs)), ("matrix_free", lambda: H.apply(psi, mf))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / 5 * 1e3
    print(f"[csr] 24q: nnz {A.nnz}, {A.nnz * 12 / 1e9:.1f} GB, build {t_build:.2f} s, "
          f"SpMV {times['csr']:.2f} ms, matrix-free {times['matrix_free']:.2f} ms", flush=True)
    a, b = cs.cpu().numpy(), mf.cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([[0, S.dim - 1], rng.integers(0, S.dim, 100)]))
    ref = oracle.apply_h(M, na, nb, x, z, c, psi.cpu().numpy(), out_idx=idx)
    assert np.abs(a[idx] - ref).max() <= 1e-12 * np.linalg.norm(ref) / math.sqrt(len(idx)) * 10
    A.close()


def test_csr_refusals(hyp):
    w = synth.WORKLOADS["h14_28q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    with pytest.raises(hyp.HypError) as e:
        hyp.CsrMatrix(H)
    assert e.value.status == 4 and "bytes" in str(e.value)
    # a Pauli sum outside the two-body number-conserving class (random real
    # strings, including three-body ones) has no structured form to materialise
    M, na, nb = 4, 2, 1
    rng = np.random.default_rng(5)
    xs, zs = [], []
    while len(xs) < 300:
        xx, zz = (int(v) for v in rng.integers(0, 1 << (2 * M), 2))
        if bin(xx & zz).count("1") % 2 == 0:
            xs.append(xx)
            zs.append(zz)
    S2 = hyp.Sector(M, na, nb)
    H2 = hyp.Hamiltonian(S2, np.array(xs, dtype=np.uint32), np.array(zs, dtype=np.uint32),
                         rng.standard_normal(len(xs)))
    assert not H2.structured
    with pytest.raises(hyp.HypError) as e:
        hyp.CsrMatrix(H2)
    assert e.value.status == 6
