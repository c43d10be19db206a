"""The sweep's singles and alpha-beta doubles as dense products on the
matrix cores (k_tdens_m) against the oracle (the whole pool on small
sectors) and against the row-batched transition values (k_tdens_rows):
sectors whose alpha dimension is and is not a multiple of the 48-column
chunk, fewer than 16 orbitals, empty and full spins, dense and sparse
states with support skipping on and off, fermionic and qubit generators,
FP32 storage, bitwise repeatability and graph replay, and the 28-qubit
workload (the 32-qubit one is in test_gpu_full_size.py)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hyp():
    import paper_2604_01176_amd as hyp
    yield hyp
    hyp.set_mixed_matrix_cores()
    hyp.set_support_skip(True)
    hyp.set_pool_kind("fermionic")


def _problem(hyp, M, na, nb, seed):
    h, g = synth.integrals(M, seed)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, cls = synth.canonical_pool(M)
    return S, H, cre, ann


def _grads(hyp, S, ops, psi, sig, mm):
    try:
        hyp.set_mixed_matrix_cores(mm)
        out = hyp.hyp_pool_gradients(S, ops, psi, sig)
        torch.cuda.synchronize()
        return out
    finally:
        hyp.set_mixed_matrix_cores()


CASES = [(4, 2, 2), (6, 3, 3), (7, 2, 5), (8, 4, 4), (9, 5, 4), (10, 5, 5), (3, 0, 2), (6, 3, 0), (6, 6, 3),
         (11, 6, 5)]


@pytest.mark.parametrize("M,na,nb", CASES)
@pytest.mark.parametrize("skip", [True, False])
@pytest.mark.parametrize("kind", ["fermionic", "qubit"])
def test_matrix_core_sweep_equals_oracle(hyp, M, na, nb, skip, kind):
    S, H, cre, ann = _problem(hyp, M, na, nb, 600 + M + nb)
    ops = hyp.exc_tensor(cre, ann)
    idx, val = synth.sparse_state(S.dim, S.da, n_random=max(1, S.dim // 30))
    sparse = np.zeros(S.dim)
    sparse[idx] = val
    hyp.set_support_skip(skip)
    hyp.set_pool_kind(kind)
    try:
        for psi_h in (synth.random_state(S.dim, 9 + M), sparse):
            psi = torch.from_numpy(psi_h).cuda()
            sig = H.apply(psi)
            got = _grads(hyp, S, ops, psi, sig, True)
            again = _grads(hyp, S, ops, psi, sig, True)
            rows = _grads(hyp, S, ops, psi, sig, False).cpu().numpy()
            assert torch.equal(got, again)  # fixed order: bit for bit
            got = got.cpu().numpy()
            scale = max(1.0, np.abs(rows).max())
            assert np.abs(got - rows).max() <= 1e-13 * scale
            if M <= 9 and kind == "fermionic":
                ref = oracle.pool_gradients(M, na, nb, cre, ann, psi_h, sig.cpu().numpy())
                assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    finally:
        hyp.set_support_skip(True)
        hyp.set_pool_kind("fermionic")


@pytest.mark.parametrize("M,na,nb", [(8, 4, 4), (11, 6, 5)])
def test_matrix_core_sweep_fp32(hyp, M, na, nb):
    """FP32 storage: both forms against the FP64 sweep of the FP32-rounded
    operands (the matrix-core form multiplies in FP64, the other in FP32)."""
    S, H, cre, ann = _problem(hyp, M, na, nb, 650 + M)
    ops = hyp.exc_tensor(cre, ann)
    psi64 = torch.from_numpy(synth.random_state(S.dim, 3)).cuda()
    sig64 = H.apply(psi64)
    psi32, sig32 = psi64.float(), sig64.float()
    ref = _grads(hyp, S, ops, psi32.double(), sig32.double(), False).cpu().numpy()
    got = _grads(hyp, S, ops, psi32, sig32, True).cpu().numpy()
    rows = _grads(hyp, S, ops, psi32, sig32, False).cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(got - ref).max() <= 1e-12 * scale
    assert np.abs(rows - ref).max() <= 1e-5 * scale


def test_matrix_core_sweep_in_captured_graph(hyp):
    """hyp_pool_gradients with the matrix-core form captured in a HIP graph
    and replayed with eager work in between: every replay equals the eager
    sweep of the buffers' current contents bit for bit."""
    S, H, cre, ann = _problem(hyp, 10, 5, 4, 91)
    ops = hyp.exc_tensor(cre, ann)
    try:
        hyp.set_mixed_matrix_cores(True)
        psi = torch.from_numpy(synth.random_state(S.dim, 1)).cuda()
        sig = H.apply(psi)
        out = hyp.hyp_pool_gradients(S, ops, psi, sig)  # eager call: scratch
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            hyp.hyp_pool_gradients(S, ops, psi, sig, out)
        for seed in (2, 3, 2):
            p = torch.from_numpy(synth.random_state(S.dim, seed)).cuda()
            sg = H.apply(p)
            ref = hyp.hyp_pool_gradients(S, ops, p, sg).clone()
            torch.cuda.synchronize()
            psi.copy_(p)
            sig.copy_(sg)
            out.fill_(-1.0)
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), seed
    finally:
        hyp.set_mixed_matrix_cores()


def test_matrix_core_sweep_28q(hyp):
    w = synth.WORKLOADS["h14_28q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, cls = synth.canonical_pool(w.n_orb)
    ops = hyp.exc_tensor(cre, ann)
    psi_h = synth.random_state(S.dim, 4)
    psi = torch.from_numpy(psi_h).cuda()
    sig = H.apply(psi)
    got = _grads(hyp, S, ops, psi, sig, True).cpu().numpy()  # (auto takes the row-batched kernel below 256 MiB)
    rows = _grads(hyp, S, ops, psi, sig, False).cpu().numpy()
    scale = max(1.0, np.abs(rows).max())
    print(f"[sweep-mm] 28q: max difference {np.abs(got - rows).max() / scale:.2e} of the largest gradient", flush=True)
    assert np.abs(got - rows).max() <= 1e-12 * scale
    rng = np.random.default_rng(2)
    pick = []
    for k in range(5):
        members = np.nonzero(cls == k)[0]
        pick += rng.choice(members, 4, replace=False).tolist()
    pick = np.array(sorted(pick))
    ref = oracle.pool_gradients(w.n_orb, w.n_alpha, w.n_beta, cre[pick], ann[pick], psi_h, sig.cpu().numpy())
    assert np.abs(got[pick] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("frac", [0.2, 0.3])
def test_device_choice_under_support_skipping(hyp, frac):
    """With support skipping the form is chosen on the device: the
    matrix-core kernel where at least a quarter of the beta rows hold
    amplitude, the row-batched one below (both launched, the other exits).
    States just under and over the quarter give the oracle's gradients."""
    M, na, nb = 9, 4, 5
    S, H, cre, ann = _problem(hyp, M, na, nb, 977)
    ops = hyp.exc_tensor(cre, ann)
    rng = np.random.default_rng(31)
    rows = rng.choice(S.db, max(1, int(round(frac * S.db))), replace=False)
    psi_h = np.zeros(S.dim)
    for r in rows:
        psi_h[r * S.da:(r + 1) * S.da] = rng.standard_normal(S.da)
    psi_h /= np.linalg.norm(psi_h)
    psi = torch.from_numpy(psi_h).cuda()
    sig = H.apply(psi)
    hyp.set_support_skip(True)
    got = _grads(hyp, S, ops, psi, sig, True).cpu().numpy()
    ref = oracle.pool_gradients(M, na, nb, cre, ann, psi_h, sig.cpu().numpy())
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    hyp.set_support_skip(False)
    try:
        full = _grads(hyp, S, ops, psi, sig, True).cpu().numpy()  # every row: the matrix-core kernel
    finally:
        hyp.set_support_skip(True)
    assert np.abs(got - full).max() <= 1e-13 * max(1.0, np.abs(full).max())
