"""The mixed alpha-beta pass as dense products on the matrix cores
(k_mixed_m) against the oracle and against the bitwise-reproducible forms
(k_mixed / k_mixed_c): sectors whose alpha dimension is and is not a multiple
of the 64-column chunk, fewer than 16 orbitals, empty and full spins, dense
and sparse states with support skipping on and off, FP64 and FP32 storage,
HIP-graph capture, and the 28- and 32-qubit workloads (every entry on a
sparse input, sampled rows of the dense benchmark state)."""
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


def _ham(hyp, M, na, nb, seed):
    h, g = synth.integrals(M, seed)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    return S, H, (x, z, c)


def _apply(hyp, H, d, mm):
    try:
        hyp.set_mixed_matrix_cores(mm)
        out = H.apply(d)
        torch.cuda.synchronize()
        return out
    finally:
        hyp.set_mixed_matrix_cores()


CASES = [(4, 2, 2), (5, 3, 2), (6, 3, 3), (7, 2, 5), (8, 4, 4), (9, 5, 4), (10, 5, 5), (3, 0, 2), (4, 4, 1),
         (11, 6, 5), (12, 2, 3), (6, 3, 0), (6, 6, 3)]


@pytest.mark.parametrize("M,na,nb", CASES)
@pytest.mark.parametrize("skip", [True, False])
def test_matrix_core_mixed_pass_equals_oracle(hyp, M, na, nb, skip):
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 500 + M + na)
    assert H.structured
    idx, val = synth.sparse_state(S.dim, S.da, n_random=max(1, S.dim // 40))
    sparse = np.zeros(S.dim)
    sparse[idx] = val
    hyp.set_support_skip(skip)
    try:
        for psi in (synth.random_state(S.dim, 3 + M), sparse):
            d = torch.from_numpy(psi).cuda()
            ref = oracle.apply_h(M, na, nb, x, z, c, psi)
            nrm = max(np.linalg.norm(ref), 1e-300)
            got = _apply(hyp, H, d, True).cpu().numpy()
            det = _apply(hyp, H, d, False).cpu().numpy()
            assert np.linalg.norm(got - ref) <= 1e-12 * nrm
            assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)
            assert np.linalg.norm(got - det) <= 1e-14 * nrm
            assert np.count_nonzero(got[ref == 0.0]) == 0 or not skip
    finally:
        hyp.set_support_skip(True)


@pytest.mark.parametrize("M,na,nb", [(8, 4, 4), (11, 6, 5), (12, 6, 6)])
def test_matrix_core_mixed_pass_fp32(hyp, M, na, nb):
    """FP32 storage: both forms against the oracle on the FP32-rounded input
    (the matrix-core form multiplies in FP64, the other in FP32)."""
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 700 + M)
    psi = synth.random_state(S.dim, 5).astype(np.float32).astype(np.float64)
    d = torch.from_numpy(psi).to("cuda", torch.float32)
    rng = np.random.default_rng(M)
    rows = np.unique(np.concatenate([[0, S.dim - 1], rng.integers(0, S.dim, 300)]))
    ref = oracle.apply_h(M, na, nb, x, z, c, psi, out_idx=rows)
    got = _apply(hyp, H, d, True)
    det = _apply(hyp, H, d, False)
    assert got.dtype == torch.float32
    scale = np.abs(ref).max()
    assert np.abs(got.cpu().numpy()[rows].astype(np.float64) - ref).max() <= 2e-6 * scale
    assert np.abs(det.cpu().numpy()[rows].astype(np.float64) - ref).max() <= 2e-6 * scale


def test_matrix_core_mixed_pass_in_captured_graph(hyp):
    """H psi with the matrix-core mixed pass captured in a HIP graph and
    replayed with eager work in between: every replay matches the eager
    product of the buffer's current state to rounding, and the oracle."""
    M, na, nb = 10, 5, 4
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 81)
    try:
        hyp.set_mixed_matrix_cores(True)
        psi = torch.from_numpy(synth.random_state(S.dim, 1)).cuda()
        sig = torch.empty_like(psi)
        H.apply(psi, sig)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            H.apply(psi, sig)
        for seed in (2, 3, 2):
            st = synth.random_state(S.dim, seed)
            p = torch.from_numpy(st).cuda()
            ref = H.apply(p).clone()
            torch.cuda.synchronize()
            psi.copy_(p)
            sig.fill_(-1.0)
            g.replay()
            torch.cuda.synchronize()
            assert (torch.linalg.norm(sig - ref) / torch.linalg.norm(ref)).item() <= 1e-15
            o = oracle.apply_h(M, na, nb, x, z, c, st)
            assert np.linalg.norm(sig.cpu().numpy() - o) <= 1e-12 * np.linalg.norm(o)
    finally:
        hyp.set_mixed_matrix_cores()


@pytest.mark.parametrize("name", ["h14_28q", "h16_32q"])
def test_matrix_core_mixed_pass_workloads(hyp, name):
    """The 28- and 32-qubit workloads: every entry of sigma on a sparse input
    against the oracle with skipping on and off, and the dense benchmark
    state against the bitwise-reproducible form (every entry) and the
    oracle on sampled rows (first and last rows, chunk edges)."""
    w = synth.WORKLOADS[name]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    idx, val = synth.sparse_state(S.dim, S.da)
    ref = oracle.apply_h_sparse(w.n_orb, w.n_alpha, w.n_beta, x, z, c, idx, val)
    d = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
    d[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).cuda()
    try:
        for skip in (True, False):
            hyp.set_support_skip(skip)
            print(f"[mixed-mm] {name}: sparse input, skipping {skip}", flush=True)
            got = _apply(hyp, H, d, True).cpu().numpy()
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            assert np.count_nonzero(got[ref == 0.0]) == 0
    finally:
        hyp.set_support_skip(True)
    del d
    psi_h = synth.random_state(S.dim, 7)
    dp = torch.from_numpy(psi_h).cuda()
    got = _apply(hyp, H, dp, True)
    det = _apply(hyp, H, dp, False)
    rel = (torch.linalg.norm(got - det) / torch.linalg.norm(det)).item()
    amax = ((got - det).abs().max() / det.abs().max()).item()
    print(f"[mixed-mm] {name} dense: relative difference {rel:.2e}, max {amax:.2e}", flush=True)
    assert rel <= 1e-14 and amax <= 1e-13
    da = S.da
    rows = np.array([0, 1, 63, 64, 65, da - 1, da, 2 * da + 127, 5 * da + 128, S.dim // 2, S.dim - da,
                     S.dim - 1], dtype=np.int64)
    ref_rows = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi_h, out_idx=rows)
    g_rows = got[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.abs(g_rows - ref_rows).max() <= 1e-12 * np.abs(ref_rows).max()
    del dp, got, det
    torch.cuda.empty_cache()


@pytest.mark.parametrize("frac", [0.2, 0.3])
def test_device_choice_under_support_skipping(hyp, frac):
    """With support skipping the mixed pass's form is chosen on the device:
    the matrix-core kernel where at least a quarter of the beta rows hold
    amplitude, k_mixed / k_mixed_c below (both launched, the other exits).
    States just under and over the quarter give the oracle's sigma."""
    M, na, nb = 10, 5, 4
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 955)
    rng = np.random.default_rng(17)
    rows = rng.choice(S.db, max(1, int(round(frac * S.db))), replace=False)
    psi_h = np.zeros(S.dim)
    for r in rows:
        psi_h[r * S.da:(r + 1) * S.da] = rng.standard_normal(S.da)
    psi_h /= np.linalg.norm(psi_h)
    d = torch.from_numpy(psi_h).cuda()
    ref = oracle.apply_h(M, na, nb, x, z, c, psi_h)
    hyp.set_support_skip(True)
    got = _apply(hyp, H, d, True).cpu().numpy()
    hyp.set_support_skip(False)
    try:
        full = _apply(hyp, H, d, True).cpu().numpy()  # every row: the matrix-core kernel
    finally:
        hyp.set_support_skip(True)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(got - full) <= 1e-14 * np.linalg.norm(full)
