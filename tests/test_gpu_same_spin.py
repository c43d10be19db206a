"""The FP64 same-spin pass, its three forms against the oracle and against
each other, with support skipping on and off: the per-row lists, the grouped
lists (8 consecutive output strings per wave sharing their source loads),
and the doubles through the strings' cores (per-core dense products on the
matrix cores, each row adding its cores' rows), on sectors whose string
counts are and are not multiples of the group size, empty and full spins,
spins without doubles, cores with more than 48 slots (no core tables: the
grouped lists serve), and the 32-qubit workload on its sparse input (every
entry) and on sampled rows of the dense state."""
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
    H = hyp.Hamiltonian(S, x, z, c)
    return S, H, (x, z, c)


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 3, 2), (6, 3, 3), (7, 2, 5), (8, 4, 4), (9, 5, 4),
                                     (10, 5, 5), (3, 0, 2), (4, 4, 1), (11, 6, 5)])
@pytest.mark.parametrize("skip", [True, False])
def test_grouped_equals_oracle_and_per_row(hyp, M, na, nb, skip):
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 300 + M)
    assert H.structured
    idx, val = synth.sparse_state(S.dim, S.da, n_random=max(1, S.dim // 50))
    states = [synth.random_state(S.dim, 7), np.zeros(S.dim)]
    states[1][idx] = val
    hyp.set_support_skip(skip)
    try:
        for psi in states:
            d = torch.from_numpy(psi).cuda()
            hyp.set_same_spin_cores(False)
            hyp.set_same_spin_groups(False)
            per_row = H.apply(d).cpu().numpy()
            ref = oracle.apply_h(M, na, nb, x, z, c, psi)
            nrm = max(np.linalg.norm(ref), 1e-300)
            for tiles in (1, 2, 4):  # the workgroup shapes of the grouped kernel
                hyp.set_same_spin_groups(tiles)
                got = H.apply(d).cpu().numpy()
                assert np.linalg.norm(got - ref) <= 1e-12 * nrm, tiles
                assert np.linalg.norm(got - per_row) <= 1e-14 * nrm, tiles
            # the doubles through the cores
            hyp.set_same_spin_cores(True)
            got = H.apply(d).cpu().numpy()
            assert np.linalg.norm(got - ref) <= 1e-12 * nrm
            assert np.linalg.norm(got - per_row) <= 1e-14 * nrm
            assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)
            assert torch.equal(H.apply(d), H.apply(d))  # fixed summation order
    finally:
        hyp.set_same_spin_cores()
        hyp.set_same_spin_groups(True)
        hyp.set_support_skip(True)


@pytest.mark.parametrize("M,na,nb", [(12, 2, 3), (11, 2, 9)])
def test_cores_beyond_48_slots_fall_back(hyp, M, na, nb):
    """An alpha space with 2 electrons in 12 (11) orbitals has cores of
    C(12, 2) = 66 (55) slots: no core tables, the grouped lists serve, and
    switching the core path on or off changes nothing."""
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 900 + M)
    psi = synth.random_state(S.dim, 11)
    d = torch.from_numpy(psi).cuda()
    ref = oracle.apply_h(M, na, nb, x, z, c, psi)
    try:
        hyp.set_same_spin_cores(True)
        a = H.apply(d)
        hyp.set_same_spin_cores(False)
        b = H.apply(d)
    finally:
        hyp.set_same_spin_cores()
    assert torch.equal(a, b)
    assert np.linalg.norm(a.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


def test_grouped_32q(hyp):
    w = synth.WORKLOADS["h16_32q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    idx, val = synth.sparse_state(S.dim, S.da)
    ref = oracle.apply_h_sparse(w.n_orb, w.n_alpha, w.n_beta, x, z, c, idx, val)
    d = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
    d[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).cuda()
    for cores in (True, False):
        for skip in (True, False):
            hyp.set_support_skip(skip)
            hyp.set_same_spin_cores(cores)
            try:
                print(f"[same-spin] 32 qubits, sparse input, cores {cores}, skipping {skip}", flush=True)
                got = H.apply(d).cpu().numpy()
            finally:
                hyp.set_support_skip(True)
                hyp.set_same_spin_cores()
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            assert np.count_nonzero(got[ref == 0.0]) == 0
    # dense benchmark state: cores and grouped lists against the per-row
    # lists on every entry, the oracle on sampled rows (first and last rows
    # of groups, tiles and column bands)
    psi_h = synth.random_state(S.dim, 7)
    dp = torch.from_numpy(psi_h).cuda()
    try:
        hyp.set_same_spin_cores(True)
        got_c = H.apply(dp)
        hyp.set_same_spin_cores(False)
        got = H.apply(dp)
        hyp.set_same_spin_groups(False)
        per_row = H.apply(dp)
    finally:
        hyp.set_same_spin_groups(True)
        hyp.set_same_spin_cores()
    for name, g in (("grouped", got), ("cores", got_c)):
        rel = (torch.linalg.norm(g - per_row) / torch.linalg.norm(per_row)).item()
        print(f"[same-spin] dense 32 qubits: {name} vs per-row relative difference {rel:.2e}", flush=True)
        assert rel <= 1e-14
    da = S.da
    rows = np.array([0, 7, 8, 255, 256, 1471, 1472, da - 1, da, 8 * da + 63, 8 * da + 1472, 12864 * da + 12865,
                     S.dim - 1], dtype=np.int64)
    ref_rows = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi_h, out_idx=rows)
    for g in (got, got_c):
        g_rows = g[torch.from_numpy(rows).cuda()].cpu().numpy()
        assert np.abs(g_rows - ref_rows).max() <= 1e-12 * np.abs(ref_rows).max()


@pytest.mark.parametrize("skip", [True, False])
def test_core_path_in_captured_graph(hyp, skip):
    """H psi with the core path (forced on a small sector) captured in a HIP
    graph and replayed with eager work in between: every replay equals the
    eager product of the buffer's current state, for dense states (core path)
    and, with support skipping, sparse ones (the device-side choice takes the
    grouped lists) alternating."""
    M, na, nb = 10, 5, 4
    S, H, (x, z, c) = _ham(hyp, M, na, nb, 77)
    idx, val = synth.sparse_state(S.dim, S.da, n_random=3)
    sparse = np.zeros(S.dim)
    sparse[idx] = val
    states = [synth.random_state(S.dim, 5), sparse, synth.random_state(S.dim, 6), sparse * 0.5]
    try:
        hyp.set_same_spin_cores(True)
        hyp.set_support_skip(skip)
        psi = torch.from_numpy(states[0]).cuda()
        sig = torch.empty_like(psi)
        H.apply(psi, sig)  # eager call first: scratch and tables
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            H.apply(psi, sig)
        for k, st in enumerate(states):
            p = torch.from_numpy(st).cuda()
            ref = H.apply(p).clone()
            torch.cuda.synchronize()
            psi.copy_(p)
            sig.fill_(-1.0)
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(sig, ref), k
            o = oracle.apply_h(M, na, nb, x, z, c, st)
            assert np.linalg.norm(sig.cpu().numpy() - o) <= 1e-12 * max(np.linalg.norm(o), 1e-300), k
    finally:
        hyp.set_same_spin_cores()
        hyp.set_support_skip(True)
