"""hyp_pool_gradients is asynchronous: nothing in it waits on the host, so
the full sweep can be captured in a HIP graph, and an invalid excitation in
the device-resident list is caught on the device (NaN gradient, recorded for
hyp_pool_check) instead of by a host copy of the list."""
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


def _problem(hyp, name):
    w = synth.WORKLOADS[name]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    return w, S, H, cre, ann, (x, z, c)


@pytest.mark.parametrize("name", ["h8_16q", "h12_24q"])
@pytest.mark.parametrize("skip", [True, False])
def test_sweep_graph_replay_equals_eager(hyp, name, skip):
    w, S, H, cre, ann, _ = _problem(hyp, name)
    ops = hyp.exc_tensor(cre, ann)
    hyp.set_support_skip(skip)
    try:
        psi = torch.from_numpy(synth.random_state(S.dim, 7)).cuda()
        sig = H.apply(psi)
        out = torch.empty(len(cre), dtype=torch.float64, device="cuda")
        hyp.hyp_pool_gradients(S, ops, psi, sig, out)  # eager call: scratch and tables
        torch.cuda.synchronize()
        eager = out.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            hyp.hyp_pool_gradients(S, ops, psi, sig, out)
        # each replay recomputes from the buffers' current contents, with the
        # program's own eager work and synchronisations in between
        states = [7, 11, 7, 13]
        for seed in states:
            out.fill_(-1.0)
            p = torch.from_numpy(synth.random_state(S.dim, seed)).cuda()
            psi.copy_(p)
            sig.copy_(H.apply(p))
            ref = hyp.hyp_pool_gradients(S, ops, p, H.apply(p)).clone()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (name, skip, seed)
        # a sparse state (support skipping takes its gathered branches on the device)
        idx, val = synth.sparse_state(S.dim, S.da)
        p = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
        p[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).cuda()
        psi.copy_(p)
        sig.copy_(H.apply(p))
        ref = hyp.hyp_pool_gradients(S, ops, p, H.apply(p)).clone()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert torch.equal(eager, hyp.hyp_pool_gradients(S, ops, torch.from_numpy(synth.random_state(S.dim, 7)).cuda(),
                                                          H.apply(torch.from_numpy(synth.random_state(S.dim, 7)).cuda())))
        hyp.hyp_pool_check()
    finally:
        hyp.set_support_skip(True)


@pytest.mark.parametrize("mode", ["auto", "pairs"])
def test_invalid_excitation_nan_and_check(hyp, mode):
    w, S, H, cre, ann, (x, z, c) = _problem(hyp, "h8_16q")
    M = w.n_orb
    cre = cre.astype(np.uint32).copy()
    ann = ann.astype(np.uint32).copy()
    bad = {5: (np.uint32(1 << 0), np.uint32(1 << M)),        # alpha created, beta annihilated: sector
           17: (np.uint32(0b11), np.uint32(0b10)),            # cre and ann overlap
           40: (np.uint32(1 << (2 * M)), np.uint32(1 << 1))}  # mask bit outside 2M qubits
    for k, (cm, am) in bad.items():
        cre[k], ann[k] = cm, am
    psi_h = synth.random_state(S.dim, 7)
    psi = torch.from_numpy(psi_h).cuda()
    sig = H.apply(psi)
    hyp.hyp_pool_check()  # clean record
    hyp.set_sweep_mode(mode)
    try:
        g = hyp.hyp_pool_gradients(S, hyp.exc_tensor(cre, ann), psi, sig).cpu().numpy()
        with pytest.raises(hyp.HypError) as ei:
            hyp.hyp_pool_check()
        assert "excitation 5 " in str(ei.value)
        assert ei.value.status == 2  # HYP_ERR_SECTOR is the largest status met
        hyp.hyp_pool_check()  # the record was cleared
    finally:
        hyp.set_sweep_mode("auto")
    assert all(np.isnan(g[k]) for k in bad)
    good = np.array([k for k in range(len(cre)) if k not in bad])
    ref = oracle.pool_gradients(M, w.n_alpha, w.n_beta, cre[good], ann[good], psi_h, sig.cpu().numpy())
    assert np.abs(g[good] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
