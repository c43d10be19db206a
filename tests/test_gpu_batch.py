"""Batched sweep: eight uneven instances (8..12 orbitals, odd orbital counts
with N_alpha != N_beta) in one persistent launch, against per-instance
gradients and the oracle; the autotuner returns a valid, timed tile."""
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


@pytest.fixture(scope="module")
def instances(hyp):
    out = []
    for w in synth.INSTANCES:
        x, z, c, _, _ = synth.hamiltonian(w)
        cre, ann, _ = synth.canonical_pool(w.n_orb)
        S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        psi_h = synth.random_state(S.dim, 7 + w.n_orb)
        psi = torch.from_numpy(psi_h).cuda()
        sig = H.apply(psi)
        out.append(dict(w=w, S=S, H=H, cre=cre, ann=ann, ops=hyp.exc_tensor(cre, ann), psi=psi,
                        sig=sig, psi_h=psi_h, xzc=(x, z, c)))
    return out


@pytest.mark.parametrize("route", ["full", "subset", "pairs"])
def test_batched_equals_single_and_oracle(hyp, instances, route):
    """Full pools (transition-value sweeps per instance), candidate subsets
    (the fused persistent launch) and full pools forced through the fused
    launch, against per-instance calls and the oracle."""
    jobs, refs, subsets = [], [], []
    rng0 = np.random.default_rng(11)
    try:
        if route == "pairs":
            hyp.set_sweep_mode("pairs")
        for d in instances:
            n = len(d["cre"])
            k = np.sort(rng0.choice(n, n // 7, replace=False)) if route == "subset" else np.arange(n)
            subsets.append(k)
            ops = hyp.exc_tensor(d["cre"][k], d["ann"][k])
            g = torch.empty(len(k), dtype=torch.float64, device="cuda")
            jobs.append((d["S"], ops, d["psi"], d["sig"], g))
            refs.append(hyp.hyp_pool_gradients(d["S"], ops, d["psi"], d["sig"]).cpu().numpy())
        for tile in [None, (128, 4, 2), (512, 32, 8), (64, 1, 1)]:
            hyp.hyp_pool_gradients_batched(jobs, tile)
            torch.cuda.synchronize()
            for (S, ops, psi, sig, g), ref in zip(jobs, refs):
                got = g.cpu().numpy()
                assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    finally:
        hyp.set_sweep_mode("auto")
    # oracle on a sample of generators of every instance
    rng = np.random.default_rng(2)
    for d, sub, (S, ops, psi, sig, g) in zip(instances, subsets, jobs):
        w = d["w"]
        j = rng.choice(len(sub), 6, replace=False)
        k = sub[j]
        sig_h = d["sig"].cpu().numpy()
        ref = oracle.pool_gradients(w.n_orb, w.n_alpha, w.n_beta, d["cre"][k], d["ann"][k],
                                    d["psi_h"], sig_h)
        got = g.cpu().numpy()[j]
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_batched_fp32(hyp, instances):
    jobs, refs = [], []
    for d in instances[:4]:
        p32 = d["psi"].float()
        s32 = d["H"].apply(p32)
        g = torch.empty(len(d["cre"]), dtype=torch.float64, device="cuda")
        jobs.append((d["S"], d["ops"], p32, s32, g))
        refs.append(hyp.hyp_pool_gradients(d["S"], d["ops"], d["psi"], d["sig"]).cpu().numpy())
    hyp.hyp_pool_gradients_batched(jobs)
    torch.cuda.synchronize()
    for (S, ops, psi, sig, g), ref in zip(jobs, refs):
        assert np.abs(g.cpu().numpy() - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_autotuner(hyp, instances):
    jobs = []
    for d in instances:
        g = torch.empty(len(d["cre"]), dtype=torch.float64, device="cuda")
        jobs.append((d["S"], d["ops"], d["psi"], d["sig"], g))
    tile, ms = hyp.hyp_tune_pool_gradients(jobs, reps=1)
    assert tile[0] in (128, 256, 512) and tile[1] in (4, 8, 16, 32) and tile[2] in (2, 4, 8)
    assert ms > 0
    print(f"autotuned tile {tile}: {ms:.3f} ms for 8 instances")


def test_batched_rejects_bad_ops(hyp, instances):
    d = instances[0]
    bad = hyp.exc_tensor([0b11], [0b100])  # |cre| != |ann|
    g = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(hyp.HypError):
        hyp.hyp_pool_gradients_batched([(d["S"], bad, d["psi"], d["sig"], g)])
