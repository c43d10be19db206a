"""Learned screen on the GPU: MFMA forward/backward and Adam against the FP64
reference with the same BF16 rounding points, the feature and occupation
kernels, the ranking, and screened ADAPT against the full sweep it screens
(argmax agreement, energies) plus the ablation against screening without a
trained network."""
import numpy as np
import pytest

import oracle
from oracle import mlp as om
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hyp():
    import paper_2604_01176_amd as hyp
    return hyp


@pytest.fixture(scope="module")
def scr():
    from paper_2604_01176_amd import screen
    return screen


def _bf16_bits(x):
    f = om.bf16(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def test_mlp_forward_parity(scr):
    p = synth.mlp_init(11)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((1000, om.N_FEAT))
    net = scr.MLP(p, 1024)
    Xd = torch.from_numpy(_bf16_bits(X)).cuda()
    y = net.forward(Xd).cpu().numpy().astype(np.float64)
    ref, _ = om.forward(p.astype(np.float64), X, quant=True)
    assert np.linalg.norm(y - ref) <= 2e-4 * np.linalg.norm(ref)
    assert np.abs(y - ref).max() <= 2e-3 * np.abs(ref).max()


def test_mlp_train_step_parity(scr):
    p = synth.mlp_init(5)
    rng = np.random.default_rng(1)
    B = 1024
    X = rng.standard_normal((B, om.N_FEAT))
    t = rng.standard_normal(B).astype(np.float32)
    net = scr.MLP(p, B)
    Xd = torch.from_numpy(_bf16_bits(X)).cuda()
    td = torch.from_numpy(t).cuda()
    net.train_step(Xd, td, lr=1e-3)
    g = net.grads().astype(np.float64)
    loss, _, gref = om.loss_grad(p.astype(np.float64), X, t.astype(np.float64), quant=True)
    blocks = [(0, 8192), (8192, 8448), (8448, 73984), (73984, 74240), (74240, 74496), (74496, 74497)]
    for lo, hi in blocks:
        a, b = g[lo:hi], gref[lo:hi]
        assert np.linalg.norm(a - b) <= 5e-3 * np.linalg.norm(b) + 1e-9, (lo, hi)
    adam = om.Adam(p.astype(np.float64), lr=1e-3)
    p1 = adam.step(g)  # the reference update applied to the GPU's own gradient
    assert np.abs(net.params() - p1).max() <= 1e-6


def test_occupations_and_features(hyp, scr):
    w = synth.WORKLOADS["h8_16q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, cls = synth.canonical_pool(M)
    S = hyp.Sector(M, na, nb)
    psi = synth.random_state(S.dim, 3)
    stat, qidx = scr.static_features(M, cre, ann, cls, h, g)
    fs = scr.FeatureState(S, stat, qidx)
    gprev = np.random.default_rng(2).standard_normal(len(cre)) * 1e-3
    gprev[::7] = np.nan
    fs.update(gprev)
    fs.update(np.where(np.arange(len(cre)) % 3 == 0, np.nan, gprev))
    X = fs.features(torch.from_numpy(psi).cuda()).cpu().numpy()
    occ_ref = oracle.occupations(M, na, nb, psi)
    assert np.abs(fs.occ.cpu().numpy() - occ_ref).max() < 1e-13
    assert abs(occ_ref[:M].sum() - na) < 1e-12 and abs(occ_ref[M:].sum() - nb) < 1e-12
    # reference g_prev / age after the two updates
    gp = np.zeros(len(cre))
    age = np.full(len(cre), 50)
    for gg in (gprev, np.where(np.arange(len(cre)) % 3 == 0, np.nan, gprev)):
        ok = ~np.isnan(gg)
        gp[ok] = gg[ok]
        age = np.where(ok, 0, age + 1)
    F, Q = om.static_features(M, cre, ann, cls, h, g)
    ref = om.bf16(om.features(F, Q, occ_ref, gp, age))
    got = (X.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    diff = np.abs(got - ref)
    assert np.all(diff <= np.abs(ref) * 2 ** -7 + 1e-30)
    assert np.mean(diff == 0) > 0.999


def test_mlp_state_roundtrip_and_clone(scr):
    """A clone continues training exactly like the original (parameters and
    Adam state), and set_state rejects a bad step count."""
    rng = np.random.default_rng(6)
    X = torch.from_numpy(_bf16_bits(rng.standard_normal((64, om.N_FEAT)))).cuda()
    t = torch.from_numpy(rng.standard_normal(64).astype(np.float32)).cuda()
    a = scr.MLP(synth.mlp_init(2), 128)
    for _ in range(3):
        a.train_step(X, t, lr=1e-3)
    b = a.clone()
    assert np.array_equal(a.state(), b.state())
    a.train_step(X, t, lr=1e-3)
    b.train_step(X, t, lr=1e-3)
    assert np.array_equal(a.params(), b.params())
    assert np.array_equal(a.forward(X).cpu().numpy(), b.forward(X).cpu().numpy())
    st = a.state()
    st[-1] = -1.0
    with pytest.raises(Exception):
        b.load_state(st)


def test_rank_scores(scr):
    net = scr.MLP(synth.mlp_init(0), 64)
    y = np.round(np.random.default_rng(4).standard_normal(5000), 1).astype(np.float32)
    order = net.rank(torch.from_numpy(y).cuda()).cpu().numpy()
    assert np.array_equal(order, np.argsort(-y, kind="stable"))


def _train_on(hyp, scr, workloads, n_iter, epochs, seed=0):
    Xs, ts = [], []
    for i, w in enumerate(workloads):
        x, z, c, h, g = synth.hamiltonian(w)
        cre, ann, cls = synth.canonical_pool(w.n_orb)
        S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        A = hyp.Adapt(H, cre, ann, max_iter=n_iter + 1)
        stat, qidx = scr.static_features(w.n_orb, cre, ann, cls, h, g)
        fs = scr.FeatureState(S, stat, qidx)
        X, t = scr.collect_rows(A, fs, n_iter, seed=i)
        Xs.append(X)
        ts.append(t)
    X = np.concatenate(Xs)
    t = np.concatenate(ts)
    assert np.all(np.isfinite(t))
    net = scr.MLP(synth.mlp_init(seed), 1 << 16)
    losses = scr.train(net, X, t, epochs=epochs, batch=1024, lr=1e-3)
    return net, losses


@pytest.fixture(scope="module")
def trained(hyp, scr):
    """Trained on the 8-qubit workload and six of the eight batch instances
    (M = 8..12); the 16-qubit workload and instance 3 are held out."""
    wl = [synth.WORKLOADS["h4_8q"]] + [synth.INSTANCES[i] for i in (0, 1, 2, 4, 5, 6, 7)]
    net, losses = _train_on(hyp, scr, wl, 8, epochs=16)
    print("training loss per epoch:", [round(l, 4) for l in losses])
    assert losses[-1] < 0.5 * losses[0]
    return net


def test_training_rows_and_floored_targets(hyp, scr):
    w = synth.WORKLOADS["h4_8q"]
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, cls = synth.canonical_pool(w.n_orb)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    stat, qidx = scr.static_features(w.n_orb, cre, ann, cls, h, g)
    fs = scr.FeatureState(S, stat, qidx)
    rng = np.random.default_rng(1)
    g_prev = rng.standard_normal(len(cre)) * 10.0 ** rng.uniform(-9, 0, len(cre))
    g_new = rng.standard_normal(len(cre)) * 10.0 ** rng.uniform(-9, 0, len(cre))
    g_prev[3] = 0.0
    g_new[5] = 0.0
    fs.update(g_prev)
    X = fs.features(torch.from_numpy(synth.random_state(S.dim, 1)).cuda())
    base_ref = np.maximum(np.log10(np.abs(g_prev) + 1e-12), scr.T_FLOOR)
    assert np.abs(fs.base.cpu().numpy() - base_ref).max() <= 2e-6 * np.abs(base_ref).max()
    fs.update(g_new)
    idx = np.arange(len(cre))[::-1].copy()
    t_abs = np.maximum(np.log10(np.abs(g_new[idx]) + 1e-12), scr.T_FLOOR)
    Xo, t = fs.rows(idx, residual=False)
    assert np.abs(t.cpu().numpy() - t_abs).max() <= 2e-6 * np.abs(t_abs).max()
    assert np.array_equal(Xo.cpu().numpy(), X.cpu().numpy()[idx])
    _, tr = fs.rows(idx)
    assert np.abs(tr.cpu().numpy() - (t_abs - base_ref[idx])).max() <= 4e-6 * np.abs(t_abs).max()
    # ranking by y + base
    net = scr.MLP(synth.mlp_init(0), 256)
    y = torch.from_numpy(np.round(rng.standard_normal(len(cre)), 1).astype(np.float32)).cuda()
    order = net.rank(y, fs.base).cpu().numpy()
    key = (y.cpu().numpy() + fs.base.cpu().numpy()).astype(np.float32)
    assert np.array_equal(order, np.argsort(-key, kind="stable"))
    keep = scr.training_rows(t_abs, np.random.default_rng(0))
    top = np.nonzero(t_abs >= t_abs.max() - scr.BAND)[0]
    assert set(top.tolist()) <= set(keep.tolist())
    assert keep.size == top.size + max(1, int((t_abs.size - top.size) * scr.REST_FRAC))


def test_ablation_recall(hyp, scr, trained):
    """Held-out problems: where the true argmax |g| ranks under the trained
    network, under the no-learning heuristic (|g_prev|) and at random."""
    net = trained
    K = 32
    hits = {"mlp": 0, "heuristic": 0, "random": 0}
    total = 0
    rng = np.random.default_rng(9)
    for w in (synth.WORKLOADS["h8_16q"], synth.INSTANCES[3]):
        x, z, c, h, g = synth.hamiltonian(w)
        cre, ann, cls = synth.canonical_pool(w.n_orb)
        S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        A = hyp.Adapt(H, cre, ann, max_iter=12)
        stat, qidx = scr.static_features(w.n_orb, cre, ann, cls, h, g)
        fs = scr.FeatureState(S, stat, qidx)
        psi = None
        for it in range(10):
            psi = A.state(psi)
            X = fs.features(psi)
            heur = fs.gprev.abs().cpu().numpy()
            y = net.forward(X).cpu().numpy() + fs.base.cpu().numpy()
            A.gradients(None)
            gfull = A.last_gradients()
            fs.update(gfull)
            A.select_optimize()
            if it == 0:
                continue  # no g_prev yet
            kstar = int(np.argmax(np.abs(gfull)))
            total += 1
            hits["mlp"] += kstar in set(np.argsort(-y, kind="stable")[:K].tolist())
            hits["heuristic"] += kstar in set(np.argsort(-heur, kind="stable")[:K].tolist())
            hits["random"] += kstar in set(rng.choice(len(cre), K, replace=False).tolist())
    rec = {k: v / total for k, v in hits.items()}
    print(f"recall@32 of the exact argmax over {total} iterations:", rec)
    assert total >= 16
    assert rec["mlp"] >= 0.75
    assert rec["mlp"] > rec["random"] + 0.5
    assert rec["mlp"] >= rec["heuristic"] - 1.0 / total


@pytest.mark.parametrize("K,audit,online,min_agree", [(512, 256, True, 9), (512, 256, False, 6),
                                                      (128, 64, True, 6)])
def test_screened_adapt_fp32_vs_full_sweep(hyp, scr, trained, K, audit, online, min_agree):
    """Screened FP32 ADAPT on the 16-qubit workload (pool 2,044; top-K plus
    an audit sample, judge every 5th iteration), judged by the full sweep on
    its own state at every iteration, and its energy trajectory against a
    plain FP64 full-sweep run from the same start.  K = 512 + 256 is the
    deployed setting; K = 128 + 64 (9% of the pool) is the harder check."""
    w = synth.WORKLOADS["h8_16q"]
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, cls = synth.canonical_pool(w.n_orb)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    n_iter = 10
    A32 = hyp.Adapt(H, cre, ann, dtype="f32", max_iter=n_iter + 1)
    stat, qidx = scr.static_features(w.n_orb, cre, ann, cls, h, g)
    net = trained.clone()  # online training must not leak into other tests
    sc = scr.Screen(A32, S, stat, qidx, net, K=K, audit=audit, judge_every=5, seed=42, online=online,
                    cost_policy=False)
    A64 = hyp.Adapt(H, cre, ann, max_iter=n_iter + 1)
    agree_own, agree_plain, e32, e64 = 0, 0, [], []
    for it in range(n_iter):
        info = sc.iterate(it, shadow=True)
        r64 = A64.iterate()
        assert info["selected"] >= 0
        agree_own += info["shadow_agree"]
        agree_plain += info["selected"] == r64["selected"]
        e32.append(info["energy"])
        e64.append(r64["energy"])
    print("screened picks in the full sweep's tie set on the same state:", agree_own, "/", n_iter)
    print("per iteration (judge, fallback, true argmax in candidates, its rank by score):",
          [(r["judge"], r["fallback"], r.get("shadow_in_candidates"), r.get("shadow_rank")) for r in sc.log])
    print("screened picks equal to the plain FP64 run's:", agree_plain, "/", n_iter)
    print("energy trajectories (screened FP32, plain FP64):", list(zip(e32, e64)))
    assert agree_own >= min_agree
    assert e32[-1] < e32[0] - 1.0           # the screened run makes progress
    if agree_own == n_iter:                 # same picks on every state: same trajectory
        assert abs(e32[-1] - e64[-1]) <= 1e-4
    if agree_plain == n_iter:
        assert abs(A32.energy_fp64() - A64.energy_fp64()) < 1e-6
    # the oracle's energy of the screened ansatz (plain definition, FP64)
    ops, th = A32.ansatz()
    from oracle.adapt import SectorProblem
    prob = SectorProblem(w.n_orb, w.n_alpha, w.n_beta, x, z, c, cre, ann)
    psi = prob.state(list(ops), th)
    e_orc = oracle.dot(psi, prob.hpsi(psi))
    assert abs(A32.energy_fp64() - e_orc) < 1e-9
    n_exact = [r["n_exact"] for r in sc.log]
    assert min(n_exact) <= K + audit < len(cre)
