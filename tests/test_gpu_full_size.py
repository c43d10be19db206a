"""Parity at the 32-qubit workload's full size (sector (8, 8), dim 165,636,900,
94,849 Pauli terms, pool 39,960), in the launch configuration the benchmark
times.

* A sparse input state makes the oracle's sigma cheap (every term pushed
  from every nonzero), so sigma, the energy and the rotations are compared
  element by element over all 165,636,900 entries.  The kernels' control
  flow does not depend on the values, so this exercises every tile and the
  ragged tail of every row.
* The benchmark's dense random state: sigma on sampled rows (the oracle's
  term-by-term sum per row), including the first and last rows and both
  edges of the column chunks.
* The full pool-gradient sweep in all three strategies against each other
  and, on a sample of generators, against the oracle.
* With support skipping off (every kernel evaluates the whole sector, the
  dense path the benchmark times): sigma over all 165,636,900 entries (FP64
  and FP32) and all 39,960 gradients of the default sweep (compact staging,
  per-core Gram blocks over the full contraction range) on the sparse input,
  against the oracle's pair sum restricted to the input's nonzeros (exact:
  every other pair contributes 0).
* Dense operands: the sweep of a dense random psi with an independent dense
  random sigma (the gradient is defined for any pair of vectors), 64
  generators of every class against the oracle's full pair sum.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = synth.WORKLOADS["h16_32q"]


@pytest.fixture(scope="module")
def hyp():
    import paper_2604_01176_amd as hyp
    return hyp


@pytest.fixture(scope="module")
def prob(hyp):
    x, z, c, _, _ = synth.hamiltonian(W)
    S = hyp.Sector(W.n_orb, W.n_alpha, W.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    assert H.structured
    idx, val = synth.sparse_state(S.dim, S.da)
    print(f"[full-size] dim {S.dim}, sparse input with {idx.size} nonzeros", flush=True)
    sig_ref = oracle.apply_h_sparse(W.n_orb, W.n_alpha, W.n_beta, x, z, c, idx, val)
    return dict(S=S, H=H, x=x, z=z, c=c, idx=idx, val=val, sig_ref=sig_ref)


def _sparse_dev(S, idx, val, dtype=torch.float64):
    d = torch.zeros(S.dim, dtype=dtype, device="cuda")
    d[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).to(dtype).cuda()
    return d


def _full(S, idx, val):
    v = np.zeros(S.dim)
    v[idx] = val
    return v


@pytest.fixture
def skip_off(hyp):
    hyp.set_support_skip(False)
    yield
    hyp.set_support_skip(True)


def test_hpsi_32q_sparse_input_every_entry(hyp, prob):
    S, H = prob["S"], prob["H"]
    psi = _sparse_dev(S, prob["idx"], prob["val"])
    sig = H.apply(psi).cpu().numpy()
    ref = prob["sig_ref"]
    nz = np.count_nonzero(ref)
    print(f"[full-size] oracle sigma has {nz} nonzeros", flush=True)
    assert nz > 100000
    assert np.linalg.norm(sig - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.abs(sig - ref).max() <= 1e-12 * np.abs(ref).max()
    # rows outside the oracle's support are exactly zero on the GPU too
    assert np.count_nonzero(sig[ref == 0.0]) == 0
    # energy <psi|sigma> / <psi|psi>
    e = hyp.hyp_expectation(S, psi, H.apply(psi)).item()
    e_ref = float(np.dot(prob["val"], ref[prob["idx"]]))
    assert abs(e - e_ref) <= 1e-9


def test_hpsi_32q_sparse_input_fp32(hyp, prob):
    S, H = prob["S"], prob["H"]
    psi = _sparse_dev(S, prob["idx"], prob["val"], torch.float32)
    sig = H.apply(psi).cpu().numpy().astype(np.float64)
    ref = prob["sig_ref"]
    assert np.linalg.norm(sig - ref) <= 2e-6 * np.linalg.norm(ref)


def test_hpsi_32q_benchmark_state_sampled_rows(hyp, prob):
    S, H = prob["S"], prob["H"]
    psi_h = synth.random_state(S.dim, 7)
    sig = H.apply(torch.from_numpy(psi_h).cuda())
    da = S.da
    rng = np.random.default_rng(3)
    rows = [0, 1, S.dim - 1, S.dim - 2, 511, 512, 767, 768, 1023, 1024, 1535, 1536, 12287, 12288,
            da - 1, da, 6 * da + 12799, 12869 * da + 1]
    rows += rng.choice(S.dim, 36, replace=False).tolist()
    rows = np.unique(np.array(rows, dtype=np.int64))
    got = sig[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = oracle.apply_h(W.n_orb, W.n_alpha, W.n_beta, prob["x"], prob["z"], prob["c"], psi_h, out_idx=rows)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_sweep_32q_all_strategies_and_oracle_sample(hyp, prob):
    S, H = prob["S"], prob["H"]
    cre, ann, cls = synth.canonical_pool(W.n_orb)
    ops = hyp.exc_tensor(cre, ann)
    psi = _sparse_dev(S, prob["idx"], prob["val"])
    sig = H.apply(psi)
    g = {}
    try:
        for mode in ("auto", "tdens", "tdens_bins", "pairs"):
            hyp.set_sweep_mode(mode)
            g[mode] = hyp.hyp_pool_gradients(S, ops, psi, sig).cpu().numpy()
            print(f"[full-size] sweep mode {mode} done", flush=True)
    finally:
        hyp.set_sweep_mode("auto")
    scale = max(1.0, np.abs(g["pairs"]).max())
    for mode in ("auto", "tdens", "tdens_bins"):
        assert np.abs(g[mode] - g["pairs"]).max() <= 1e-12 * scale, mode
    # oracle on a sample: the largest gradients and random ones of every class
    rng = np.random.default_rng(4)
    pick = list(np.argsort(-np.abs(g["auto"]), kind="stable")[:6])
    for k in range(5):
        members = np.nonzero(cls == k)[0]
        pick += rng.choice(members, 2, replace=False).tolist()
    pick = np.array(sorted(set(int(p) for p in pick)))
    psi_full = _full(S, prob["idx"], prob["val"])
    ref = oracle.pool_gradients(W.n_orb, W.n_alpha, W.n_beta, cre[pick], ann[pick], psi_full, prob["sig_ref"])
    assert np.abs(ref).max() > 1e-3
    assert np.abs(g["auto"][pick] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("cls_pick", [0, 4])
def test_rotation_32q_every_entry(hyp, prob, cls_pick):
    S = prob["S"]
    cre, ann, cls = synth.canonical_pool(W.n_orb)
    k = int(np.nonzero(cls == cls_pick)[0][0])
    psi = _sparse_dev(S, prob["idx"], prob["val"])
    hyp.hyp_apply_excitation(S, int(cre[k]), int(ann[k]), 0.37, psi)
    got = psi.cpu().numpy()
    ref = oracle.rotate(W.n_orb, W.n_alpha, W.n_beta, int(cre[k]), int(ann[k]), 0.37, _full(S, prob["idx"], prob["val"]))
    assert np.abs(got - ref).max() <= 1e-13
    assert np.count_nonzero(ref) > np.size(prob["idx"])  # the rotation moved weight


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hpsi_32q_skip_off_every_entry(hyp, prob, skip_off, dtype):
    S, H = prob["S"], prob["H"]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    psi = _sparse_dev(S, prob["idx"], prob["val"], tdt)
    print(f"[full-size] H psi {dtype}, support skipping off", flush=True)
    sig = H.apply(psi).cpu().numpy().astype(np.float64)
    ref = prob["sig_ref"]
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert np.linalg.norm(sig - ref) <= tol * np.linalg.norm(ref)
    if dtype == "f64":
        assert np.abs(sig - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.count_nonzero(sig[ref == 0.0]) == 0


def test_sweep_32q_skip_off_every_gradient(hyp, prob, skip_off):
    S = prob["S"]
    cre, ann, _ = synth.canonical_pool(W.n_orb)
    ops = hyp.exc_tensor(cre, ann)
    psi = _sparse_dev(S, prob["idx"], prob["val"])
    sig = torch.from_numpy(prob["sig_ref"]).cuda()  # the oracle's sigma as the input
    print("[full-size] sweep, support skipping off", flush=True)
    g = hyp.hyp_pool_gradients(S, ops, psi, sig).cpu().numpy()
    ref = oracle.pool_gradients_sparse(W.n_orb, W.n_alpha, W.n_beta, cre, ann, prob["idx"],
                                       _full(S, prob["idx"], prob["val"]), prob["sig_ref"])
    assert np.count_nonzero(ref) > 1000
    assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_sweep_32q_dense_operands_oracle_sample(hyp, prob):
    S = prob["S"]
    cre, ann, cls = synth.canonical_pool(W.n_orb)
    ops = hyp.exc_tensor(cre, ann)
    psi_h = synth.random_state(S.dim, 7)
    sig_h = synth.random_state(S.dim, 8)
    print("[full-size] sweep on dense random psi and sigma", flush=True)
    g = hyp.hyp_pool_gradients(S, ops, torch.from_numpy(psi_h).cuda(), torch.from_numpy(sig_h).cuda())
    g = g.cpu().numpy()
    rng = np.random.default_rng(5)
    pick = list(np.argsort(-np.abs(g), kind="stable")[:4])
    for k in range(5):
        members = np.nonzero(cls == k)[0]
        pick += [int(members[0]), int(members[-1])] + rng.choice(members, 14, replace=False).tolist()
    pick = np.array(sorted(set(int(p) for p in pick)))
    assert pick.size >= 64
    print(f"[full-size] oracle on {pick.size} generators", flush=True)
    ref = oracle.pool_gradients(W.n_orb, W.n_alpha, W.n_beta, cre[pick], ann[pick], psi_h, sig_h)
    assert np.abs(g[pick] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
