"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Index work is bit-exact; FP64 amplitudes must match to
||d sigma|| / ||sigma|| <= 1e-12 and |dE| <= 1e-9 Ha; FP32 storage within the
rounding bound of single precision."""
import math

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


def _ham(hyp, M, na, nb, seed=42):
    h, g = synth.integrals(M, seed)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    return S, H, (x, z, c)


def _dev(v, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)


# ------------------------------------------------------------- indexing

@pytest.mark.parametrize("M,na,nb", [(1, 0, 1), (4, 2, 2), (6, 1, 4), (8, 4, 4), (9, 5, 4), (16, 8, 8)])
def test_rank_unrank_bit_exact(hyp, M, na, nb):
    S = hyp.Sector(M, na, nb)
    assert S.dim == oracle.sector_dim(M, na, nb)
    rng = np.random.default_rng(M)
    idx = np.arange(S.dim) if S.dim <= 100_000 else rng.integers(0, S.dim, 200_000)
    bits = S.unrank(idx)
    assert np.array_equal(bits, oracle.unrank(M, na, nb, idx))
    assert np.array_equal(S.rank(bits), idx)
    junk = rng.integers(0, 1 << min(2 * M, 31), 1000).astype(np.uint32)
    assert np.array_equal(S.rank(junk), oracle.rank(M, na, nb, junk))


# ------------------------------------------------------------- H psi

CASES = [(4, 2, 2), (5, 3, 2), (6, 3, 3), (7, 2, 5), (8, 4, 4), (9, 5, 4), (10, 5, 5), (3, 0, 2), (4, 4, 1)]


@pytest.mark.parametrize("M,na,nb", CASES)
def test_apply_h_fp64_full(hyp, M, na, nb):
    S, H, (x, z, c) = _ham(hyp, M, na, nb, seed=100 + M)
    assert H.structured
    psi = synth.random_state(S.dim, 7)
    ref = oracle.apply_h(M, na, nb, x, z, c, psi)
    out = H.apply(_dev(psi)).cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
    e_gpu = hyp.hyp_expectation(S, _dev(psi), _dev(out)).item()
    assert abs(e_gpu - oracle.dot(psi, ref)) < 1e-9


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (8, 4, 4), (9, 5, 4)])
def test_apply_h_fp32(hyp, M, na, nb):
    S, H, (x, z, c) = _ham(hyp, M, na, nb)
    psi = synth.random_state(S.dim, 7)
    psi32 = psi.astype(np.float32)
    ref = oracle.apply_h(M, na, nb, x, z, c, psi32.astype(np.float64))
    out = H.apply(_dev(psi32, torch.float32)).cpu().numpy().astype(np.float64)
    # each term: coefficient and product rounded to FP32 (2 * 2^-24 relative),
    # FP64 sums, one final FP32 store; sum|terms| / |sigma| is O(10) here
    assert np.linalg.norm(out - ref) <= 2e-6 * np.linalg.norm(ref)


def test_generic_path_arbitrary_pauli_sum(hyp):
    """A real Pauli sum with particle-number-breaking and three-body terms
    takes the generic kernel (P_S H P_S)."""
    M, na, nb = 4, 2, 1
    rng = np.random.default_rng(5)
    n = 2 * M
    xs, zs = [], []
    while len(xs) < 300:
        xx, zz = (int(v) for v in rng.integers(0, 1 << n, 2))
        if bin(xx & zz).count("1") % 2 == 0:
            xs.append(xx)
            zs.append(zz)
    x = np.array(xs, dtype=np.uint32)
    z = np.array(zs, dtype=np.uint32)
    c = rng.standard_normal(len(xs))
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    assert not H.structured
    psi = synth.random_state(S.dim, 3)
    ref = oracle.apply_h(M, na, nb, x, z, c, psi)
    out = H.apply(_dev(psi)).cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)


def test_apply_h_24q_sampled_rows(hyp):
    w = synth.WORKLOADS["h12_24q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    psi = synth.random_state(S.dim, 7)
    out = H.apply(_dev(psi)).cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([[0, S.dim - 1], rng.integers(0, S.dim, 300)]))
    ref = oracle.apply_h(w.n_orb, w.n_alpha, w.n_beta, x, z, c, psi, out_idx=idx)
    assert np.abs(out[idx] - ref).max() <= 1e-12 * np.linalg.norm(ref) / math.sqrt(len(idx)) * 10
    # Hermiticity at full size: <phi|H psi> = <H phi|psi>
    phi = synth.random_state(S.dim, 8)
    hphi = H.apply(_dev(phi)).cpu().numpy()
    a, b = float(phi @ out), float(hphi @ psi)
    assert abs(a - b) <= 1e-12 * (abs(a) + 1)


def test_empty_hamiltonian_and_constant(hyp):
    S = hyp.Sector(3, 1, 2)
    H = hyp.Hamiltonian(S, np.array([0], dtype=np.uint32), np.array([0], dtype=np.uint32),
                        np.array([2.5]))
    psi = synth.random_state(S.dim, 1)
    out = H.apply(_dev(psi)).cpu().numpy()
    assert np.allclose(out, 2.5 * psi, rtol=0, atol=1e-15)
    H0 = hyp.Hamiltonian(S, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0))
    assert np.all(H0.apply(_dev(psi)).cpu().numpy() == 0.0)


def test_build_errors(hyp):
    S = hyp.Sector(3, 1, 1)
    with pytest.raises(hyp.HypError) as e:
        hyp.Hamiltonian(S, np.array([1], np.uint32), np.array([1], np.uint32), np.array([1.0]))
    assert e.value.status == 3  # odd n_Y
    with pytest.raises(hyp.HypError) as e:
        hyp.Hamiltonian(S, np.array([1 << 6], np.uint32), np.array([0], np.uint32), np.array([1.0]))
    assert e.value.status == 1  # bit beyond 2M
    psi = _dev(np.zeros(S.dim))
    H = hyp.Hamiltonian(S, np.array([0], np.uint32), np.array([0], np.uint32), np.array([1.0]))
    with pytest.raises(hyp.HypError):
        hyp.hyp_apply_h(H, psi, psi)  # aliasing


# ------------------------------------------------------------- gradients / rotations

@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 2, 3), (8, 4, 4)])
def test_pool_gradients_fp64(hyp, M, na, nb):
    S, H, (x, z, c) = _ham(hyp, M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    psi = synth.random_state(S.dim, 11)
    sig = oracle.apply_h(M, na, nb, x, z, c, psi)
    ref = oracle.pool_gradients(M, na, nb, cre, ann, psi, sig)
    ops = hyp.exc_tensor(cre, ann)
    g = hyp.hyp_pool_gradients(S, ops, _dev(psi), _dev(sig)).cpu().numpy()
    assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_pool_gradients_24q_subset(hyp):
    w = synth.WORKLOADS["h12_24q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, cls = synth.canonical_pool(w.n_orb)
    rng = np.random.default_rng(3)
    pick = np.unique(np.concatenate([np.nonzero(cls == k)[0][:3] for k in range(5)] +
                                    [rng.integers(0, len(cre), 40)]))
    psi = synth.random_state(S.dim, 11)
    sig_d = H.apply(_dev(psi))
    sig = sig_d.cpu().numpy()
    ref = oracle.pool_gradients(w.n_orb, w.n_alpha, w.n_beta, cre[pick], ann[pick], psi, sig)
    g_all = hyp.hyp_pool_gradients(S, hyp.exc_tensor(cre, ann), _dev(psi), sig_d).cpu().numpy()
    assert np.abs(g_all[pick] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 3, 2), (8, 4, 4)])
def test_rotations_fp64(hyp, M, na, nb):
    S = hyp.Sector(M, na, nb)
    cre, ann, cls = synth.canonical_pool(M)
    psi = synth.random_state(S.dim, 4)
    d = _dev(psi)
    ref = psi.copy()
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([np.nonzero(cls == k)[0][:4] for k in range(5)] +
                                  [rng.integers(0, len(cre), 10)]))
    for i, k in enumerate(ks):
        th = 0.37 * (i + 1)
        ref = oracle.rotate(M, na, nb, cre[k], ann[k], th, ref)
        hyp.hyp_apply_excitation(S, int(cre[k]), int(ann[k]), th, d)
    out = d.cpu().numpy()
    assert np.abs(out - ref).max() <= 1e-13
    assert abs(np.linalg.norm(out) - 1.0) < 1e-13


def test_rotation_errors(hyp):
    S = hyp.Sector(4, 2, 2)
    d = _dev(np.zeros(S.dim))
    with pytest.raises(hyp.HypError) as e:
        hyp.hyp_apply_excitation(S, 0b0001_0000, 0b0000_0001, 0.1, d)  # alpha -> beta
    assert e.value.status == 2
    with pytest.raises(hyp.HypError) as e:
        hyp.hyp_apply_excitation(S, 0b11, 0b1, 0.1, d)
    assert e.value.status == 1
    with pytest.raises(hyp.HypError):
        hyp.hyp_apply_excitation(S, 0b10, 0b10, 0.1, d)


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (5, 2, 3), (6, 3, 3), (8, 4, 4), (9, 5, 4), (3, 0, 2), (4, 4, 1),
                                     (7, 3, 2), (10, 4, 5), (2, 1, 1)])
def test_pool_gradients_transition_values(hyp, M, na, nb):
    """The transition-value sweep (forced) against the oracle and the pair kernel."""
    S, H, (x, z, c) = _ham(hyp, M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    psi = synth.random_state(S.dim, 13)
    sig = oracle.apply_h(M, na, nb, x, z, c, psi)
    ref = oracle.pool_gradients(M, na, nb, cre, ann, psi, sig)
    ops = hyp.exc_tensor(cre, ann)
    try:
        res = {}
        for mode in ("tdens", "tdens_bins"):
            hyp.set_sweep_mode(mode)
            res[mode] = (hyp.hyp_pool_gradients(S, ops, _dev(psi), _dev(sig)).cpu().numpy(),
                         hyp.hyp_pool_gradients(S, ops, _dev(psi, torch.float32),
                                                _dev(sig, torch.float32)).cpu().numpy())
        hyp.set_sweep_mode("pairs")
        gp = hyp.hyp_pool_gradients(S, ops, _dev(psi), _dev(sig)).cpu().numpy()
    finally:
        hyp.set_sweep_mode("auto")
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(gp - ref).max() <= 1e-12 * scale
    for mode, (g, g32) in res.items():
        assert np.abs(g - ref).max() <= 1e-12 * scale, mode
        assert np.abs(g32 - ref).max() <= 1e-5 * scale, mode


def test_pool_gradients_24q_full_sweep_modes(hyp):
    """Full 24-qubit sweep: transition values vs the pair kernel (all 11,814
    generators), and the oracle on a sample."""
    w = synth.WORKLOADS["h12_24q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    psi = synth.random_state(S.dim, 17)
    d_psi = _dev(psi)
    d_sig = H.apply(d_psi)
    ops = hyp.exc_tensor(cre, ann)
    try:
        hyp.set_sweep_mode("tdens_bins")
        g_b = hyp.hyp_pool_gradients(S, ops, d_psi, d_sig).cpu().numpy()
        hyp.set_sweep_mode("tdens")
        g_t = hyp.hyp_pool_gradients(S, ops, d_psi, d_sig).cpu().numpy()
        hyp.set_sweep_mode("pairs")
        g_p = hyp.hyp_pool_gradients(S, ops, d_psi, d_sig).cpu().numpy()
    finally:
        hyp.set_sweep_mode("auto")
    assert np.abs(g_t - g_p).max() <= 1e-12 * max(1.0, np.abs(g_p).max())
    assert np.abs(g_b - g_p).max() <= 1e-12 * max(1.0, np.abs(g_p).max())
    k = np.random.default_rng(5).choice(len(cre), 12, replace=False)
    ref = oracle.pool_gradients(w.n_orb, w.n_alpha, w.n_beta, cre[k], ann[k], psi, d_sig.cpu().numpy())
    assert np.abs(g_t[k] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_apply_h_autotuner_keeps_parity(hyp):
    M, na, nb = 10, 5, 5
    S, H, (x, z, c) = _ham(hyp, M, na, nb, seed=110)
    psi = synth.random_state(S.dim, 7)
    d = _dev(psi)
    t, ms = H.tune(d, reps=1)
    assert 64 <= t <= 1024 and t % 64 == 0 and ms > 0
    ref = oracle.apply_h(M, na, nb, x, z, c, psi)
    out = H.apply(d).cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
