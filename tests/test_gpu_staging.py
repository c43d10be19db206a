"""GPU parity of the compact, double-buffered row staging of the FP64
transition-value sweep and mixed pass: gradients and sigma equal those of
whole-row staging bit for bit (the products and their order are the same),
the oracle on samples of generators and rows, the fallbacks (odd alpha
dimension, chunks below 512 columns, FP32), support skipping, and the
32-qubit sweep and product both ways."""
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
    yield hyp
    hyp.set_row_staging("compact")
    hyp.set_sweep_mode("auto")
    hyp.set_support_skip(True)


def _dev(v, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)


def _grads(hyp, S, ops, psi, sig, staging):
    # the two staging forms of the row-batched kernel (the matrix-core form
    # switched off)
    try:
        hyp.set_mixed_matrix_cores(False)
        hyp.set_sweep_mode("tdens")
        hyp.set_row_staging(staging)
        return hyp.hyp_pool_gradients(S, ops, psi, sig).cpu().numpy()
    finally:
        hyp.set_row_staging("compact")
        hyp.set_sweep_mode("auto")
        hyp.set_mixed_matrix_cores()


# (11,5), (12,6), (12,5), (13,6), (14,7): even alpha dimension above 448,
# compact staging; (13,5), (14,4): odd alpha dimension, whole rows; (10,5):
# 256-column chunks, whole rows; N_beta = 0 and N_beta = M: no beta singles
# (no stages, one identity slice)
CASES = [(11, 5, 5), (11, 5, 3), (12, 6, 6), (12, 5, 4), (13, 6, 2), (13, 5, 1), (14, 7, 1), (10, 5, 5), (14, 4, 2),
         (12, 6, 0), (12, 5, 12)]


@pytest.mark.parametrize("M,na,nb", CASES)
def test_compact_staging_bit_exact_and_oracle(hyp, M, na, nb):
    h, g = synth.integrals(M, 300 + M)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(M)
    ops = hyp.exc_tensor(cre, ann)
    psi = _dev(synth.random_state(S.dim, 31 + M))
    sig = H.apply(psi)
    g_c = _grads(hyp, S, ops, psi, sig, "compact")
    g_r = _grads(hyp, S, ops, psi, sig, "rows")
    assert np.array_equal(g_c, g_r)
    k = np.random.default_rng(M + na).choice(cre.size, 10, replace=False)
    ref = oracle.pool_gradients(M, na, nb, cre[k], ann[k], psi.cpu().numpy(), sig.cpu().numpy())
    assert np.abs(g_c[k] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_compact_staging_fp32_unchanged(hyp):
    M, na, nb = 12, 6, 4
    h, g = synth.integrals(M, 7)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(M)
    ops = hyp.exc_tensor(cre, ann)
    psi = _dev(synth.random_state(S.dim, 5), torch.float32)
    sig = H.apply(psi)
    assert np.array_equal(_grads(hyp, S, ops, psi, sig, "compact"), _grads(hyp, S, ops, psi, sig, "rows"))


def test_compact_staging_with_support_skipping(hyp):
    """Near-Hartree-Fock state (kept row pairs and identity lists in LDS):
    both stagings with skipping on, bit for bit, and against the dense sweep."""
    M, na, nb = 12, 6, 6
    h, g = synth.integrals(M, 12)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(M)
    ops = hyp.exc_tensor(cre, ann)
    idx = np.unique(oracle.rank(M, na, nb, synth.near_hf_bits(M, na, nb, 24, seed=5)))
    val = np.random.default_rng(2).standard_normal(idx.size)
    val /= np.linalg.norm(val)
    psi = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
    psi[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).cuda()
    sig = H.apply(psi)
    try:
        hyp.set_support_skip(True)
        g_c = _grads(hyp, S, ops, psi, sig, "compact")
        g_r = _grads(hyp, S, ops, psi, sig, "rows")
        hyp.set_support_skip(False)
        g_d = _grads(hyp, S, ops, psi, sig, "compact")
    finally:
        hyp.set_support_skip(True)
    assert np.array_equal(g_c, g_r)
    assert np.abs(g_c - g_d).max() <= 1e-13 * max(1.0, np.abs(g_d).max())
    assert np.abs(g_c).max() > 0.0


def test_row_staging_argument_check(hyp):
    from paper_2604_01176_amd import _lib
    assert _lib.load().hyp_set_row_staging(2) != 0
    assert _lib.load().hyp_set_row_staging(-1) != 0
    assert _lib.load().hyp_set_row_staging(0) == 0


def test_compact_staging_32q(hyp):
    """32-qubit full sweep (39,960 generators) both ways, bit for bit, and
    the transition-value phase timed."""
    w = synth.WORKLOADS["h16_32q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    ops = hyp.exc_tensor(cre, ann)
    psi = _dev(synth.random_state(S.dim, 3))
    sig = H.apply(psi)
    out, times = {}, {}
    for staging in ("compact", "rows"):
        out[staging] = _grads(hyp, S, ops, psi, sig, staging)  # first call builds the tables
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _grads(hyp, S, ops, psi, sig, staging)
        torch.cuda.synchronize()
        times[staging] = (time.perf_counter() - t0) * 1e3
    print(f"[staging] 32q full sweep: compact {times['compact']:.1f} ms, whole rows {times['rows']:.1f} ms",
          flush=True)
    assert np.array_equal(out["compact"], out["rows"])
    del psi, sig
    torch.cuda.empty_cache()


def _apply(hyp, H, psi, staging):
    # the two staging forms of k_mixed / k_mixed_c (the matrix-core form,
    # which reproduces sigma to rounding only, switched off)
    try:
        hyp.set_mixed_matrix_cores(False)
        hyp.set_row_staging(staging)
        out = H.apply(psi)
        torch.cuda.synchronize()
        return out
    finally:
        hyp.set_row_staging("compact")
        hyp.set_mixed_matrix_cores()


@pytest.mark.parametrize("M,na,nb", CASES)
def test_compact_mixed_pass_bit_exact_and_oracle(hyp, M, na, nb):
    """H psi with the compact, double-buffered mixed pass (FP64, 512-column
    chunks) equals the whole-row mixed pass bit for bit, and the oracle on
    sampled rows."""
    h, g = synth.integrals(M, 400 + M)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    p = synth.random_state(S.dim, 41 + M)
    psi = _dev(p)
    s_c = _apply(hyp, H, psi, "compact")
    s_r = _apply(hyp, H, psi, "rows")
    assert torch.equal(s_c, s_r)
    rng = np.random.default_rng(M * 7 + nb)
    idx = np.unique(np.concatenate([[0, S.dim - 1], rng.integers(0, S.dim, 150)]))
    ref = oracle.apply_h(M, na, nb, x, z, c, p, out_idx=idx)
    assert np.abs(s_c.cpu().numpy()[idx] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_compact_mixed_pass_with_support_skipping(hyp):
    M, na, nb = 12, 6, 6
    h, g = synth.integrals(M, 13)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    idx = np.unique(oracle.rank(M, na, nb, synth.near_hf_bits(M, na, nb, 24, seed=9)))
    val = np.random.default_rng(4).standard_normal(idx.size)
    val /= np.linalg.norm(val)
    psi = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
    psi[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).cuda()
    try:
        hyp.set_support_skip(True)
        s_c = _apply(hyp, H, psi, "compact")
        s_r = _apply(hyp, H, psi, "rows")
        hyp.set_support_skip(False)
        s_d = _apply(hyp, H, psi, "compact")
    finally:
        hyp.set_support_skip(True)
    assert torch.equal(s_c, s_r)
    ref = oracle.apply_h_sparse(M, na, nb, x, z, c, idx, val)
    a = s_c.cpu().numpy()
    assert np.linalg.norm(a - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(s_d.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


def test_compact_mixed_pass_32q(hyp):
    """32-qubit H psi both ways, bit for bit, timed."""
    w = synth.WORKLOADS["h16_32q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    psi = _dev(synth.random_state(S.dim, 8))
    out, times = {}, {}
    for staging in ("compact", "rows"):
        out[staging] = _apply(hyp, H, psi, staging)
        t0 = time.perf_counter()
        hyp.set_mixed_matrix_cores(False)
        hyp.set_row_staging(staging)
        H.apply(psi, out[staging])
        torch.cuda.synchronize()
        hyp.set_row_staging("compact")
        hyp.set_mixed_matrix_cores()
        times[staging] = (time.perf_counter() - t0) * 1e3
    print(f"[staging] 32q H psi (768 threads): compact {times['compact']:.1f} ms, whole rows {times['rows']:.1f} ms",
          flush=True)
    assert torch.equal(out["compact"], out["rows"])
    del psi, out
    torch.cuda.empty_cache()


def test_compact_mixed_pass_in_captured_graph_24q(hyp):
    """The ADAPT evaluation graph captured with the compact mixed pass (24
    qubits: 924-column alpha space, two 768-column chunks), replayed with
    eager work in between, against eager evaluations with whole-row staging."""
    w = synth.WORKLOADS["h12_24q"]
    x, z, c, _, _ = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    Ag = hyp.Adapt(H, cre, ann, max_iter=8, use_graph=True)
    Ae = hyp.Adapt(H, cre, ann, max_iter=8, use_graph=False)
    ops = [int(v) for v in np.random.default_rng(1).integers(0, len(cre), 6)]
    th = np.linspace(-0.25, 0.35, 6)
    Ag.set_ansatz(ops, th)
    Ae.set_ansatz(ops, th)
    outs = []
    for rep in range(3):
        th2 = th * (1 + 0.2 * rep)
        e_g, g_g = Ag.eval(th2)
        try:
            hyp.set_row_staging("rows")
            e_e, g_e = Ae.eval(th2)
        finally:
            hyp.set_row_staging("compact")
        outs.append((e_g, g_g, e_e, g_e))
        torch.cuda.synchronize()
    for e_g, g_g, e_e, g_e in outs:
        assert abs(e_g - e_e) < 1e-13
        assert np.abs(g_g - g_e).max() < 1e-12
    assert len({round(o[0], 12) for o in outs}) == 3  # the replays saw the new parameters
