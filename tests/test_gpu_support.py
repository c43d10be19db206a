"""GPU parity of support skipping in H psi (the product of the sparse matrix
with a sparse vector): with skipping on (the default) and off, sigma must
match the oracle to ||d sigma|| / ||sigma|| <= 1e-12 (FP64), and the two
modes must agree to rounding, on states whose support is a few rows and
columns (Hartree-Fock, a few rotations away from it, one beta row, one alpha
column), on the zero state (sigma exactly zero) and on a dense state."""
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
    yield hyp
    hyp.set_support_skip(True)


def _dev(v, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)


def _hf_exciting_ops(M, na, nb, k, seed):
    """k pool generators whose excitation or de-excitation applies to the
    Hartree-Fock determinant, drawn at random (seeded)."""
    cre, ann, _ = synth.canonical_pool(M)
    hf = synth.hf_bits(M, na, nb)
    ok = [i for i in range(cre.size)
          if ((int(ann[i]) & hf) == int(ann[i]) and (int(cre[i]) & hf) == 0)]
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(ok), size=min(k, len(ok)), replace=False)
    return [(int(cre[ok[i]]), int(ann[ok[i]])) for i in pick]


def _states(M, na, nb, da, db):
    """Named input states of the sector (FP64, host)."""
    dim = da * db
    rng = np.random.default_rng(1000 + M)
    out = {}
    hf = np.zeros(dim)
    hf[int(oracle.rank(M, na, nb, np.array([synth.hf_bits(M, na, nb)]))[0])] = 1.0
    out["hartree_fock"] = hf
    v = hf.copy()
    for j, (c, a) in enumerate(_hf_exciting_ops(M, na, nb, 3, seed=M)):
        v = oracle.rotate(M, na, nb, c, a, 0.3 + 0.2 * j, v)
    out["hf_three_rotations"] = v
    idx, val = synth.sparse_state(dim, da, n_random=8, seed=5)
    v = np.zeros(dim)
    v[idx] = val
    out["sparse_random"] = v
    v = np.zeros(dim)
    b = db // 2
    v[b * da:(b + 1) * da] = rng.standard_normal(da)
    out["one_beta_row"] = v
    v = np.zeros(dim)
    a = da - 1
    v[a::da] = rng.standard_normal(db)
    out["one_alpha_column"] = v
    out["zero"] = np.zeros(dim)
    out["dense"] = synth.random_state(dim, 7)
    return out


CASES = [(4, 2, 2), (5, 3, 2), (6, 3, 3), (7, 2, 5), (8, 4, 4), (9, 5, 4), (3, 0, 2), (4, 4, 1), (10, 4, 5),
         (5, 2, 0), (4, 1, 4)]


@pytest.mark.parametrize("M,na,nb", CASES)
def test_support_skip_fp64(hyp, M, na, nb):
    h, g = synth.integrals(M, 300 + M)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    assert H.structured
    for name, psi in _states(M, na, nb, S.da, S.db).items():
        ref = oracle.apply_h(M, na, nb, x, z, c, psi)
        hyp.set_support_skip(True)
        on = H.apply(_dev(psi)).cpu().numpy()
        hyp.set_support_skip(False)
        off = H.apply(_dev(psi)).cpu().numpy()
        hyp.set_support_skip(True)
        nref = np.linalg.norm(ref)
        if name == "zero":
            assert np.all(on == 0.0) and np.all(off == 0.0), name
            continue
        assert np.linalg.norm(on - ref) <= 1e-12 * nref, name
        assert np.linalg.norm(off - ref) <= 1e-12 * nref, name
        assert np.linalg.norm(on - off) <= 1e-14 * nref, name


@pytest.mark.parametrize("M,na,nb", [(8, 4, 4), (9, 5, 4)])
def test_support_skip_fp32(hyp, M, na, nb):
    h, g = synth.integrals(M, 300 + M)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    for name, psi in _states(M, na, nb, S.da, S.db).items():
        p32 = psi.astype(np.float32)
        ref = oracle.apply_h(M, na, nb, x, z, c, p32.astype(np.float64))
        hyp.set_support_skip(True)
        on = H.apply(_dev(p32, torch.float32)).cpu().numpy().astype(np.float64)
        hyp.set_support_skip(False)
        off = H.apply(_dev(p32, torch.float32)).cpu().numpy().astype(np.float64)
        hyp.set_support_skip(True)
        nref = np.linalg.norm(ref)
        if name == "zero":
            assert np.all(on == 0.0) and np.all(off == 0.0), name
            continue
        # FP32 coefficient and product per term, FP64 sums, one FP32 store
        assert np.linalg.norm(on - ref) <= 2e-6 * nref, name
        assert np.linalg.norm(on - off) <= 2e-7 * nref, name


def test_support_skip_argument_check(hyp):
    from paper_2604_01176_amd import _lib
    assert _lib.load().hyp_set_support_skip(2) != 0
    assert _lib.load().hyp_set_support_skip(-1) != 0
    hyp.set_support_skip(True)


def test_support_skip_32q_near_hartree_fock(hyp):
    """32-qubit sector (8, 8): Hartree-Fock plus 24 singly and doubly excited
    determinants (an early-ADAPT support), every entry of sigma against the
    oracle with skipping on, and the product timed both ways."""
    w = synth.WORKLOADS["h16_32q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    idx = np.unique(oracle.rank(M, na, nb, synth.near_hf_bits(M, na, nb, 24, seed=3)))
    assert idx.min() >= 0
    rng = np.random.default_rng(11)
    val = rng.standard_normal(idx.size)
    val /= math.sqrt(float(val @ val))
    print(f"[support] 32q state with {idx.size} nonzeros", flush=True)
    ref = oracle.apply_h_sparse(M, na, nb, x, z, c, idx, val)
    psi = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
    psi[torch.from_numpy(idx).cuda()] = torch.from_numpy(val).cuda()
    times = {}
    outs = {}
    for on in (True, False):
        hyp.set_support_skip(on)
        out = H.apply(psi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            H.apply(psi, out)
        torch.cuda.synchronize()
        times[on] = (time.perf_counter() - t0) / 3 * 1e3
        outs[on] = out.cpu().numpy()
    hyp.set_support_skip(True)
    print(f"[support] 32q H psi near Hartree-Fock: skipping {times[True]:.2f} ms, dense {times[False]:.2f} ms",
          flush=True)
    nref = np.linalg.norm(ref)
    assert np.linalg.norm(outs[True] - ref) <= 1e-12 * nref
    assert np.linalg.norm(outs[False] - ref) <= 1e-12 * nref
    assert times[True] < times[False]


# ------------------------------------------------------------- gradient sweep

GCASES = [(4, 2, 2), (5, 2, 3), (6, 3, 3), (8, 4, 4), (9, 5, 4), (3, 0, 2), (4, 4, 1), (7, 3, 2), (10, 4, 5),
          (2, 1, 1), (5, 2, 0)]


@pytest.mark.parametrize("M,na,nb", GCASES)
def test_sweep_support_skip(hyp, M, na, nb):
    """Gradients restricted to psi's support, in the transition-value sweep
    (row pairs, identity slices and both Gram sums) and in the pair kernel
    (pairs whose two determinants lie outside the support skipped), against
    the oracle, FP64 and FP32, and against the unrestricted computation."""
    h, g = synth.integrals(M, 300 + M)
    x, z, c = synth.jw_pauli_list(h, g)
    S = hyp.Sector(M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    ops = hyp.exc_tensor(cre, ann)
    try:
        for mode in ("tdens", "pairs"):
            hyp.set_sweep_mode(mode)
            for name, psi in _states(M, na, nb, S.da, S.db).items():
                sig = oracle.apply_h(M, na, nb, x, z, c, psi)
                ref = oracle.pool_gradients(M, na, nb, cre, ann, psi, sig)
                got = {}
                for on in (True, False):
                    hyp.set_support_skip(on)
                    got[on] = (hyp.hyp_pool_gradients(S, ops, _dev(psi), _dev(sig)).cpu().numpy(),
                               hyp.hyp_pool_gradients(S, ops, _dev(psi, torch.float32),
                                                      _dev(sig, torch.float32)).cpu().numpy())
                hyp.set_support_skip(True)
                if name == "zero":
                    assert all(np.all(v == 0.0) for pair in got.values() for v in pair), (mode, name)
                    continue
                scale = max(1.0, np.abs(ref).max())
                for on, (g64, g32) in got.items():
                    assert np.abs(g64 - ref).max() <= 1e-12 * scale, (mode, name, on)
                    assert np.abs(g32 - ref).max() <= 1e-5 * scale, (mode, name, on)
                assert np.abs(got[True][0] - got[False][0]).max() <= 1e-13 * scale, (mode, name)
    finally:
        hyp.set_support_skip(True)
        hyp.set_sweep_mode("auto")


def test_sweep_support_skip_32q_near_hartree_fock(hyp):
    """32-qubit sector (8, 8), the near-Hartree-Fock state of the H psi test:
    all 39,960 gradients with skipping on against the unrestricted sweep, a
    sample against the oracle, and both timed."""
    w = synth.WORKLOADS["h16_32q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    ops = hyp.exc_tensor(cre, ann)
    idx = np.unique(oracle.rank(M, na, nb, synth.near_hf_bits(M, na, nb, 24, seed=3)))
    rng = np.random.default_rng(11)
    val = rng.standard_normal(idx.size)
    val /= math.sqrt(float(val @ val))
    sig = oracle.apply_h_sparse(M, na, nb, x, z, c, idx, val)
    psi_h = np.zeros(S.dim)
    psi_h[idx] = val
    d_psi, d_sig = _dev(psi_h), _dev(sig)
    times, outs = {}, {}
    try:
        for on in (True, False):
            hyp.set_support_skip(on)
            out = hyp.hyp_pool_gradients(S, ops, d_psi, d_sig)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                hyp.hyp_pool_gradients(S, ops, d_psi, d_sig, out)
            torch.cuda.synchronize()
            times[on] = (time.perf_counter() - t0) / 2 * 1e3
            outs[on] = out.cpu().numpy()
    finally:
        hyp.set_support_skip(True)
    print(f"[support] 32q full sweep near Hartree-Fock: skipping {times[True]:.2f} ms, "
          f"dense {times[False]:.2f} ms", flush=True)
    scale = max(1.0, np.abs(outs[False]).max())
    assert np.abs(outs[True] - outs[False]).max() <= 1e-13 * scale
    k = np.random.default_rng(5).choice(len(cre), 8, replace=False)
    k = np.concatenate([k, [int(np.argmax(np.abs(outs[True])))]])
    ref = oracle.pool_gradients(M, na, nb, cre[k], ann[k], psi_h, sig)
    assert np.abs(outs[True][k] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert times[True] < times[False]


def test_apply_excitations_sequence(hyp):
    M, na, nb = 6, 3, 3
    S = hyp.Sector(M, na, nb)
    cre, ann, _ = synth.canonical_pool(M)
    rng = np.random.default_rng(4)
    k = rng.choice(cre.size, 10, replace=False)
    th = rng.uniform(-1, 1, 10)
    psi = synth.random_state(S.dim, 6)
    ref = psi.copy()
    for i in range(10):
        ref = oracle.rotate(M, na, nb, cre[k[i]], ann[k[i]], th[i], ref)
    d = _dev(psi)
    hyp.hyp_apply_excitations(S, cre[k], ann[k], th, d)
    assert np.abs(d.cpu().numpy() - ref).max() <= 1e-13
    # an invalid generator anywhere in the list: nothing is applied
    bad_c, bad_a = cre[k].copy(), ann[k].copy()
    bad_c[5] = bad_a[5]
    d2 = _dev(psi)
    with pytest.raises(hyp.HypError):
        hyp.hyp_apply_excitations(S, bad_c, bad_a, th, d2)
    assert np.array_equal(d2.cpu().numpy(), psi)
    # the empty sequence
    hyp.hyp_apply_excitations(S, [], [], [], d2)
    assert np.array_equal(d2.cpu().numpy(), psi)
