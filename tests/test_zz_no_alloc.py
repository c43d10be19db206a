"""hyp_pool_gradients_noalloc (the pair kernel with its partials in the
library's static per-GPU scratch array, no allocation on any call) against
hyp_pool_gradients on the same inputs, through the C ABI: two calls in a row,
the second with a smaller input (a smaller sector and fewer generators), so
that a stale partial left in the shared scratch would show."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hyp():
    import paper_2604_01176_amd as hyp
    return hyp


def _noalloc(hyp, S, ops, psi, sig):
    from paper_2604_01176_amd import _lib
    n = ops.shape[0]
    out = torch.full((n,), float("nan"), dtype=torch.float64, device=psi.device)
    st = _lib.load().hyp_pool_gradients_noalloc(S.handle, 0 if psi.dtype == torch.float64 else 1,
                                                ctypes.c_void_p(ops.data_ptr()), n,
                                                ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                                ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    return out


def _case(hyp, name, n_ops, seed, dtype):
    w = synth.WORKLOADS[name]
    x, z, c, _, _ = synth.hamiltonian(w)
    S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
    H = hyp.Hamiltonian(S, x, z, c)
    cre, ann, _ = synth.canonical_pool(w.n_orb)
    pick = np.sort(np.random.default_rng(seed).choice(len(cre), n_ops, replace=False))
    ops = hyp.exc_tensor(cre[pick], ann[pick])
    psi = torch.from_numpy(synth.random_state(S.dim, seed)).cuda().to(dtype)
    sig = H.apply(psi)
    return S, ops, psi, sig


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_equals_pool_gradients_two_calls(hyp, dtype):
    cases = [("h8_16q", 2044, 7), ("h4_8q", 37, 8)]  # the second call: smaller sector, fewer generators
    hyp.set_sweep_mode("pairs")
    try:
        for name, n_ops, seed in cases:
            S, ops, psi, sig = _case(hyp, name, n_ops, seed, dtype)
            got = _noalloc(hyp, S, ops, psi, sig).cpu().numpy()
            ref = hyp.hyp_pool_gradients(S, ops, psi, sig).cpu().numpy()
            tol = 1e-12 if dtype == torch.float64 else 1e-5
            assert np.all(np.isfinite(got)), name
            assert np.abs(got - ref).max() <= tol * max(1.0, np.abs(ref).max()), name
    finally:
        hyp.set_sweep_mode("auto")
    hyp.hyp_pool_check()


def test_noalloc_rejects_oversize(hyp):
    from paper_2604_01176_amd import _lib
    S, ops, psi, sig = _case(hyp, "h4_8q", 10, 3, torch.float64)
    big = 32769
    st = _lib.load().hyp_pool_gradients_noalloc(S.handle, 0, ctypes.c_void_p(ops.data_ptr()), big,
                                                ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                                ctypes.c_void_p(psi.data_ptr()), None)
    assert st == 1  # HYP_ERR_ARG, nothing enqueued
    assert b"32768" in _lib.load().hyp_last_error()
