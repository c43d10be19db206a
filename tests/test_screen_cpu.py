"""CPU pins of the screen reference (oracle/mlp.py) and of the library's
host-side static feature builder against it."""
import math

import numpy as np
import pytest

from oracle import mlp as om
import synth


def test_bf16_rounding_matches_definition():
    # exact halfway cases round to even; values are representable after rounding
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-5, 1e30])
    r = om.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0  # 1 + 2^-8 is a tie -> even (1.0)
    assert r[1] == 1.0
    assert r[2] == 1.0                          # below half an ulp
    assert r[3] == 1.0 + 2 ** -7                # above half -> up
    assert r[4] == -2.5
    f = r.astype(np.float32).view(np.uint32)
    assert np.all((f & 0xFFFF) == 0)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8)


def test_mlp_backward_finite_differences():
    """Exact (unquantised) backward against central differences of the loss."""
    rng = np.random.default_rng(0)
    p = synth.mlp_init(3).astype(np.float64)
    X = rng.standard_normal((32, om.N_FEAT))
    t = rng.standard_normal(32)
    loss, _, g = om.loss_grad(p, X, t, quant=False)
    idx = np.concatenate([rng.choice(om.N_PARAM, 60, replace=False), [om.N_PARAM - 1]])
    for i in idx:
        h = 1e-6
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (om.loss_grad(pp, X, t, quant=False)[0] - om.loss_grad(pm, X, t, quant=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))


def test_adam_matches_closed_form_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.1, -0.2, 0.0])
    a = om.Adam(p, lr=1e-3)
    out = a.step(g)
    # first step: m_hat = g, v_hat = g^2  -> update = lr * g / (|g| + eps)
    exp = p - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(out, exp, rtol=0, atol=1e-15)


def test_select_top_k_and_audit():
    scores = np.array([0.1, 0.9, 0.9, -1.0, 0.5, 0.3])
    top, aud = om.select(scores, 2, [0, 2])
    assert list(top) == [1, 2]           # tie kept in index order
    assert list(aud) == [4, 0]           # ranks 0 and 2 among the rest (4, 5, 0, 3)


def test_static_features_reference_values():
    M = 4
    h, g = synth.integrals(M, 1)
    cre, ann, cls = synth.canonical_pool(M)
    F, Q = om.static_features(M, cre, ann, cls, h, g)
    # first alpha single: a=0 -> c=1
    assert F[0, 0] == 1.0 and F[0, 5] == pytest.approx(1 / 3) and F[0, 6] == 0.0
    assert F[0, 9] == pytest.approx(math.log10(abs(h[1, 0]) + 1e-12))
    assert list(Q[0]) == [1, 0, -1, -1]
    ab = np.nonzero(cls == 4)[0][0]
    assert F[ab, 4] == 1.0 and F[ab, 17] == 0.25
    assert np.all(F[:, 18:] == 0)


def test_library_static_features_match_reference():
    lib_so = pytest.importorskip("paper_2604_01176_amd.screen")
    for M in (4, 6):
        h, g = synth.integrals(M, 5)
        cre, ann, cls = synth.canonical_pool(M)
        F, Q = om.static_features(M, cre, ann, cls, h, g)
        stat, qidx = lib_so.static_features(M, cre, ann, cls, h, g)
        assert np.array_equal(qidx, Q.astype(np.int32))
        assert np.abs(stat - F.astype(np.float32)).max() <= 1e-6


def test_last_selection_features_by_hand():
    """Slots 18..21 against counts made by hand at M = 4: qubits 0..3 are
    alpha orbitals 0..3, 4..7 beta."""
    M = 4
    # qidx rows: an alpha single (c=2, a=0), an alpha-beta double (c=2, 6; a=0, 4),
    # a beta single (c=7, a=5), and the last selection itself
    Q = np.array([[2, 0, -1, -1], [2, 6, 0, 4], [7, 5, -1, -1], [3, 7, 1, 5]])
    F = np.zeros((4, om.N_FEAT))
    last = np.array([3, 7, 1, 5])           # alpha-beta double c=(3, 7) a=(1, 5): spatial {3, 1}
    X = om.features(F, Q, np.zeros(2 * M), np.ones(4), np.zeros(4), n_orb=M, last=last, last_g=0.01)
    assert list(X[:, 18]) == [0, 0, 0, 1]
    # spin-orbitals shared with {3, 7, 1, 5}: none; none; {7, 5}; all four
    assert list(X[:, 19]) == [0, 0, 0.5, 1.0]
    # spatial orbitals shared with {1, 3}: none; none ({2, 0}); {3, 1}; {3, 1}
    assert list(X[:, 20]) == [0, 0, 0.5, 0.5]
    assert np.allclose(X[:, 21], -2.0)
    X0 = om.features(F, Q, np.zeros(2 * M), np.ones(4), np.zeros(4))
    assert np.all(X0[:, 18:22] == 0)
