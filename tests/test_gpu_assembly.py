"""GPU parity of the device-side Hamiltonian assembly (integrals -> merged,
sorted Jordan-Wigner Pauli list on the GPU) against the oracle's own
expansion (oracle/jw.py, pinned to the dense second-quantised matrix):
masks and term counts bit-exact, coefficients within two ulps; H psi of the
Hamiltonian built from the integrals on the device against the oracle to
||d sigma|| / ||sigma|| <= 1e-12."""
import math
import time

import numpy as np
import pytest

import oracle
import synth
from oracle import jw

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hyp():
    import paper_2604_01176_amd as hyp
    return hyp


def _same_list(got, ref):
    x, z, c = got
    xr, zr, cr = ref
    assert x.size == xr.size
    assert np.array_equal(x, xr) and np.array_equal(z, zr)
    assert np.all(np.abs(c - cr) <= 4.5e-16 * np.abs(cr))


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6, 8, 10, 12])
def test_assemble_pauli_matches_oracle(hyp, M):
    h, g = synth.integrals(M, 500 + M)
    got = hyp.hyp_assemble_pauli(h, g, e_core=0.375 * M)
    _same_list(got, jw.jw_pauli_list(h, g, e_core=0.375 * M))


def test_assemble_pauli_edge_cases(hyp):
    # constant only
    x, z, c = hyp.hyp_assemble_pauli(np.zeros((3, 3)), np.zeros((3, 3, 3, 3)), e_core=2.5)
    assert list(x) == [0] and list(z) == [0] and list(c) == [2.5]
    # nothing at all
    x, z, c = hyp.hyp_assemble_pauli(np.zeros((2, 2)), np.zeros((2, 2, 2, 2)))
    assert x.size == 0
    # sparse integrals: one-body diagonal only, and a single (pq|rs) quadruple
    # with its 8-fold images
    M = 4
    h = np.diag(np.arange(1.0, M + 1.0))
    g = np.zeros((M, M, M, M))
    for p, q, r, s in {(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 0, 1),
                       (2, 3, 1, 0), (3, 2, 1, 0)}:
        g[p, q, r, s] = 0.125
    _same_list(hyp.hyp_assemble_pauli(h, g), jw.jw_pauli_list(h, g))
    # not real-symmetric
    h2, g2 = synth.integrals(3, 1)
    h2[0, 2] += 0.5
    with pytest.raises(hyp.HypError) as e:
        hyp.hyp_assemble_pauli(h2, g2)
    assert e.value.status == 3
    # capacity below the count
    from paper_2604_01176_amd import _lib
    import ctypes
    h3, g3 = synth.integrals(3, 2)
    hd, gd = torch.from_numpy(h3).cuda(), torch.from_numpy(g3).cuda()
    n = ctypes.c_int64()
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    xo = torch.empty(4, dtype=torch.int32, device="cuda")
    zo = torch.empty(4, dtype=torch.int32, device="cuda")
    rc = _lib.load().hyp_assemble_pauli(3, hd.data_ptr(), gd.data_ptr(), 0.0, xo.data_ptr(), zo.data_ptr(),
                                        out.data_ptr(), 4, ctypes.byref(n), None)
    assert rc == 1 and n.value == jw.jw_pauli_list(h3, g3)[0].size
    rc = _lib.load().hyp_assemble_pauli(17, hd.data_ptr(), gd.data_ptr(), 0.0, None, None, None, 0,
                                        ctypes.byref(n), None)
    assert rc == 1


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (6, 3, 3), (7, 2, 5), (8, 4, 4), (9, 5, 4), (3, 0, 2), (10, 5, 5)])
def test_hamiltonian_from_integrals(hyp, M, na, nb):
    h, g = synth.integrals(M, 600 + M)
    e_core = 1.25
    S = hyp.Sector(M, na, nb)
    Hd = hyp.Hamiltonian.from_integrals(S, h, g, e_core)
    assert Hd.structured
    x, z, c = jw.jw_pauli_list(h, g, e_core)
    psi = synth.random_state(S.dim, 19)
    ref = oracle.apply_h(M, na, nb, x, z, c, psi)
    d = torch.from_numpy(psi).cuda()
    out = Hd.apply(d).cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
    # same tables as the build from the host list
    Hh = hyp.Hamiltonian(S, x, z, c)
    out2 = Hh.apply(d).cpu().numpy()
    assert np.linalg.norm(out - out2) <= 1e-14 * np.linalg.norm(ref)


def test_hamiltonian_from_integrals_checks_orbital_count(hyp):
    S = hyp.Sector(4, 2, 2)
    h, g = synth.integrals(5, 1)
    from paper_2604_01176_amd import _lib
    import ctypes
    hd, gd = torch.from_numpy(h).cuda(), torch.from_numpy(g).cuda()
    hh = ctypes.c_void_p()
    rc = _lib.load().hyp_build_hamiltonian_integrals(S.handle, 5, hd.data_ptr(), gd.data_ptr(), 0.0, None,
                                                     ctypes.byref(hh))
    assert rc == 1


def test_assembly_32q(hyp):
    """32-qubit workload: the device list equals the oracle's (94,849 terms),
    sigma from the device-built Hamiltonian on sampled rows against the
    oracle, and the assembly timed."""
    w = synth.WORKLOADS["h16_32q"]
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    h, g = synth.integrals(M, w.seed)
    t0 = time.perf_counter()
    ref_list = jw.jw_pauli_list(h, g)
    t_oracle = time.perf_counter() - t0
    hyp.hyp_assemble_pauli(h, g)  # warm-up (rocPRIM kernels, allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = hyp.hyp_assemble_pauli(h, g)
    t_gpu = time.perf_counter() - t0
    print(f"[assembly] 32q: {got[0].size} terms, device {t_gpu * 1e3:.1f} ms, oracle {t_oracle:.2f} s", flush=True)
    _same_list(got, ref_list)
    S = hyp.Sector(M, na, nb)
    Hd = hyp.Hamiltonian.from_integrals(S, h, g)
    assert Hd.structured
    psi = synth.random_state(S.dim, 7)
    out = Hd.apply(torch.from_numpy(psi).cuda()).cpu().numpy()
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([[0, S.dim - 1], rng.integers(0, S.dim, 200)]))
    x, z, c = ref_list
    ref = oracle.apply_h(M, na, nb, x, z, c, psi, out_idx=idx)
    assert np.abs(out[idx] - ref).max() <= 1e-12 * np.linalg.norm(ref) / math.sqrt(len(idx)) * 10
