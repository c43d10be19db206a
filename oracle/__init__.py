"""Plain FP64 CPU oracle for the sparse state-vector ADAPT-VQE hot path.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code,
header, table or helper with the GPU library (``paper_2604_01176_amd``) and
never imports it; the two meet only at the seeded inputs of ``synth``.

Contents
  * oracle.c   -- literal term-by-term / pair-by-pair sector operations
                  (H psi, <a|b>, pool gradients, exp(theta A) psi, A psi,
                  occupations, rank/unrank), compiled to liboracle.so.
  * brute      -- dense 2^n brute force: explicit ladder matrices, the
                  second-quantised H, Kronecker-product Pauli matrices, FCI.
  * adapt      -- the ADAPT-VQE loop with scipy BFGS.
  * mlp        -- FP64 3-layer MLP forward/backward with BF16 quantisation
                  points, and Adam; gradient-screen features.

Parity status of each function is stated in its docstring; every function
here is pinned by tests in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        i64, u32p, f64p, i64p = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
        ci = ctypes.c_int
        L.orc_binom.restype = i64
        L.orc_binom.argtypes = [ci, ci]
        L.orc_rank_string.restype = i64
        L.orc_rank_string.argtypes = [ctypes.c_uint32]
        L.orc_unrank_string.restype = ctypes.c_uint32
        L.orc_unrank_string.argtypes = [ci, ci, i64]
        L.orc_sector_dim.restype = i64
        L.orc_sector_dim.argtypes = [ci, ci, ci]
        L.orc_sector_rank.argtypes = [ci, ci, ci, u32p, i64, i64p]
        L.orc_sector_unrank.argtypes = [ci, ci, ci, i64p, i64, u32p]
        L.orc_apply_h.restype = ci
        L.orc_apply_h.argtypes = [ci, ci, ci, i64, u32p, u32p, f64p, f64p, i64p, i64, f64p]
        L.orc_apply_h_sparse.restype = ci
        L.orc_apply_h_sparse.argtypes = [ci, ci, ci, i64, u32p, u32p, f64p, i64, i64p, f64p, f64p]
        L.orc_dot.restype = ctypes.c_double
        L.orc_dot.argtypes = [i64, f64p, f64p]
        L.orc_apply_tau.restype = ci
        L.orc_apply_tau.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_uint32)]
        L.orc_pool_gradients.argtypes = [ci, ci, ci, i64, u32p, u32p, f64p, f64p, f64p]
        L.orc_pool_gradients_sparse.argtypes = [ci, ci, ci, i64, u32p, u32p, i64, i64p, f64p, f64p, f64p]
        L.orc_apply_generator.argtypes = [ci, ci, ci, ctypes.c_uint32, ctypes.c_uint32, f64p, f64p]
        L.orc_rotate.argtypes = [ci, ci, ci, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, f64p]
        L.orc_set_qubit_excitations.restype = None
        L.orc_set_qubit_excitations.argtypes = [ci]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ci]
        L.orc_max_threads.restype = ci
        L.orc_max_threads.argtypes = []
        L.orc_pair_count.restype = i64
        L.orc_pair_count.argtypes = [ci, ci, ci, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_occupations.argtypes = [ci, ci, ci, f64p, f64p]
        L.orc_pair_list.restype = i64
        L.orc_pair_list.argtypes = [ci, ci, ci, ctypes.c_uint32, ctypes.c_uint32, i64p, i64p, ctypes.c_void_p]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def binom(m, k):
    return int(lib().orc_binom(m, k))


def sector_dim(M, na, nb):
    return int(lib().orc_sector_dim(M, na, nb))


def rank(M, na, nb, bits):
    """Sector index of each bitstring (-1 if outside the sector)."""
    bits = _u32(bits)
    out = np.empty(bits.shape, dtype=np.int64)
    lib().orc_sector_rank(M, na, nb, _p(bits), bits.size, _p(out))
    return out


def unrank(M, na, nb, idx):
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.shape, dtype=np.uint32)
    lib().orc_sector_unrank(M, na, nb, _p(idx), idx.size, _p(out))
    return out


def apply_h(M, na, nb, x, z, c, psi, out_idx=None):
    """sigma = P_S H P_S psi (all outputs, or the sector indices out_idx)."""
    x, z, c, psi = _u32(x), _u32(z), _f64(c), _f64(psi)
    if out_idx is None:
        n_out = psi.size
        out = np.empty(n_out)
        rc = lib().orc_apply_h(M, na, nb, c.size, _p(x), _p(z), _p(c), _p(psi), None, n_out, _p(out))
    else:
        out_idx = np.ascontiguousarray(out_idx, dtype=np.int64)
        out = np.empty(out_idx.size)
        rc = lib().orc_apply_h(M, na, nb, c.size, _p(x), _p(z), _p(c), _p(psi), _p(out_idx),
                               out_idx.size, _p(out))
    if rc != 0:
        raise ValueError("odd-n_Y term: Hamiltonian is not real")
    return out


def apply_h_sparse(M, na, nb, x, z, c, in_idx, in_val):
    """sigma = H psi (all dim outputs) for psi given by its nonzeros."""
    x, z, c = _u32(x), _u32(z), _f64(c)
    in_idx = np.ascontiguousarray(in_idx, dtype=np.int64)
    in_val = _f64(in_val)
    out = np.empty(sector_dim(M, na, nb))
    rc = lib().orc_apply_h_sparse(M, na, nb, c.size, _p(x), _p(z), _p(c), in_idx.size, _p(in_idx),
                                  _p(in_val), _p(out))
    if rc != 0:
        raise ValueError("odd-n_Y term: Hamiltonian is not real")
    return out


def dot(a, b):
    a, b = _f64(a), _f64(b)
    return float(lib().orc_dot(a.size, _p(a), _p(b)))


def energy(M, na, nb, x, z, c, psi):
    """E = <psi|H|psi> / <psi|psi>."""
    s = apply_h(M, na, nb, x, z, c, psi)
    return dot(psi, s) / dot(psi, psi)


def set_threads(n: int):
    """Thread count of the oracle's parallel loops (for timing)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


class qubit_excitations:
    """Context: the excitation functions below act as qubit excitations
    (QEB: no Jordan-Wigner parity, every sign +1) inside the block."""

    def __enter__(self):
        lib().orc_set_qubit_excitations(1)
        return self

    def __exit__(self, *exc):
        lib().orc_set_qubit_excitations(0)
        return False


def apply_tau(cre, ann, b):
    out = ctypes.c_uint32(0)
    s = lib().orc_apply_tau(int(cre), int(ann), int(b), ctypes.byref(out))
    return s, int(out.value)


def pool_gradients(M, na, nb, cre, ann, psi, sigma):
    """g_k = 2 <sigma|A_k psi> for every generator (cre[k], ann[k])."""
    cre, ann, psi, sigma = _u32(cre), _u32(ann), _f64(psi), _f64(sigma)
    out = np.empty(cre.size)
    lib().orc_pool_gradients(M, na, nb, cre.size, _p(cre), _p(ann), _p(psi), _p(sigma), _p(out))
    return out


def pool_gradients_sparse(M, na, nb, cre, ann, nz, psi, sigma):
    """The same g_k for a psi whose nonzeros are the sector indices nz (each
    once): the pair sum taken over pairs with a listed end only, exact since
    every other pair contributes 0 (psi and sigma dense, all dim entries)."""
    cre, ann, psi, sigma = _u32(cre), _u32(ann), _f64(psi), _f64(sigma)
    nz = np.ascontiguousarray(nz, dtype=np.int64)
    out = np.empty(cre.size)
    lib().orc_pool_gradients_sparse(M, na, nb, cre.size, _p(cre), _p(ann), nz.size, _p(nz), _p(psi), _p(sigma),
                                    _p(out))
    return out


def apply_generator(M, na, nb, cre, ann, psi):
    psi = _f64(psi)
    out = np.empty_like(psi)
    lib().orc_apply_generator(M, na, nb, int(cre), int(ann), _p(psi), _p(out))
    return out


def rotate(M, na, nb, cre, ann, theta, psi):
    """Return exp(theta A) psi (copy)."""
    out = _f64(psi).copy()
    lib().orc_rotate(M, na, nb, int(cre), int(ann), float(theta), _p(out))
    return out


def pair_count(M, na, nb, cre, ann):
    return int(lib().orc_pair_count(M, na, nb, int(cre), int(ann)))


def occupations(M, na, nb, psi):
    psi = _f64(psi)
    out = np.empty(2 * M)
    lib().orc_occupations(M, na, nb, _p(psi), _p(out))
    return out


def pair_list(M, na, nb, cre, ann):
    """(D, D', s) arrays of one generator's pairs, by literal application of tau."""
    n = pair_count(M, na, nb, cre, ann)
    src = np.empty(n, dtype=np.int64)
    dst = np.empty(n, dtype=np.int64)
    sg = np.empty(n, dtype=np.int8)
    m = lib().orc_pair_list(M, na, nb, int(cre), int(ann), _p(src), _p(dst), _p(sg))
    assert m == n
    return src, dst, sg
