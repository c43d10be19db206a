"""MI355X (gfx950) sparse state-vector ADAPT-VQE hot path.

Thin Python binding over the C ABI of libhyperion_mi355x.so: argument
marshalling only.  Device buffers are torch tensors on the current HIP device
and every call is enqueued on torch's current stream; all arithmetic runs in
the library's HIP kernels.  Importing this package needs the built library
(there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib
from ._lib import HYP_F32, HYP_F64, HypError, HypExc, check

__all__ = ["Sector", "Hamiltonian", "Adapt", "hyp_apply_h", "hyp_expectation",
           "hyp_pool_gradients", "hyp_pool_check", "hyp_apply_excitation", "HypError", "HYP_F64", "HYP_F32",
           "exc_tensor", "profile_enable", "profile_reset", "profile_read"]

_lib.load()


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return HYP_F64
    if t.dtype == torch.float32:
        return HYP_F32
    raise TypeError(f"state buffers must be float64 or float32, got {t.dtype}")


def _dev_ptr(t, n=None, what="buffer"):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


class Sector:
    """hyp_sector: the (N_alpha, N_beta) configuration space of n_orb orbitals."""

    def __init__(self, n_orb: int, n_alpha: int, n_beta: int):
        h = ctypes.c_void_p()
        check(_lib.load().hyp_sector_create(n_orb, n_alpha, n_beta, ctypes.byref(h)))
        self._h = h
        self.n_orb, self.n_alpha, self.n_beta = n_orb, n_alpha, n_beta
        self.dim = int(_lib.load().hyp_sector_dim(h))
        self.da = math.comb(n_orb, n_alpha)
        self.db = math.comb(n_orb, n_beta)

    @property
    def handle(self):
        return self._h

    def rank(self, bits) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint32)
        out = np.empty(bits.shape, dtype=np.int64)
        check(_lib.load().hyp_sector_rank(self._h, bits.ctypes.data, bits.size, out.ctypes.data))
        return out

    def unrank(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty(idx.shape, dtype=np.uint32)
        check(_lib.load().hyp_sector_unrank(self._h, idx.ctypes.data, idx.size, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hyp_sector_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hamiltonian:
    """hyp_ham: X-grouped Pauli table uploaded for one sector."""

    def __init__(self, sector: Sector, x, z, c, *, _handle=None):
        if _handle is not None:
            self._h = _handle
            self.sector = sector
            self.structured = bool(_lib.load().hyp_ham_is_structured(_handle))
            return
        x = np.ascontiguousarray(x, dtype=np.uint32)
        z = np.ascontiguousarray(z, dtype=np.uint32)
        c = np.ascontiguousarray(c, dtype=np.float64)
        if not (x.shape == z.shape == c.shape and x.ndim == 1):
            raise ValueError("x, z, c must be 1-D arrays of equal length")
        h = ctypes.c_void_p()
        check(_lib.load().hyp_build_hamiltonian(sector.handle, x.ctypes.data, z.ctypes.data,
                                                c.ctypes.data, x.size, _stream(), ctypes.byref(h)))
        self._h = h
        self.sector = sector
        self.structured = bool(_lib.load().hyp_ham_is_structured(h))

    @classmethod
    def from_integrals(cls, sector: Sector, h, g, e_core: float = 0.0):
        """hyp_build_hamiltonian_integrals: Jordan-Wigner assembly of the
        integrals on the device, then the common build."""
        torch = _torch()
        M = sector.n_orb
        hd = torch.as_tensor(np.ascontiguousarray(h, dtype=np.float64)).reshape(M, M).cuda()
        gd = torch.as_tensor(np.ascontiguousarray(g, dtype=np.float64)).reshape(M, M, M, M).cuda()
        hh = ctypes.c_void_p()
        check(_lib.load().hyp_build_hamiltonian_integrals(sector.handle, M, hd.data_ptr(), gd.data_ptr(),
                                                          float(e_core), _stream(), ctypes.byref(hh)))
        return cls(sector, None, None, None, _handle=hh)

    def apply(self, psi, out=None):
        """sigma = H psi (hyp_apply_h)."""
        if out is None:
            out = _torch().empty_like(psi)
        hyp_apply_h(self, psi, out)
        return out

    def tune(self, psi, reps: int = 2):
        """hyp_tune_apply_h: (workgroup width, ms per H psi) of the fastest tile."""
        sig = _torch().empty_like(psi)
        t = ctypes.c_int()
        ms = ctypes.c_double()
        check(_lib.load().hyp_tune_apply_h(self._h, _dtype_code(psi), _dev_ptr(psi, self.sector.dim, "psi"),
                                           _dev_ptr(sig, self.sector.dim, "sigma"), int(reps), _stream(),
                                           ctypes.byref(t), ctypes.byref(ms)))
        return t.value, ms.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hyp_ham_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CsrMatrix:
    """hyp_csr: the sector Hamiltonian materialised in CSR form (comparison
    for the matrix-free product)."""

    def __init__(self, ham: Hamiltonian):
        m = ctypes.c_void_p()
        check(_lib.load().hyp_csr_build(ham._h, _stream(), ctypes.byref(m)))
        self._m = m
        self.dim = ham.sector.dim
        self.nnz = int(_lib.load().hyp_csr_nnz(m))

    def apply(self, psi, out=None):
        if out is None:
            out = _torch().empty_like(psi)
        check(_lib.load().hyp_csr_apply(self._m, _dtype_code(psi), _dev_ptr(psi, self.dim, "psi"),
                                        _dev_ptr(out, self.dim, "sigma"), _stream()))
        return out

    def export(self):
        """(row_ptr, col, val) host arrays."""
        rp = np.empty(self.dim + 1, dtype=np.int64)
        col = np.empty(self.nnz, dtype=np.int32)
        val = np.empty(self.nnz, dtype=np.float64)
        check(_lib.load().hyp_csr_export(self._m, rp.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rp, col, val

    def close(self):
        if getattr(self, "_m", None):
            _lib.load().hyp_csr_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hyp_assemble_pauli(h, g, e_core: float = 0.0):
    """Device-side Jordan-Wigner assembly of the integrals (hyp_assemble_pauli):
    (x, z, c) as host numpy arrays, sorted by (x, z)."""
    torch = _torch()
    M = int(np.asarray(h).shape[0])
    hd = torch.as_tensor(np.ascontiguousarray(h, dtype=np.float64)).cuda()
    gd = torch.as_tensor(np.ascontiguousarray(g, dtype=np.float64)).cuda()
    n = ctypes.c_int64()
    L = _lib.load()
    check(L.hyp_assemble_pauli(M, hd.data_ptr(), gd.data_ptr(), float(e_core), None, None, None, 0,
                               ctypes.byref(n), _stream()))
    k = max(1, n.value)
    x = torch.empty(k, dtype=torch.int32, device="cuda")
    z = torch.empty(k, dtype=torch.int32, device="cuda")
    c = torch.empty(k, dtype=torch.float64, device="cuda")
    check(L.hyp_assemble_pauli(M, hd.data_ptr(), gd.data_ptr(), float(e_core), x.data_ptr(), z.data_ptr(),
                               c.data_ptr(), k, ctypes.byref(n), _stream()))
    m = n.value
    return (x[:m].cpu().numpy().view(np.uint32), z[:m].cpu().numpy().view(np.uint32), c[:m].cpu().numpy())


def hyp_apply_h(ham: Hamiltonian, psi, sigma):
    n = ham.sector.dim
    if psi.dtype != sigma.dtype:
        raise TypeError("psi and sigma dtypes differ")
    check(_lib.load().hyp_apply_h(ham._h, _dtype_code(psi), _dev_ptr(psi, n, "psi"),
                                  _dev_ptr(sigma, n, "sigma"), _stream()))
    return sigma


def hyp_expectation(sector: Sector, a, b, out=None):
    """<a|b> into a 1-element float64 device tensor."""
    torch = _torch()
    if a.dtype != b.dtype:
        raise TypeError("a and b dtypes differ")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=a.device)
    check(_lib.load().hyp_expectation(sector.handle, _dtype_code(a), _dev_ptr(a, sector.dim, "a"),
                                      _dev_ptr(b, sector.dim, "b"), _dev_ptr(out, 1, "out"),
                                      _stream()))
    return out


def exc_tensor(cre, ann, device="cuda"):
    """Pack (cre, ann) masks into an int32 [n, 2] device tensor laid out as
    the hyp_exc array."""
    torch = _torch()
    arr = np.stack([np.asarray(cre, dtype=np.uint32), np.asarray(ann, dtype=np.uint32)], axis=1)
    return torch.from_numpy(arr.view(np.int32).copy()).to(device)


def hyp_pool_gradients(sector: Sector, ops, psi, sigma, out=None):
    """Enqueue g_k = 2 <sigma|A_k psi> on the current stream (no host wait).
    Invalid excitations get NaN and are reported by hyp_pool_check()."""
    torch = _torch()
    if ops.dtype != torch.int32 or ops.dim() != 2 or ops.shape[1] != 2:
        raise TypeError("ops must be an int32 [n, 2] tensor of (cre, ann) masks")
    n = ops.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=psi.device)
    check(_lib.load().hyp_pool_gradients(sector.handle, _dtype_code(psi), _dev_ptr(ops, None, "ops"), n,
                                         _dev_ptr(psi, sector.dim, "psi"),
                                         _dev_ptr(sigma, sector.dim, "sigma"),
                                         _dev_ptr(out, n, "grad"), _stream()))
    return out


def hyp_pool_check():
    """Wait for the current stream; raise HypError for the first invalid
    excitation hyp_pool_gradients met on this device since the last check."""
    check(_lib.load().hyp_pool_check(_stream()))


def hyp_apply_excitation(sector: Sector, cre: int, ann: int, theta: float, psi):
    check(_lib.load().hyp_apply_excitation(sector.handle, _dtype_code(psi), HypExc(int(cre), int(ann)),
                                           float(theta), _dev_ptr(psi, sector.dim, "psi"), _stream()))
    return psi


def hyp_apply_excitations(sector: Sector, cre, ann, theta, psi):
    """psi <- exp(theta[n-1] A_{n-1}) ... exp(theta[0] A_0) psi in place."""
    n = len(theta)
    ops = (_lib.HypExc * max(1, n))()
    for i, (c_, a_) in enumerate(zip(np.asarray(cre).tolist(), np.asarray(ann).tolist())):
        ops[i].cre, ops[i].ann = int(c_), int(a_)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    check(_lib.load().hyp_apply_excitations(sector.handle, _dtype_code(psi), ops, th.ctypes.data if n else None,
                                            n, _dev_ptr(psi, sector.dim, "psi"), _stream()))
    return psi


def set_sweep_mode(mode: str = "auto"):
    """hyp_set_sweep_mode: "auto", "pairs" (per-generator kernel), "tdens"
    (row-batched transition values) or "tdens_bins" (per-stage LDS bins)."""
    check(_lib.load().hyp_set_sweep_mode({"auto": 0, "pairs": 1, "tdens": 2, "tdens_bins": 3}[mode]))


def set_pool_kind(kind: str = "fermionic"):
    """hyp_set_pool_kind: "fermionic" or "qubit" (QEB) excitations."""
    check(_lib.load().hyp_set_pool_kind({"fermionic": 0, "qubit": 1}[kind]))


def set_row_staging(mode: str = "compact"):
    """hyp_set_row_staging: "compact" (default; FP64 sweep stages only the
    blocks of each source row its chunk reaches, double-buffered) or "rows"
    (whole rows).  Same results bit for bit."""
    check(_lib.load().hyp_set_row_staging({"compact": 0, "rows": 1}[mode]))


def set_support_skip(on: bool = True):
    """hyp_set_support_skip: restrict H psi to psi's row and column support."""
    check(_lib.load().hyp_set_support_skip(1 if on else 0))


def set_same_spin_groups(tiles=2):
    """hyp_set_same_spin_groups: FP64 same-spin pass over grouped lists (8
    output strings per wave sharing their source loads; `tiles` = 1, 2 or 4
    column tiles per four-wave workgroup; True = the default 2) or, for
    0 / False, per-row lists."""
    t = 2 if tiles is True else (0 if tiles is False else int(tiles))
    check(_lib.load().hyp_set_same_spin_groups(t))


def set_same_spin_cores(mode="auto"):
    """hyp_set_same_spin_cores: FP64 same-spin doubles as per-core dense
    products on the matrix cores: "auto" (default; where the FP64 state
    exceeds the 256 MiB Infinity Cache), True (wherever built) or False
    (the lists of set_same_spin_groups)."""
    m = 2 if mode == "auto" else (1 if mode else 0)
    check(_lib.load().hyp_set_same_spin_cores(m))


def set_mixed_matrix_cores(mode="auto"):
    """hyp_set_mixed_matrix_cores: the alpha-beta products of H psi and of
    the sweep as dense products on the matrix cores: "auto" (default; H psi
    from 64 MiB FP64 states, the sweep from 256 MiB, where the row fits LDS),
    True (wherever the row fits) or False (the bitwise-reproducible
    k_mixed / k_mixed_c and k_tdens_rows)."""
    m = 2 if mode == "auto" else (1 if mode else 0)
    check(_lib.load().hyp_set_mixed_matrix_cores(m))


def profile_enable(on: bool = True):
    check(_lib.load().hyp_profile_enable(1 if on else 0))


def profile_reset():
    check(_lib.load().hyp_profile_reset())


def profile_read() -> dict:
    """{kernel name: (total device ms, launches)} of the events recorded so far."""
    L = _lib.load()
    out = {}
    for i in range(L.hyp_profile_count()):
        buf = ctypes.create_string_buffer(128)
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(L.hyp_profile_get(i, buf, 128, ctypes.byref(ms), ctypes.byref(n)))
        out[buf.value.decode()] = (ms.value, n.value)
    return out


class Adapt:
    """hyp_adapt: the native ADAPT-VQE driver over one Hamiltonian and pool.

    dtype "f64" or "f32" (FP32 storage, FP64 accumulation).  Defaults follow
    the selection/optimiser readings: tie_tol 1e-9 (f64) / 1e-5 (f32),
    BFGS gtol 1e-9 (f64) / 1e-5 (f32, the gradient's noise floor), early stop
    when max|g| < 1e-10; BFGS starts from the previous iteration's
    inverse-Hessian estimate (recycle_hessian).
    """

    def __init__(self, ham: Hamiltonian, cre, ann, dtype: str = "f64", max_iter: int = 64,
                 max_bfgs: int = 1000, use_graph: bool = True, tie_tol=None, gtol=None,
                 gmax_stop: float = 1e-10, recycle_hessian: bool = True):
        f32 = dtype == "f32"
        self.dtype = dtype
        self.ham = ham
        self.n_pool = len(cre)
        pool = (_lib.HypExc * self.n_pool)()
        for i, (c_, a_) in enumerate(zip(np.asarray(cre).tolist(), np.asarray(ann).tolist())):
            pool[i].cre, pool[i].ann = int(c_), int(a_)
        o = _lib.AdaptOpts(max_iter=max_iter, max_bfgs=max_bfgs, use_graph=1 if use_graph else 0,
                           recycle_hessian=1 if recycle_hessian else 0, tie_tol=(1e-5 if f32 else 1e-9) if tie_tol is None else tie_tol,
                           gtol=(1e-5 if f32 else 1e-9) if gtol is None else gtol,
                           gmax_stop=gmax_stop)
        h = ctypes.c_void_p()
        check(_lib.load().hyp_adapt_create(ham._h, HYP_F32 if f32 else HYP_F64, pool, self.n_pool,
                                           ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def iterate(self, cand=None) -> dict:
        rec = _lib.AdaptRecord()
        if cand is None:
            check(_lib.load().hyp_adapt_iterate(self._h, None, 0, ctypes.byref(rec)))
        else:
            c = np.ascontiguousarray(cand, dtype=np.int32)
            check(_lib.load().hyp_adapt_iterate(self._h, c.ctypes.data, c.size, ctypes.byref(rec)))
        return {f: getattr(rec, f) for f, _ in rec._fields_ if f != "reserved"}

    def gradients(self, cand=None) -> dict:
        """Exact pool gradients of the current state (all, or the candidates)."""
        rec = _lib.AdaptRecord()
        if cand is None:
            check(_lib.load().hyp_adapt_gradients(self._h, None, 0, ctypes.byref(rec)))
        else:
            c = np.ascontiguousarray(cand, dtype=np.int32)
            check(_lib.load().hyp_adapt_gradients(self._h, c.ctypes.data, c.size, ctypes.byref(rec)))
        self._rec = rec
        return {f: getattr(rec, f) for f, _ in rec._fields_ if f != "reserved"}

    def select_optimize(self) -> dict:
        rec = getattr(self, "_rec", None) or _lib.AdaptRecord()
        check(_lib.load().hyp_adapt_select_optimize(self._h, ctypes.byref(rec)))
        self._rec = None
        return {f: getattr(rec, f) for f, _ in rec._fields_ if f != "reserved"}

    def optimize(self) -> dict:
        """hyp_adapt_optimize: re-optimise the current ansatz's parameters."""
        rec = _lib.AdaptRecord()
        check(_lib.load().hyp_adapt_optimize(self._h, ctypes.byref(rec)))
        return {f: getattr(rec, f) for f, _ in rec._fields_ if f != "reserved"}

    def last_gradients(self) -> np.ndarray:
        out = np.empty(self.n_pool)
        check(_lib.load().hyp_adapt_last_gradients(self._h, out.ctypes.data, self.n_pool))
        return out

    def ansatz(self):
        n = ctypes.c_int64()
        check(_lib.load().hyp_adapt_ansatz(self._h, None, None, 0, ctypes.byref(n)))
        ops = np.empty(n.value, dtype=np.int32)
        th = np.empty(n.value)
        check(_lib.load().hyp_adapt_ansatz(self._h, ops.ctypes.data, th.ctypes.data, n.value,
                                           ctypes.byref(n)))
        return ops, th

    def set_ansatz(self, ops, theta):
        ops = np.ascontiguousarray(ops, dtype=np.int32)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        check(_lib.load().hyp_adapt_set_ansatz(self._h, ops.ctypes.data, th.ctypes.data, ops.size))

    def eval(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        e = ctypes.c_double()
        g = np.empty(th.size)
        check(_lib.load().hyp_adapt_eval(self._h, th.ctypes.data if th.size else None,
                                         ctypes.byref(e), g.ctypes.data if th.size else None))
        return e.value, g

    def state(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.ham.sector.dim, device="cuda",
                              dtype=torch.float32 if self.dtype == "f32" else torch.float64)
        check(_lib.load().hyp_adapt_state(self._h, _dev_ptr(out, self.ham.sector.dim, "psi")))
        return out

    def energy_fp64(self) -> float:
        e = ctypes.c_double()
        check(_lib.load().hyp_adapt_energy_fp64(self._h, ctypes.byref(e)))
        return e.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hyp_adapt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hyp_pool_gradients_batched(jobs, tile=None):
    """jobs: list of (sector, ops, psi, sigma, grad_out) tensors; one persistent launch."""
    arr = (_lib.GradJob * len(jobs))()
    for i, (sec, ops, psi, sig, g) in enumerate(jobs):
        arr[i].sector = sec.handle
        arr[i].dtype = _dtype_code(psi)
        arr[i].ops_dev = _dev_ptr(ops, None, "ops")
        arr[i].n_ops = ops.shape[0]
        arr[i].psi_dev = _dev_ptr(psi, sec.dim, "psi")
        arr[i].sigma_dev = _dev_ptr(sig, sec.dim, "sigma")
        arr[i].grad_dev = _dev_ptr(g, ops.shape[0], "grad")
    t = None
    if tile is not None:
        t = ctypes.byref(_lib.SweepTile(int(tile[0]), int(tile[1]), int(tile[2]), 0))
    check(_lib.load().hyp_pool_gradients_batched(arr, len(jobs), t, _stream()))
    return arr


def hyp_tune_pool_gradients(jobs, reps: int = 2):
    """Autotune the batched sweep tile on these jobs: ((threads, chunks, blocks_per_cu), ms)."""
    arr = (_lib.GradJob * len(jobs))()
    for i, (sec, ops, psi, sig, g) in enumerate(jobs):
        arr[i].sector = sec.handle
        arr[i].dtype = _dtype_code(psi)
        arr[i].ops_dev = _dev_ptr(ops, None, "ops")
        arr[i].n_ops = ops.shape[0]
        arr[i].psi_dev = _dev_ptr(psi, sec.dim, "psi")
        arr[i].sigma_dev = _dev_ptr(sig, sec.dim, "sigma")
        arr[i].grad_dev = _dev_ptr(g, ops.shape[0], "grad")
    best = _lib.SweepTile()
    ms = ctypes.c_double()
    check(_lib.load().hyp_tune_pool_gradients(arr, len(jobs), reps, ctypes.byref(best), ctypes.byref(ms),
                                              _stream()))
    return (best.threads, best.chunks, best.blocks_per_cu), ms.value
