"""ctypes declarations of libhyperion_mi355x.so (the C ABI in
include/hyperion_mi355x.h).  Loading fails loudly when the library is
missing: there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhyperion_mi355x.so")

HYP_OK, HYP_ERR_ARG, HYP_ERR_SECTOR, HYP_ERR_NONREAL, HYP_ERR_NOMEM, HYP_ERR_HIP, HYP_ERR_UNSUPPORTED = range(7)
HYP_F64, HYP_F32 = 0, 1
STATUS_NAMES = {0: "HYP_OK", 1: "HYP_ERR_ARG", 2: "HYP_ERR_SECTOR", 3: "HYP_ERR_NONREAL",
                4: "HYP_ERR_NOMEM", 5: "HYP_ERR_HIP", 6: "HYP_ERR_UNSUPPORTED"}


class HypExc(ctypes.Structure):
    _fields_ = [("cre", ctypes.c_uint32), ("ann", ctypes.c_uint32)]


class AdaptOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("max_bfgs", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("recycle_hessian", ctypes.c_int32),
                ("tie_tol", ctypes.c_double), ("gtol", ctypes.c_double),
                ("gmax_stop", ctypes.c_double)]


class AdaptRecord(ctypes.Structure):
    _fields_ = [("selected", ctypes.c_int32), ("tie_count", ctypes.c_int32),
                ("n_evals", ctypes.c_int32), ("bfgs_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("gmax", ctypes.c_double), ("energy_before", ctypes.c_double),
                ("energy", ctypes.c_double), ("grad_ms", ctypes.c_double),
                ("opt_ms", ctypes.c_double), ("grad_inf", ctypes.c_double)]


class GradJob(ctypes.Structure):
    _fields_ = [("sector", ctypes.c_void_p), ("dtype", ctypes.c_int), ("ops_dev", ctypes.c_void_p),
                ("n_ops", ctypes.c_int64), ("psi_dev", ctypes.c_void_p),
                ("sigma_dev", ctypes.c_void_p), ("grad_dev", ctypes.c_void_p)]


class SweepTile(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class HypError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_ci = ctypes.c_int
_d = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "hyp_last_error": (ctypes.c_char_p, []),
    "hyp_sector_create": (_ci, [_ci, _ci, _ci, ctypes.POINTER(_vp)]),
    "hyp_sector_destroy": (_ci, [_vp]),
    "hyp_sector_dim": (_i64, [_vp]),
    "hyp_sector_rank": (_ci, [_vp, _vp, _i64, _vp]),
    "hyp_sector_unrank": (_ci, [_vp, _vp, _i64, _vp]),
    "hyp_build_hamiltonian": (_ci, [_vp, _vp, _vp, _vp, _i64, _vp, ctypes.POINTER(_vp)]),
    "hyp_ham_destroy": (_ci, [_vp]),
    "hyp_assemble_pauli": (_ci, [_ci, _vp, _vp, _d, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp]),
    "hyp_build_hamiltonian_integrals": (_ci, [_vp, _ci, _vp, _vp, _d, _vp, ctypes.POINTER(_vp)]),
    "hyp_ham_is_structured": (_ci, [_vp]),
    "hyp_apply_h": (_ci, [_vp, _ci, _vp, _vp, _vp]),
    "hyp_tune_apply_h": (_ci, [_vp, _ci, _vp, _vp, _ci, _vp, ctypes.POINTER(_ci), ctypes.POINTER(_d)]),
    "hyp_expectation": (_ci, [_vp, _ci, _vp, _vp, _vp, _vp]),
    "hyp_pool_gradients": (_ci, [_vp, _ci, _vp, _i64, _vp, _vp, _vp, _vp]),
    "hyp_pool_check": (_ci, [_vp]),
    "hyp_pool_gradients_noalloc": (_ci, [_vp, _ci, _vp, _i64, _vp, _vp, _vp, _vp]),
    "hyp_apply_excitation": (_ci, [_vp, _ci, HypExc, _d, _vp, _vp]),
    "hyp_set_sweep_mode": (_ci, [_ci]),
    "hyp_set_row_staging": (_ci, [_ci]),
    "hyp_set_support_skip": (_ci, [_ci]),
    "hyp_set_same_spin_groups": (_ci, [_ci]),
    "hyp_set_same_spin_cores": (_ci, [_ci]),
    "hyp_set_mixed_matrix_cores": (_ci, [_ci]),
    "hyp_set_pool_kind": (_ci, [_ci]),
    "hyp_apply_excitations": (_ci, [_vp, _ci, _vp, _vp, _i64, _vp, _vp]),
    "hyp_csr_build": (_ci, [_vp, _vp, ctypes.POINTER(_vp)]),
    "hyp_csr_apply": (_ci, [_vp, _ci, _vp, _vp, _vp]),
    "hyp_csr_export": (_ci, [_vp, _vp, _vp, _vp]),
    "hyp_csr_nnz": (_i64, [_vp]),
    "hyp_csr_destroy": (_ci, [_vp]),
    "hyp_pool_gradients_batched": (_ci, [_vp, _ci, _vp, _vp]),
    "hyp_tune_pool_gradients": (_ci, [_vp, _ci, _ci, ctypes.POINTER(SweepTile), ctypes.POINTER(_d), _vp]),
    "hyp_mlp_create": (_ci, [_vp, _i64, ctypes.POINTER(_vp)]),
    "hyp_mlp_destroy": (_ci, [_vp]),
    "hyp_mlp_params": (_ci, [_vp, _vp]),
    "hyp_mlp_forward": (_ci, [_vp, _vp, _i64, _vp, _vp]),
    "hyp_mlp_train_step": (_ci, [_vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp]),
    "hyp_mlp_grads": (_ci, [_vp, _vp]),
    "hyp_mlp_get_state": (_ci, [_vp, _vp]),
    "hyp_mlp_set_state": (_ci, [_vp, _vp]),
    "hyp_screen_static": (_ci, [_ci, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "hyp_occupations": (_ci, [_vp, _ci, _vp, _vp, _vp, _vp]),
    "hyp_features": (_ci, [_vp, _vp, _vp, _vp, _vp, _i64, _ci, _vp, _d, _vp, _vp]),
    "hyp_screen_update": (_ci, [_vp, _i64, _vp, _vp, _vp]),
    "hyp_screen_base": (_ci, [_vp, _i64, ctypes.c_float, _vp, _vp]),
    "hyp_screen_batch": (_ci, [_vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp, _vp, _vp]),
    "hyp_rank_scores": (_ci, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "hyp_adapt_create": (_ci, [_vp, _ci, _vp, _i64, ctypes.POINTER(AdaptOpts), ctypes.POINTER(_vp)]),
    "hyp_adapt_destroy": (_ci, [_vp]),
    "hyp_adapt_iterate": (_ci, [_vp, _vp, _i64, ctypes.POINTER(AdaptRecord)]),
    "hyp_adapt_gradients": (_ci, [_vp, _vp, _i64, ctypes.POINTER(AdaptRecord)]),
    "hyp_adapt_select_optimize": (_ci, [_vp, ctypes.POINTER(AdaptRecord)]),
    "hyp_adapt_optimize": (_ci, [_vp, _vp]),
    "hyp_adapt_last_gradients": (_ci, [_vp, _vp, _i64]),
    "hyp_adapt_ansatz": (_ci, [_vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]),
    "hyp_adapt_set_ansatz": (_ci, [_vp, _vp, _vp, _i64]),
    "hyp_adapt_eval": (_ci, [_vp, _vp, ctypes.POINTER(_d), _vp]),
    "hyp_adapt_state": (_ci, [_vp, _vp]),
    "hyp_adapt_energy_fp64": (_ci, [_vp, ctypes.POINTER(_d)]),
    "hyp_profile_enable": (_ci, [_ci]),
    "hyp_profile_reset": (_ci, []),
    "hyp_profile_count": (_ci, []),
    "hyp_profile_get": (_ci, [_ci, ctypes.c_char_p, _ci, ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
}

_lib = None


def load():
    """Load the library (built by __graft_entry__.build / build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded; loaded the other way round, torch finds no HIP device
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != HYP_OK:
        raise HypError(status, load().hyp_last_error().decode(errors="replace"))
