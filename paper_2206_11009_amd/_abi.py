"""ctypes mirror of ``include/otip.h`` (argument marshalling only).

Every function here forwards to the HIP library ``libotip.so``; none of them
computes anything.  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotip.so")

OTIP_OK, OTIP_EINVAL, OTIP_ENOMEM, OTIP_EHIP, OTIP_EMAXITER, OTIP_ENUMERIC, OTIP_EUNSUPPORTED = range(7)
OTIP_LS_AUTO, OTIP_LS_PCG, OTIP_LS_DIRECT = 0, 1, 2
OTIP_FP64, OTIP_MIXED = 0, 1
OTIP_COST_SQEUCLID, OTIP_COST_L1, OTIP_COST_L2, OTIP_COST_LINF = 0, 1, 2, 3

_c_i32, _c_i64, _c_f64, _p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class otip_params(ctypes.Structure):
    _fields_ = [
        ("tol", _c_f64), ("cg_tol_pred", _c_f64), ("cg_tol_corr", _c_f64),
        ("max_iter", _c_i32), ("cg_max_iter", _c_i32), ("max_corr", _c_i32),
        ("step_scale", _c_f64), ("kappa", _c_f64), ("switch_window", _c_i32),
        ("switch_drop", _c_f64), ("mcc_beta_min", _c_f64), ("mcc_beta_max", _c_f64),
        ("mcc_delta", _c_f64), ("mcc_accept", _c_f64), ("remove_gate", _c_f64),
        ("remove_rel", _c_f64), ("pivot_tol", _c_f64), ("cert_rel", _c_f64),
        ("polish_tol", _c_f64), ("polish_steps", _c_i32), ("drop_rel", _c_f64),
        ("cg_eta", _c_f64), ("cg_floor", _c_f64), ("linear_solver", _c_i32),
        ("precision", _c_i32), ("dense_max_n", _c_i32), ("force_switch_at", _c_i32),
        ("enter_cap", _c_i32), ("scale", _c_i32), ("verbose", _c_i32), ("profile", _c_i32),
        ("switch_cost", _c_i32),
        ("batch_workers", _c_i32),
        ("price_tile", _c_i32),
        ("ws_kappa", ctypes.c_double),
        ("heur_radius", _c_f64), ("heur_run", _c_i32), ("switch_back_grow", _c_f64),
        ("force_switch_back_at", _c_i32), ("schur_reuse", _c_i32), ("ws_union", _c_i32),
    ]


class otip_problem(ctypes.Structure):
    _fields_ = [("m", _c_i32), ("n", _c_i32), ("a", _p), ("b", _p), ("xs", _p), ("xt", _p),
                ("y0", _p), ("z0", _p), ("cost_kind", _c_i32)]


class otip_info(ctypes.Structure):
    _fields_ = [
        ("status", _c_i32), ("iterations", _c_i32), ("cg_iterations", _c_i32),
        ("direct_iterations", _c_i32), ("nnz", _c_i64), ("psi_max", _c_i64),
        ("objective", _c_f64), ("dual_bound", _c_f64), ("rel_gap", _c_f64),
        ("marginal_residual", _c_f64), ("r_min", _c_f64), ("max_fill_pct", _c_f64),
        ("seconds_total", _c_f64), ("seconds_pricing", _c_f64), ("seconds_newton", _c_f64),
        ("seconds_direct", _c_f64), ("seconds_update", _c_f64), ("seconds_setup", _c_f64),
        ("seconds_final", _c_f64), ("pricing_scans", _c_i64), ("spmv_launches", _c_i64),
        ("spmv_ms", _c_f64), ("spmv_bytes", _c_f64), ("price_launches", _c_i64),
        ("price_ms", _c_f64), ("price_elems", _c_f64), ("diag_launches", _c_i64),
        ("diag_ms", _c_f64), ("diag_flops", _c_f64), ("update_launches", _c_i64),
        ("update_ms", _c_f64), ("update_flops", _c_f64),
        ("heuristic_scans", _c_i64), ("switches_back", _c_i64), ("patterns_kept", _c_i64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); exactly the declarations of include/otip.h
SIGNATURES = {
    "otip_version": (ctypes.c_int, []),
    "otip_source_id": (ctypes.c_char_p, []),
    "otip_params_default": (None, [ctypes.POINTER(otip_params)]),
    "otip_create": (ctypes.c_int, [ctypes.POINTER(_p), ctypes.c_int, _p]),
    "otip_destroy": (None, [_p]),
    "otip_last_error": (ctypes.c_char_p, [_p]),
    "otip_solve": (ctypes.c_int, [_p, ctypes.POINTER(otip_problem), ctypes.POINTER(otip_params),
                                  ctypes.POINTER(_p)]),
    "otip_solve_batch": (ctypes.c_int, [_p, ctypes.POINTER(otip_problem), _c_i32,
                                        ctypes.POINTER(otip_params), ctypes.POINTER(_p)]),
    "otip_result_info": (ctypes.c_int, [_p, ctypes.POINTER(otip_info)]),
    "otip_result_copy": (ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
    "otip_result_free": (None, [_p]),
    "otip_price": (ctypes.c_int, [_p, _c_i32, _c_i32, _p, _p, _p, _p, _p, _c_i64, _c_i32, _c_i32,
                                  _c_i32, _p, _p, _p, ctypes.POINTER(_c_i64),
                                  ctypes.POINTER(_c_i64)]),
    "otip_price_subset": (ctypes.c_int, [_p, _c_i32, _c_i32, _p, _p, _p, _p, _p, _c_i64, _c_i32,
                                         _c_i64, _p, _p, _p, ctypes.POINTER(_c_i64),
                                         ctypes.POINTER(_c_i64), ctypes.POINTER(_c_i64)]),
    "otip_rmin": (ctypes.c_int, [_p, _c_i32, _c_i32, _p, _p, _p, _p, _c_i32,
                                 ctypes.POINTER(_c_f64), ctypes.POINTER(_c_i64)]),
    "otip_kron_apply": (ctypes.c_int, [_p, _c_i32, _c_i32, _p, _p, _p]),
    "otip_kron_apply_t": (ctypes.c_int, [_p, _c_i32, _c_i32, _p, _p, _p]),
    "otip_kron_apply_noalloc": (ctypes.c_int, [_p, _c_i32, _c_i32, _p, _p, _p]),
    "otip_schur": (ctypes.c_int, [_p, _c_i32, _c_i32, _c_i64, _p, _p, ctypes.POINTER(_c_i64),
                                  _p, _p, _p, _p, _p]),
    "otip_pcg": (ctypes.c_int, [_p, _c_i32, _c_i64, _p, _p, _p, _p, _p, _c_f64, _c_i32, _c_i32,
                                ctypes.POINTER(_c_i32), ctypes.POINTER(_c_f64), _p]),
    "otip_ldl_solve": (ctypes.c_int, [_p, _c_i32, _c_i64, _p, _p, _p, _c_f64, _c_i32, _p, _p,
                                      ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i64)]),
    "otip_state_save": (ctypes.c_int, [_p, _p, _c_i64, ctypes.POINTER(_c_i64)]),
    "otip_state_load": (ctypes.c_int, [_p, _p, _c_i64]),
    "otip_ws_param_count": (_c_i64, []),
    "otip_ws_forward": (ctypes.c_int, [_p, _p, _c_i32, _c_i32, _c_i32, _p, _p]),
    "otip_ws_grad": (ctypes.c_int, [_p, _p, _c_i32, _c_i32, _c_i32, _p, _p, _p,
                                    ctypes.POINTER(_c_f64)]),
    "otip_ws_adam": (ctypes.c_int, [_p, _p, _p, _p, _p, _c_i32, _c_f64, _c_f64, _c_f64, _c_f64]),
    "otip_ws_predict": (ctypes.c_int, [_p, _p, _c_i32, _p, _p, _p, _p]),
}

_lib = None


def load():
    """Load libotip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch provides the device memory and streams: its HIP runtime must be
        # the one in the process before the library binds to libamdhip64
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2206_11009_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        # a library built from other sources than the ones beside it is refused
        from .build import source_id
        built, here = L.otip_source_id().decode(), source_id()
        if built != here:
            raise ImportError(f"{LIB_PATH} was built from other sources ({built}, sources "
                              f"here {here}); rebuild with paper_2206_11009_amd/build.py")
        _lib = L
    return _lib
