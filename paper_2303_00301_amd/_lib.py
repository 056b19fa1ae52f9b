"""ctypes binding of libauxkf.so (include/akf.h).  Argument marshalling only:
every step of the sampler runs in the library's HIP kernels.  The library must
have been built (``python -m paper_2303_00301_amd.build`` or
``__graft_entry__.build()``); there is no fallback."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libauxkf.so")

AKF_OK = 0
NOALLOC_SCRATCH_BYTES = 64 << 20  # AKF_NOALLOC_SCRATCH_BYTES
ERR_NAMES = {1: "AKF_ERR_INVALID", 2: "AKF_ERR_SHAPE", 3: "AKF_ERR_WORKSPACE", 4: "AKF_ERR_HIP",
             5: "AKF_ERR_UNSUPPORTED"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class AkfModel(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("dx", C.c_int32), ("dy", C.c_int32),
        ("m0", C.c_void_p), ("P0", C.c_void_p), ("F", C.c_void_p), ("b", C.c_void_p),
        ("Q", C.c_void_p),
        ("emit", C.c_int32),
        ("H", C.c_void_p), ("R", C.c_void_p),
        ("site", C.c_void_p),
        ("nu", C.c_double), ("scale", C.c_double),
        ("dyn", C.c_int32), ("dyn_par", C.c_double * 4),
        ("dtype", C.c_int32),
        ("obs_beta", C.c_double), ("slr_var", C.c_double),
    ]


# akf_dtype
AKF_F64, AKF_F32 = 0, 1


class AkfLgssm(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("dx", C.c_int32), ("dy", C.c_int32),
        ("m0", C.c_void_p), ("P0", C.c_void_p),
        ("F", C.c_void_p), ("logq", C.c_void_p),
        ("H", C.c_void_p), ("logr", C.c_void_p),
        ("y", C.c_void_p),
    ]


class AkfChain(C.Structure):
    _fields_ = [
        ("model", AkfModel),
        ("y", C.c_void_p), ("x", C.c_void_p), ("xi", C.c_void_p), ("unif", C.c_void_p),
        ("delta", C.c_double), ("order", C.c_int32),
        ("log_ratio", C.c_void_p), ("accepted", C.c_void_p), ("logZ_fwd", C.c_void_p),
        ("logZ_rev", C.c_void_p), ("status", C.c_void_p),
    ]


# name -> (restype, argtypes); the exported symbols of include/akf.h
_vp, _sz, _i32, _d = C.c_void_p, C.c_size_t, C.c_int32, C.c_double
_MP = C.POINTER(AkfModel)
SIGNATURES = {
    "akf_last_error": (C.c_char_p, []),
    "akf_mh_workspace_bytes": (_sz, [_MP, _i32, _i32]),
    "akf_mh_step": (C.c_int, [_MP, _vp, _vp, _d, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                              _vp, _sz, _i32, _vp]),
    "akf_mh_run": (C.c_int, [_MP, _vp, _vp, _d, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                             _vp, _sz, _i32, _vp]),
    "akf_mh_step_noalloc": (C.c_int, [_MP, _vp, _vp, _d, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _i32, _vp]),
    "akf_mh_first_order_workspace_bytes": (_sz, [_MP, _i32]),
    "akf_mh_run_first_order": (C.c_int, [_MP, _vp, _vp, _d, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _vp, _vp, _sz, _i32, _vp]),
    "akf_mh_reuse_workspace_bytes": (_sz, [_MP, _i32, _i32]),
    "akf_mh_run_reuse": (C.c_int, [_MP, _vp, _vp, _d, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _sz, _i32, _vp]),
    "akf_mh_factorised_workspace_bytes": (_sz, [_MP, _i32]),
    "akf_mh_step_factorised": (C.c_int, [_MP, _vp, _vp, _d, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _vp, _vp, _vp, _sz, _vp]),
    "akf_mh_run_factorised": (C.c_int, [_MP, _vp, _vp, _d, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _sz, _vp]),
    "akf_filter_workspace_bytes": (_sz, [_MP, _i32]),
    "akf_aux_filter": (C.c_int, [_MP, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32, _vp]),
    "akf_sampler_workspace_bytes": (_sz, [_MP, _i32]),
    "akf_rts_sample": (C.c_int, [_MP, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32, _vp]),
    "akf_sqrt_workspace_bytes": (_sz, [_MP, _i32]),
    "akf_sqrt_filter_sample": (C.c_int, [_MP, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _sz, _i32, _vp]),
    "akf_dnc_workspace_bytes": (_sz, [_MP]),
    "akf_dnc_sample": (C.c_int, [_MP, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "akf_smoother_workspace_bytes": (_sz, [_MP, _i32]),
    "akf_smoother": (C.c_int, [_MP, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32, _vp]),
    "akf_lgssm_workspace_bytes": (_sz, [C.c_void_p, _i32]),
    "akf_lgssm_loglik": (C.c_int, [C.c_void_p, _vp, _vp, _vp, _vp, _sz, _i32, _vp]),
    "akf_lgssm_loglik_grad": (C.c_int, [C.c_void_p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32,
                                        _vp]),
    "akf_gibbs_state_bytes": (_sz, [C.c_void_p]),
    "akf_gibbs_workspace_bytes": (_sz, [C.c_void_p, _i32]),
    "akf_gibbs_init": (C.c_int, [C.c_void_p, _vp, _d, _vp, _vp, _vp, _sz, _vp, _vp, _sz, _i32,
                                 _vp]),
    "akf_gibbs_sweep": (C.c_int, [C.c_void_p, _vp, _vp, _vp, _vp, _vp, _sz, _d, _d, _vp, _vp,
                                  _vp, _d, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                  _i32, _vp]),
    "akf_batch_plan_create": (C.c_int, [C.POINTER(C.c_void_p), _i32, C.POINTER(AkfChain), _i32,
                                        _i32, C.c_char_p, _vp]),
    "akf_batch_mh_run": (C.c_int, [_vp, _i32, _vp]),
    "akf_batch_plan_info": (C.c_int, [_vp, _i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]),
    "akf_batch_plan_destroy": (None, [_vp]),
    "akf_timing_enable": (C.c_int, [_i32, _i32]),
    "akf_timing_collect": (C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
}

# kernel families of akf_timing_enable
FAMILIES = {"filter_fold": 0, "filter_up": 1, "filter_down": 2, "filter_final": 3,
            "samp_build": 4, "samp_fold": 5, "samp_up": 6, "samp_down": 7, "samp_final": 8,
            "fact_scan": 9, "lin": 10, "dnc": 11, "fixed_mean_fold": 12, "fixed_samp_fold": 13,
            "adj_grad": 14, "adj_build": 15, "batch_fold16": 16, "batch_fold32": 17,
            "batch_fold64": 18, "batch_sbuild16": 19, "batch_sbuild32": 20,
            "batch_sbuild64": 21, "mh": 22}

_lib = None


class AkfError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load the library and declare every exported entry point."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise AkfError(f"HIP library not built: {path} is missing "
                           "(run `python -m paper_2303_00301_amd.build`)")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int, what: str):
    if rc != AKF_OK:
        msg = load().akf_last_error()
        raise AkfError(f"{what} failed with {ERR_NAMES.get(rc, rc)}: "
                       f"{msg.decode() if msg else ''}")
