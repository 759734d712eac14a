"""ctypes binding of libnepmi.so (argument marshalling only).

Every computation runs in the HIP library; this module only passes device
pointers, sizes and the current HIP stream.  It raises if the library is not
built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libnepmi.so"

OK, INVALID_ARG, CELL_TOO_SMALL, NEIGHBOR_OVERFLOW, HIP_ERROR, NAN_DETECTED, UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
_CODES = {-1: "INVALID_ARG", -2: "CELL_TOO_SMALL", -3: "NEIGHBOR_OVERFLOW", -4: "HIP_ERROR", -5: "NAN_DETECTED",
          -6: "UNSUPPORTED"}


class NepmiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nepmi error {_CODES.get(code, code)}: {msg}")
        self.code = code


class HParams(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_radial", C.c_int32), ("n_angular", C.c_int32),
                ("basis_radial", C.c_int32), ("basis_angular", C.c_int32), ("l_max", C.c_int32),
                ("use_4body", C.c_int32), ("use_5body", C.c_int32), ("n_hidden", C.c_int32),
                ("reserved", C.c_int32), ("rc_radial", C.c_double), ("rc_angular", C.c_double)]

    @classmethod
    def from_any(cls, h):
        d = h if isinstance(h, dict) else h.as_dict()
        return cls(d["n_species"], d["n_radial"], d["n_angular"], d["basis_radial"], d["basis_angular"],
                   d["l_max"], d["use_4body"], d["use_5body"], d["n_hidden"], 0, d["rc_radial"], d["rc_angular"])


# (name, restype, argtypes) of every exported entry point, in header order.
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_hp = C.POINTER(HParams)
_i64p, _dp = C.POINTER(C.c_int64), C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
SIGNATURES = [
    ("nepmi_last_error", C.c_char_p, []),
    ("nepmi_param_count", C.c_int, [_hp, _i64p]),
    ("nepmi_descriptor_dim", C.c_int, [_hp, C.POINTER(C.c_int32)]),
    ("nepmi_model_create", C.c_int, [_hp, C.POINTER(_vp)]),
    ("nepmi_supported", C.c_int, [_hp]),
    ("nepmi_model_set_params", C.c_int, [_vp, _vp, _vp]),
    ("nepmi_model_reuse_lists", C.c_int, [_vp, _i32]),
    ("nepmi_model_destroy", None, [_vp]),
    ("nepmi_compute", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("nepmi_compute_noalloc", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("nepmi_descriptors", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp]),
    ("nepmi_neighbors", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp]),
    ("nepmi_autotune", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, C.POINTER(C.c_int32), _vp]),
    ("nepmi_set_variants", C.c_int, [_vp, _i32, _i32]),
    ("nepmi_get_variants", C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("nepmi_set_gather_variant", C.c_int, [_vp, _i32]),
    ("nepmi_get_gather_variant", C.c_int, [_vp, C.POINTER(C.c_int32)]),
    ("nepmi_backward_params", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("nepmi_loss_grad", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp, _vp, _dp, _i32, _vp, _vp, _vp]),
    ("nepmi_md_create", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _dp, _d, _d, C.POINTER(_vp), _vp]),
    ("nepmi_compute_f64", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("nepmi_backward_params_f64", C.c_int, [_vp, _i32, _i64p, _dp, _i32p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("nepmi_adam_step", C.c_int, [C.c_int64, _vp, _vp, _vp, _vp, C.c_int64, C.c_double, C.c_double, C.c_double,
                                  C.c_double, _vp]),
    ("nepmi_lr_schedule", C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double, _dp]),
    ("nepmi_loss_weights", C.c_int, [C.c_double, C.c_double, _dp, _dp, _i32, _dp]),
    ("nepmi_md_step", C.c_int, [_vp, _i32, _vp]),
    ("nepmi_md_step_timed", C.c_int, [_vp, _i32, _dp, _vp]),
    ("nepmi_md_get", C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("nepmi_md_stats", C.c_int, [_vp, _i64p, _i64p, _i64p]),
    ("nepmi_md_capacity", C.c_int, [_vp, _i32, _i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("nepmi_md_destroy", None, [_vp]),
    ("nepmi_md_time_kernels", C.c_int, [_vp, _i32, _dp, _vp]),
]

_lib = None


def load():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_06969_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(str(LIB_PATH))
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != 0:
        raise NepmiError(rc, load().nepmi_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _host_i64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(_i64p)


def _host_f64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    return a, a.ctypes.data_as(_dp)


def param_count(hp) -> int:
    out = C.c_int64()
    check(load().nepmi_param_count(C.byref(HParams.from_any(hp)), C.byref(out)))
    return out.value


def descriptor_dim(hp) -> int:
    out = C.c_int32()
    check(load().nepmi_descriptor_dim(C.byref(HParams.from_any(hp)), C.byref(out)))
    return out.value


def supported(hp) -> bool:
    return bool(load().nepmi_supported(C.byref(HParams.from_any(hp))))
