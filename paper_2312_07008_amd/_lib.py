"""ctypes loader of libdfpt2.so (built in-tree by ``paper_2312_07008_amd.build``)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdfpt2.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_WORKSPACE = -2
ERR_HIP = -3
ERR_NOT_CONVERGED = -4
ERR_NONFINITE = -5
ERR_UNSUPPORTED = -6
STATIC_SCRATCH_BYTES = 64 << 20  # DFPT2_STATIC_SCRATCH_BYTES

FP64 = 0
BF16_SLICED = 1
FP8_SLICED = 2
INT8_SLICED = 3
TRUNC_CUMULATIVE, TRUNC_FRACTION, TRUNC_CUTOFF, TRUNC_FIXED = 0, 1, 2, 3


class DfptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"dfpt2 status {status}: {message}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("n_core", ctypes.c_int64),
        ("n_act", ctypes.c_int64),
        ("n_vir", ctypes.c_int64),
        ("n_aux", ctypes.c_int64),
        ("s", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("slices_gemm1", ctypes.c_int32),
        ("slices_gemm2", ctypes.c_int32),
        ("density_convention", ctypes.c_int32),
        ("pair_batch", ctypes.c_int64),
    ]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_int = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "dfpt2_last_error": (ctypes.c_char_p, []),
    "dfpt2_status_string": (ctypes.c_char_p, [_int]),
    "dfpt2_version": (ctypes.c_char_p, []),
    "dfpt2_workspace_size": (_int, [ctypes.POINTER(Opts), ctypes.POINTER(_sz)]),
    "dfpt2_build_vv_density": (_int, [ctypes.POINTER(Opts), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _sz, _vp]),
    "dfpt2_build_vv_density_noalloc": (_int, [ctypes.POINTER(Opts), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                              _vp]),
    "fno_truncate_workspace_size": (_int, [_i64, ctypes.POINTER(_sz)]),
    "fno_truncate": (_int, [_vp, _i64, _dbl, _dbl, _vp, _vp, ctypes.POINTER(_i64),
                            ctypes.POINTER(_dbl), _vp, _sz, _vp]),
    "fno_truncate_rule": (_int, [_vp, _i64, _int, _dbl, _dbl, _vp, _vp, ctypes.POINTER(_i64),
                                 ctypes.POINTER(_dbl), _vp, _sz, _vp]),
    "dfpt2_eigh_sym": (_int, [_vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "dfpt2_active_particle_workspace_size": (_int, [ctypes.POINTER(Opts), ctypes.POINTER(_sz)]),
    "dfpt2_add_active_particle_density": (_int, [ctypes.POINTER(Opts), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "dfpt2_cumulant_singles_workspace_size": (_int, [ctypes.POINTER(Opts), _int, ctypes.POINTER(_sz)]),
    "dfpt2_add_cumulant_singles_density": (_int, [ctypes.POINTER(Opts), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                  _sz, _vp]),
    "pp_ladder_workspace_size": (_int, [_i64, _i64, _i64, _i64, ctypes.POINTER(_sz)]),
    "pp_ladder": (_int, [_i64, _i64, _i64, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _sz, _vp]),
    "naf_compress_workspace_size": (_int, [ctypes.POINTER(Opts), ctypes.POINTER(_sz)]),
    "naf_compress": (_int, [ctypes.POINTER(Opts), _vp, _dbl, _vp, _vp, ctypes.POINTER(_i64), _vp, _sz, _vp]),
    "pt2_correction_workspace_size": (_int, [ctypes.POINTER(Opts), _i64, ctypes.POINTER(_sz)]),
    "pt2_energy_correction": (_int, [ctypes.POINTER(Opts), _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp,
                                     _vp, _sz, _vp]),
    "pairscreen_num_params": (_int, []),
    "pairscreen_workspace_size": (_int, [ctypes.POINTER(Opts), ctypes.POINTER(_sz)]),
    "pairscreen_features": (_int, [ctypes.POINTER(Opts), _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pairscreen_mlp_forward": (_int, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "pairscreen_backward_workspace_size": (_int, [_i64, ctypes.POINTER(_sz)]),
    "pairscreen_mlp_backward": (_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "pairscreen_adam_step": (_int, [_vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _i64, _vp]),
    "pairscreen_train_workspace_size": (_int, [_i64, ctypes.POINTER(_sz)]),
    "pairscreen_train": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, _vp, _vp, _sz, _vp]),
    "pairscreen_targets": (_int, [_vp, _vp, _i64, _i64, _vp, _vp]),
    "pairscreen_build_mask": (_int, [_vp, _vp, _i64, _i64, _dbl, _dbl, _int, _vp, ctypes.POINTER(_i64), _vp, _sz,
                                     _vp]),
    "dfpt2_profile_enable": (_int, [_int]),
    "dfpt2_profile_read": (_int, [ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
}

STAGES = ["pair", "density", "split", "reduce", "active", "eigh", "transform", "kept_pair", "screen", "split_t",
          "ladder_transform", "ladder", "pair_epilogue"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libdfpt2.so not found at {path}; build it with `python -m paper_2312_07008_amd.build` "
            "(the DF-DSRG-PT2 pass has no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != OK:
        lib = load()
        raise DfptError(status, lib.dfpt2_last_error().decode() or lib.dfpt2_status_string(status).decode())
