"""ctypes binding of libmlb.so (argument marshalling only).

Every step of the path runs in the library's HIP kernels; this module only
converts Python values and torch tensors (device memory, streams) into the
plain pointers of include/mlb.h.  It raises if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlb.so")

MAX_SPECIES = 4
Q = 19
NPASS = 6

MLB_OK = 0
STATUS = {0: "MLB_OK", -1: "MLB_EINVAL", -2: "MLB_ENOMEM", -3: "MLB_EHIP", -4: "MLB_EUNSTABLE", -5: "MLB_ENONFINITE",
          -6: "MLB_ESTATE", -7: "MLB_EUNSUPPORTED"}

SCHEME_CN_J1, SCHEME_FE = 0, 1
TAIL_AUTO, TAIL_DIRECT, TAIL_SPECTRAL = 0, 1, 2
PART_MF, PART_TAIL, PART_DISS, PART_EXT, PART_ALL = 1, 2, 4, 8, 15


class MlbError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("nspecies", C.c_int32), ("precision", C.c_int32), ("scheme", C.c_int32),
        ("tail_mode", C.c_int32), ("walls_y", C.c_int32),
        ("tau", C.c_double), ("kT", C.c_double),
        ("mass", C.c_double * MAX_SPECIES),
        ("sigma", C.c_double * MAX_SPECIES),
        ("eps", C.c_double * (MAX_SPECIES * MAX_SPECIES)),
        ("rc_factor", C.c_double),
        ("ext_force", C.c_double * (MAX_SPECIES * 3)),
        ("wall_ux", C.c_double * 2),
    ]


# (name, restype, argtypes)
_SIGS = [
    ("mlb_workspace_bytes", C.c_size_t, [C.POINTER(Params)]),
    ("mlb_init_mixture", C.c_int, [C.POINTER(Params), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.POINTER(C.c_void_p)]),
    ("mlb_init_mixture_ex", C.c_int, [C.POINTER(Params), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                      C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("mlb_init_mixture_static", C.c_int, [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(C.c_void_p)]),
    ("mlb_check_stability", C.c_int, [C.POINTER(Params), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mlb_tuning", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("mlb_tuning_ex", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_double)]),
    ("mlb_tuning_groups", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("mlb_tuning_gather1_shape", C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("mlb_step", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("mlb_moments", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mlb_forces", C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p]),
    ("mlb_fields", C.c_int, [C.c_void_p] + [C.c_void_p] * 7 + [C.c_void_p]),
    ("mlb_get_populations", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mlb_set_populations", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mlb_set_step_count", C.c_int, [C.c_void_p, C.c_int64]),
    ("mlb_set_force_profile", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_conserved", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_record_mode", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    ("mlb_record_spread", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("mlb_series_capacity", C.c_int32, []),
    ("mlb_series_reset", C.c_int, [C.c_void_p, C.c_void_p]),
    ("mlb_fit_series", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_fit_series_ex", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_get_series", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32,
                                 C.POINTER(C.c_int32), C.c_void_p]),
    ("mlb_step_count", C.c_int64, [C.c_void_p]),
    ("mlb_profile_begin", C.c_int, [C.c_void_p]),
    ("mlb_profile_end", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p]),
    ("mlb_pass_name", C.c_char_p, [C.c_int32]),
    ("mlb_set_graph", C.c_int, [C.c_void_p, C.c_int32]),
    ("mlb_destroy", C.c_int, [C.c_void_p]),
    ("mlb_last_error", C.c_char_p, []),
    ("mlb_batch_workspace_bytes", C.c_size_t, [C.POINTER(Params), C.c_int32]),
    ("mlb_init_batch", C.c_int, [C.POINTER(Params), C.c_int32, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_void_p), C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("mlb_batch_step", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("mlb_batch_moments", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mlb_batch_get_populations", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("mlb_batch_set_populations", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("mlb_batch_set_step_count", C.c_int, [C.c_void_p, C.c_int64]),
    ("mlb_batch_record_modes", C.c_int, [C.c_void_p, C.c_void_p]),
    ("mlb_batch_fit", C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_batch_fit_ex", C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_batch_get_series", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.c_int32, C.POINTER(C.c_int32), C.c_void_p]),
    ("mlb_batch_tuning", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("mlb_batch_tuning_ex", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double)]),
    ("mlb_batch_tuning_groups", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("mlb_batch_tuning_gather1_shape", C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("mlb_batch_profile_begin", C.c_int, [C.c_void_p]),
    ("mlb_batch_profile_end", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p]),
    ("mlb_batch_step_count", C.c_int64, [C.c_void_p]),
    ("mlb_batch_destroy", C.c_int, [C.c_void_p]),
    ("mlb_net_param_count", C.c_size_t, []),
    ("mlb_net_workspace_bytes", C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("mlb_net_create", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    ("mlb_net_set_params", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_void_p]),
    ("mlb_net_get_params", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_void_p]),
    ("mlb_net_set_scales", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double]),
    ("mlb_net_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mlb_net_train_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_float, C.c_int32,
                                     C.POINTER(C.c_double), C.POINTER(C.c_float), C.c_void_p]),
    ("mlb_net_pool_stats", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                     C.c_void_p]),
    ("mlb_net_pool_rescale", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double,
                                       C.c_void_p]),
    ("mlb_net_rel_error", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    ("mlb_net_adam_steps", C.c_int32, [C.c_void_p]),
    ("mlb_net_destroy", C.c_int, [C.c_void_p]),
    ("mlb_set_closure", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double]),
    ("mlb_closure_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("mlb_closure_usage", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("mlb_closure_sample", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
]
OPT_TUNE, OPT_NO_GRAPH, OPT_NO_STABILITY_CHECK = 1, 2, 512
STATIC_WORKSPACE_BYTES = 64 << 20   # MLB_STATIC_WORKSPACE_BYTES


def opt_tiling(shape: int, order: int, gather1_split: int = 0, sign_groups: int = 0, own_tiles: int = 0) -> int:
    """Option bits of a fixed float32 tiling (MLB_OPT_TILING,
    MLB_OPT_GATHER1_SPLIT, MLB_OPT_GATHER1_SIGN_GROUPS and
    MLB_OPT_GATHER1_OWN_TILES in mlb.h; split 0 = the default, 3; sign_groups
    1 = the sign-grouped shell loop; own_tiles 1 = the first gather on 4x8x8
    tiles)."""
    return (((shape + 1) & 15) << 4 | (order & 1) << 8 | (gather1_split & 3) << 10
            | (2 if sign_groups else 1) << 12 | (2 if own_tiles else 1) << 14)

_lib = None


def load() -> C.CDLL:
    """Load libmlb.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(or python paper_1105_3634_amd/build.py); there is no fallback path")
    # torch first: its HIP runtime owns the device memory and streams handed to
    # the library, and the library must bind to that same runtime (same
    # soname).  Loaded the other way round, the system runtime comes first
    # and library calls on torch's allocations have failed with "no
    # ROCm-capable device".
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return [s[0] for s in _SIGS]


def check(status: int, where: str) -> None:
    if status != MLB_OK:
        raise MlbError(status, where, load().mlb_last_error().decode())
