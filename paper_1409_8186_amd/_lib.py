"""ctypes declarations of the C ABI in include/mudiff.h (libmudiff.so, built in-tree).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmudiff.so")

# name -> (restype, argtypes), one entry per function of include/mudiff.h
_vp = ctypes.c_void_p
_i32 = ctypes.c_int
_i64p = ctypes.POINTER(ctypes.c_int64)
_sz = ctypes.c_size_t
_d = ctypes.c_double

SIGNATURES = {
    "mudiff_tables_workspace_size": (_sz, [_i32, _vp, _vp, _i32]),
    "mudiff_tables": (_i32, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i32, _vp, ctypes.POINTER(_vp)]),
    "mudiff_circulant_info": (_i32, [_vp, _i64p, _i64p, ctypes.POINTER(_i32)]),
    "mudiff_set_circulant": (_i32, [_vp, _i32, _i32]),
    "mudiff_circulant_tile": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mudiff_set_circulant_tile": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32]),
    "mudiff_destroy": (_i32, [_vp]),
    "mudiff_sizes": (_i32, [_vp, _i64p]),
    "mudiff_disk_tables": (_i32, [_vp, _vp, _vp, _vp]),
    "mudiff_pair_tables": (_i32, [_vp, _vp, _i64p, _vp]),
    "mudiff_apply_config": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mudiff_set_apply_config": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32]),
    "mudiff_matvec_workspace_size": (_sz, [_vp, _i32]),
    "mudiff_matvec": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp, _sz, _vp]),
    "mudiff_matvec_noalloc": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp]),
    "mudiff_rhs": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp]),
    "mudiff_rhs_point": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp]),
    "mudiff_gmres_workspace_size": (_sz, [_vp, _i32, _i32, _i32]),
    "mudiff_gmres": (_i32, [_vp, _i32, _vp, _vp, _vp, _i32, _d, _i32, _i32, _vp, _sz,
                            _vp, _vp, _vp, _vp, _vp]),
    "mudiff_farfield": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _vp]),
    "mudiff_nearfield": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _i32, _vp, _vp]),
    "mudiff_grad_workspace_size": (_sz, [_vp, _i32, _i32, _i32, _i32]),
    "mudiff_grad": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _i32, _d, _i32, _i32, _vp, _sz,
                           _vp, _vp, _vp, _vp, _vp]),
    "mudiff_operator_workspace_size": (_sz, [_vp]),
    "mudiff_set_operator": (_i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mudiff_set_formulation": (_i32, [_vp, _i32, _d, _d, _d, _vp, _sz, _vp]),
    "mudiff_set_penetrable": (_i32, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "mudiff_interior_workspace_size": (_sz, [_vp, _i32]),
    "mudiff_interior_field": (_i32, [_vp, _i32, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "mudiff_tro": (_i32, [_i32, _i32, _vp, _vp, _vp]),
    "mudiff_tro_eigh_workspace_size": (_sz, [_i32, _i32]),
    "mudiff_tro_eigh": (_i32, [_i32, _i32, _vp, _vp, _vp, _i32, _d, _vp, _sz,
                               ctypes.POINTER(ctypes.c_int32), _vp]),
    "mudiff_herglotz": (_i32, [_i32, _vp, _i32, _vp, _d, _d, _i32, _vp, _vp, _vp]),
    "mudiff_probe_workspace_size": (_sz, [_i32, _sz]),
    "mudiff_probe": (_i32, [_i32, _sz, _vp, _sz, ctypes.POINTER(_d), _vp]),
    "mudiff_profile_begin": (_i32, [_vp, _i32]),
    "mudiff_profile_end": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_d)]),
    "mudiff_last_error": (ctypes.c_char_p, []),
}

STATUS = {0: "OK", 1: "INVALID", 2: "OVERLAP", 3: "NOMEM", 4: "DEVICE", 5: "NOT_CONVERGED"}
OP_L, OP_A, OP_LT = 0, 1, 2
X0, GRAPH, POINT_SOURCE, NO_PRECOND, BLOCK, SSTEP = 1, 2, 4, 8, 16, 32


def block_size(s: int) -> int:
    """Flag bits of the block size of a MUDIFF_BLOCK solve (MUDIFF_BLOCK_SIZE)."""
    return (s & 0xFF) << 8


def sstep_size(s: int) -> int:
    """Flag bits of the Newton vectors per block of a MUDIFF_SSTEP solve (MUDIFF_SSTEP_SIZE)."""
    return (s & 0xFF) << 16
TABLES_CIRCULANT = 1
N_PHASES = 5
PHASES = ("scale", "forward_transform", "frequency_products", "mfma_or_lane", "output_pass")
PROBE_FP64_FMA, PROBE_FP64_MFMA, PROBE_COPY = 0, 1, 2


class MudiffError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mudiff {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Loads libmudiff.so and declares every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1409_8186_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        msg = load().mudiff_last_error()
        raise MudiffError(status, msg.decode() if msg else "")
