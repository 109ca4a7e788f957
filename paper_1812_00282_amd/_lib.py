"""ctypes binding of libvate.so (the C ABI in include/vate.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Loading fails loudly if the library has not been built; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvate.so")

VATE_OK = 0
VATE_E_INVAL = 1
VATE_E_STATE = 2
VATE_E_DEVICE = 3
VATE_E_NOMEM = 4
VATE_E_UNSUPPORTED = 5


class VateParams(ctypes.Structure):
    _fields_ = [
        ("log2_pool", ctypes.c_uint32),
        ("width", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("g", ctypes.c_uint32),
        ("partition", ctypes.c_uint32),
        ("seed_a", ctypes.c_uint32),
        ("seed_b", ctypes.c_uint32),
        ("counter", ctypes.c_uint32),
        ("block_log2", ctypes.c_uint32),
    ]


class VateError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vate error {code}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int

_SIGS = {
    "vate_state_bytes": (_i32, [ctypes.POINTER(VateParams), ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "vate_create": (_i32, [ctypes.POINTER(VateParams), _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "vate_ingest": (_i32, [_vp, _vp, _sz, _vp]),
    "vate_close_slice": (_i32, [_vp, _vp]),
    "vate_estimate": (_i32, [_vp, _vp, _sz, _u32, _vp, _vp, _vp, _vp]),
    "vate_read_census": (_i32, [_vp, _vp, _vp]),
    "vate_estimate_workspace_bytes": (_i32, [_vp, _sz, ctypes.POINTER(_sz)]),
    "vate_estimate_ws": (_i32, [_vp, _vp, _sz, _u32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vate_estimate_noalloc": (_i32, [_vp, _vp, _sz, _u32, _vp, _vp, _vp, _vp]),
    "vate_estimate_plan": (_i32, [_vp, _vp, _sz, _vp, _sz, _vp]),
    "vate_estimate_run": (_i32, [_vp, _sz, _u32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vate_estimate_multi_workspace_bytes": (_i32, [_vp, _sz, ctypes.POINTER(_sz)]),
    "vate_estimate_multi_ws": (_i32, [_vp, _vp, _sz, _vp, _u32, _vp, _vp, _sz, _vp]),
    "vate_read_state": (_i32, [_vp, _vp, ctypes.POINTER(_u64), ctypes.POINTER(_u32),
                               ctypes.POINTER(_i32), _vp]),
    "vate_load_state": (_i32, [_vp, _vp, _u64, _u32, _i32, _vp]),
    "vate_last_error": (ctypes.c_char_p, [_vp]),
    "vate_status_string": (ctypes.c_char_p, [_i32]),
    "vate_destroy": (None, [_vp]),
    "vate_host_hash": (_u32, [ctypes.POINTER(VateParams), _u32, _u32, _u32]),
    "vate_host_block": (_u32, [ctypes.POINTER(VateParams), _u64]),
    # learned estimator (include/vate_mlp.h)
    "vate_mlp_pack": (_i32, [_vp, _vp, _vp]),
    "vate_mlp_forward": (_i32, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "vate_mlp_train_step": (_i32, [_vp, _vp, _vp, _vp, _sz, _vp, _vp, _vp]),
    "vate_mlp_adam": (_i32, [_vp, _vp, _vp, _vp, _u32, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, ctypes.c_float, _vp]),
    "vate_mlp_fill": (_i32, [_vp, _sz, ctypes.c_float, _vp]),
    "vate_mlp_features": (_i32, [_vp, _vp, _sz, _u32, _u32, ctypes.c_float, _vp, _vp, _vp]),
    "vate_estimate_learned": (_i32, [_vp, _vp, _sz, _vp, _vp, _vp, _vp]),
    "vate_estimate_learned_workspace_bytes": (_i32, [_vp, _sz, ctypes.POINTER(_sz)]),
    "vate_estimate_learned_ws": (_i32, [_vp, _vp, _sz, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vate_estimate_learned_run": (_i32, [_vp, _sz, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vate_mlp_mfma_selftest": (_i32, [_vp, _vp, _vp, _vp]),
}


class VateMlpEnvelope(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("g", ctypes.c_uint32), ("log2_pool", ctypes.c_uint32),
                ("width", ctypes.c_uint32), ("lo", ctypes.c_float * 64), ("hi", ctypes.c_float * 64)]


_SIGS.update({
    "vate_mlp_set_envelope": (_i32, [_vp, ctypes.POINTER(VateMlpEnvelope), _vp]),
    "vate_mlp_fallbacks": (_i32, [_vp, ctypes.POINTER(_u64), _i32, _vp]),
})


class VateBatchTune(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in
                ("ingest_tile", "census_tile", "estimate_block", "grid_preserve",
                 "grid_ingest", "grid_census", "grid_estimate", "estimate_lanes", "census_unroll")]


_SIGS.update({
    # batched sketches (include/vate_batch.h)
    "vate_batch_bytes": (_i32, [_u32, ctypes.POINTER(_sz)]),
    "vate_batch_create": (_i32, [_vp, _u32, _vp, _vp, ctypes.POINTER(_vp)]),
    "vate_batch_set_io": (_i32, [_vp, _u32, _vp, _u64, _vp, _u32, _u32, _vp, _vp]),
    "vate_batch_slice": (_i32, [_vp, _vp]),
    "vate_batch_capture": (_i32, [_vp, _vp]),
    "vate_batch_replay": (_i32, [_vp, _vp]),
    "vate_batch_get_tune": (_i32, [_vp, ctypes.POINTER(VateBatchTune)]),
    "vate_batch_set_tune": (_i32, [_vp, ctypes.POINTER(VateBatchTune)]),
    "vate_batch_autotune": (_i32, [_vp, _vp, ctypes.c_char_p, _sz]),
    "vate_batch_last_error": (ctypes.c_char_p, [_vp]),
    "vate_batch_destroy": (None, [_vp]),
})

MLP_FEATURES = 64
MLP_HIDDEN = 64
MLP_PARAMS = 8385
MLP_WEIGHT_BYTES = 26368
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


def lib() -> ctypes.CDLL:
    """Load libvate.so (import torch first so one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGS)


def check(rc: int, handle=None) -> None:
    if rc != VATE_OK:
        msg = ""
        if handle:
            msg = (lib().vate_last_error(handle) or b"").decode()
        if not msg:
            msg = lib().vate_status_string(rc).decode()
        raise VateError(rc, msg)
