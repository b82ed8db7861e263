"""ctypes declarations of include/dtb.h.  Loading fails loudly when the
compiled library is absent: there is no CPU fallback for any entry point."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdtb.so")

DTB_OK = 0
STATUS = {0: "DTB_OK", -1: "DTB_ERR_INVALID", -2: "DTB_ERR_OOM", -3: "DTB_ERR_HIP", -4: "DTB_ERR_STATE",
          -5: "DTB_ERR_NUMERIC", -6: "DTB_ERR_UNSUPPORTED"}
W_F32, W_BF16 = 0, 1
FIELDS = {"V": 0, "j_AMPA": 1, "j_NMDA": 2, "j_GABAa": 3, "j_GABAb": 4, "ref": 5, "I_ou": 6}


class DtbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Ptype(ctypes.Structure):
    _fields_ = [("C", ctypes.c_float), ("gL", ctypes.c_float), ("EL", ctypes.c_float),
                ("Vth", ctypes.c_float), ("Vreset", ctypes.c_float), ("tref_ms", ctypes.c_float),
                ("Iext", ctypes.c_float), ("g", ctypes.c_float * 4)]


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_regions", ctypes.c_int32), ("max_delay", ctypes.c_int32),
                ("n_ptypes", ctypes.c_int32), ("member", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("delay", ctypes.c_void_p), ("is_inh", ctypes.c_void_p), ("region", ctypes.c_void_p),
                ("ptype", ctypes.c_void_p), ("ptypes", ctypes.c_void_p), ("V0", ctypes.c_void_p),
                ("E", ctypes.c_float * 4), ("tau_ms", ctypes.c_float * 4), ("dt_ms", ctypes.c_float),
                ("bg_w", ctypes.c_float), ("bg_lambda", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("wtype", ctypes.c_int32), ("record_steps", ctypes.c_int32),
                ("gather_bundle_syn", ctypes.c_int32),
                ("gather_unroll", ctypes.c_int32),
                ("gather_fuse", ctypes.c_int32),
                ("gather_events", ctypes.c_int32)]


TUNE_MAX_BUNDLES = 8


class TuneResult(ctypes.Structure):
    _fields_ = [("bundle_syn", ctypes.c_int32), ("unroll", ctypes.c_int32), ("fuse", ctypes.c_int32),
                ("events", ctypes.c_int32), ("ms_per_step", ctypes.c_float),
                ("from_cache", ctypes.c_int32), ("n_tried", ctypes.c_int32),
                ("tried_bundle", ctypes.c_int32 * (8 * TUNE_MAX_BUNDLES)),
                ("tried_unroll", ctypes.c_int32 * (8 * TUNE_MAX_BUNDLES)),
                ("tried_fuse", ctypes.c_int32 * (8 * TUNE_MAX_BUNDLES)),
                ("tried_events", ctypes.c_int32 * (8 * TUNE_MAX_BUNDLES)),
                ("tried_ms", ctypes.c_float * (8 * TUNE_MAX_BUNDLES))]


# every symbol include/dtb.h declares, with its ctypes signature
_P = ctypes.c_void_p
_I32, _I64 = ctypes.c_int32, ctypes.c_int64
SIGNATURES = {
    "dtb_abi_version": ([], ctypes.c_int),
    "dtb_last_error": ([], ctypes.c_char_p),
    "dtb_bitmap_words": ([_I64], _I64),
    "dtb_create": ([ctypes.POINTER(Desc), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "dtb_step": ([_P, _I32], ctypes.c_int),
    "dtb_autotune": ([_P, _I32, _P, ctypes.c_char_p, _P, _I32, _I32, _I32, ctypes.POINTER(TuneResult)],
                     ctypes.c_int),
    "dtb_reset": ([_P], ctypes.c_int),
    "dtb_set_background": ([_P, ctypes.c_double, ctypes.c_float], ctypes.c_int),
    "dtb_set_background_ou": ([_P, ctypes.c_float, ctypes.c_float, ctypes.c_float], ctypes.c_int),
    "dtb_force_spikes": ([_P, _P, _I32], ctypes.c_int),
    "dtb_set_remote_block": ([_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P, _P, _P], ctypes.c_int),
    "dtb_push_remote_spikes": ([_P, _P, _I32], ctypes.c_int),
    "dtb_save": ([_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "dtb_load": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
    "dtb_partition": ([ctypes.c_int64, _P, _P, _P, _P, _P, _P, _I32, ctypes.c_double, ctypes.c_double, _P, _I32,
                       _P, _P, _P], ctypes.c_int),
    "dtb_enkf_analysis": ([_I32, _I32, _I32, _P, _P, _P, _P, ctypes.c_float, ctypes.c_uint64, ctypes.c_int64,
                           ctypes.c_float, ctypes.c_float, _P], ctypes.c_int),
    "dtb_read_spikes": ([_P, _I64, _I64, _P, ctypes.c_int], ctypes.c_int),
    "dtb_read_spike_ids": ([_P, _I64, _P, _I64, ctypes.POINTER(_I64)], ctypes.c_int),
    "dtb_read_state": ([_P, _I32, _P, ctypes.c_int], ctypes.c_int),
    "dtb_read_region_counts": ([_P, _I64, _I64, _P], ctypes.c_int),
    "dtb_read_region_rates": ([_P, _I64, _I64, _P], ctypes.c_int),
    "dtb_read_step_events": ([_P, _I64, _I64, _P, _P], ctypes.c_int),
    "dtb_read_counters": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "dtb_set_timing": ([_P, ctypes.c_int], ctypes.c_int),
    "dtb_read_timing": ([_P, _P, _P], ctypes.c_int),
    "dtb_create_batch": ([ctypes.POINTER(Desc), _I32, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "dtb_batch_info": ([_P, _P, _P, _P, _I32], ctypes.c_int),
    "dtb_set_gains": ([_P, _P, ctypes.c_int], ctypes.c_int),
    "dtb_run": ([_P, _I32], ctypes.c_int),
    "dtb_read_bold": ([_P, _P, _P, ctypes.c_int], ctypes.c_int),
    "dtb_mlp_create": ([_I32, _I32, _I32, _I32, ctypes.c_uint64, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "dtb_mlp_num_params": ([_P], _I64),
    "dtb_mlp_params": ([_P, _P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "dtb_mlp_set_operands": ([_P, ctypes.c_int], ctypes.c_int),
    "dtb_mlp_forward": ([_P, _P, _I32, _P, ctypes.c_int], ctypes.c_int),
    "dtb_mlp_grad": ([_P, _P, _P, _I32, _P, _P, ctypes.c_int], ctypes.c_int),
    "dtb_mlp_train_step": ([_P, _P, _P, _I32, ctypes.c_float, _P, ctypes.c_int], ctypes.c_int),
    "dtb_mlp_destroy": ([_P], None),
    "dtb_topk": ([_P, _I32, _I32, _P, _P, ctypes.c_int], ctypes.c_int),
    "dtb_topk_noalloc": ([_P, _I32, _I32, _P, _P], ctypes.c_int),
    "dtb_sync": ([_P], ctypes.c_int),
    "dtb_destroy": ([_P], None),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libdtb.so.  torch (if installed) is imported first so that the
    process holds one HIP runtime, the one torch's streams belong to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                          f"g.build()'` (there is no CPU fallback)")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if lib.dtb_abi_version() != 14:
        raise ImportError("libdtb.so ABI version mismatch")
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != DTB_OK:
        raise DtbError(status, load().dtb_last_error().decode(errors="replace"))
