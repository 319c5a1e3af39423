"""ctypes view of libgrafx.so (the C ABI declared in include/grafx.h). Argument marshalling only.

The library is loaded from this package's directory; if it is missing the import fails loudly
(build it with `python -m paper_2408_03204_amd.build`). There is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrafx.so")

NUM_TYPES = 13
STATUS = {0: "GRAFX_OK", 1: "GRAFX_E_ARG", 2: "GRAFX_E_GRAPH", 3: "GRAFX_E_CYCLE",
          4: "GRAFX_E_TYPE", 5: "GRAFX_E_SHAPE", 6: "GRAFX_E_LIMIT", 7: "GRAFX_E_WORKSPACE",
          8: "GRAFX_E_HIP"}

# Symbols declared in include/grafx.h (checked by the CPU test suite).
EXPORTS = ("grafx_schedule", "grafx_schedule_with_lengths", "grafx_schedule_free",
           "grafx_schedule_query", "grafx_schedule_export", "grafx_plan_upload",
           "grafx_workspace_bytes", "grafx_render", "grafx_render_backward", "grafx_render_step",
           "grafx_render_backward_step", "grafx_mrstft_workspace_bytes", "grafx_mrstft_loss",
           "grafx_mrstft_backward", "grafx_logmel", "grafx_encoder_gather",
           "grafx_encoder_sizes", "grafx_encoder_forward", "grafx_encoder_backward", "grafx_adam",
           "grafx_encoder_params", "grafx_schedule_set_tuning", "grafx_schedule_get_tuning",
           "grafx_set_schedule_threads", "grafx_workspace_error", "grafx_last_error",
           "grafx_render_noalloc", "grafx_schedule_set_reverb_noise",
           "grafx_schedule_set_delay_surrogate", "grafx_delay_phasor_regularise")


class GrafxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class ScheduleSizes(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int32), ("num_edges", ctypes.c_int32),
                ("num_steps", ctypes.c_int32), ("num_inputs", ctypes.c_int32),
                ("num_outputs", ctypes.c_int32), ("type_count", ctypes.c_int32 * NUM_TYPES),
                ("plan_bytes", ctypes.c_int64), ("max_len", ctypes.c_int64)]


_lib = None

c_i32p = ctypes.POINTER(ctypes.c_int32)
vp = ctypes.c_void_p
i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
ptr_array = ctypes.c_void_p * NUM_TYPES


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python -m paper_2408_03204_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "grafx_schedule": (i32, [i32, c_i32p, i32, c_i32p, c_i32p, c_i32p, i32, i32, i64,
                                 ctypes.POINTER(vp)]),
        "grafx_schedule_with_lengths": (i32, [i32, c_i32p, i32, c_i32p, c_i32p, c_i32p, c_i32p,
                                              i32, i32, i64, ctypes.POINTER(vp)]),
        "grafx_schedule_free": (None, [vp]),
        "grafx_set_schedule_threads": (i32, [i32]),
        "grafx_schedule_query": (i32, [vp, ctypes.POINTER(ScheduleSizes)]),
        "grafx_schedule_export": (i32, [vp] + [c_i32p] * 8),
        "grafx_plan_upload": (i32, [vp, vp, sz, vp]),
        "grafx_workspace_bytes": (i32, [vp, i64, i32, ctypes.POINTER(sz)]),
        "grafx_render": (i32, [vp, vp, i64, vp, ptr_array, vp, vp, sz, vp]),
        "grafx_render_noalloc": (i32, [vp, vp, i64, vp, ptr_array, vp, vp]),
        "grafx_render_backward": (i32, [vp, vp, i64, vp, ptr_array, vp, vp, vp, vp, ptr_array,
                                        vp, sz, vp]),
        "grafx_render_step": (i32, [vp, vp, i64, vp, ptr_array, vp, vp, sz, i32, vp]),
        "grafx_render_backward_step": (i32, [vp, vp, i64, vp, ptr_array, vp, vp, vp, vp, sz,
                                             i32, vp]),
        "grafx_mrstft_workspace_bytes": (i32, [i32, i64, ctypes.POINTER(sz)]),
        "grafx_mrstft_loss": (i32, [i32, i64, vp, vp, vp, vp, sz, vp]),
        "grafx_mrstft_backward": (i32, [i32, i64, vp, vp, vp, vp, vp, sz, vp]),
        "grafx_logmel": (i32, [i32, i64, vp, vp, vp]),
        "grafx_encoder_gather": (i32, [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "grafx_encoder_sizes": (i32, [i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz),
                                      ctypes.POINTER(sz)]),
        "grafx_encoder_forward": (i32, [i32, i32, vp, vp, i32, vp, vp, vp]),
        "grafx_encoder_backward": (i32, [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "grafx_adam": (i32, [i64, vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, ctypes.c_float, vp]),
        "grafx_encoder_params": (i32, [i32, vp, vp, vp, vp, vp]),
        "grafx_schedule_set_tuning": (i32, [vp, i32, i32]),
        "grafx_schedule_get_tuning": (i32, [vp, i32, c_i32p]),
        "grafx_schedule_set_reverb_noise": (i32, [vp, vp, i64]),
        "grafx_schedule_set_delay_surrogate": (i32, [vp, i32]),
        "grafx_delay_phasor_regularise": (i32, [i32, i32, vp, vp, ctypes.c_float, vp]),
        "grafx_workspace_error": (i32, [vp, i64, vp, sz, vp, vp]),
        "grafx_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != 0:
        raise GrafxError(code, load().grafx_last_error().decode())
