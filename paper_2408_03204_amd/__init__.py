"""MI355X-native batched render and adjoint of audio processing graphs (GRAFX, arXiv
2408.03204): host C++ scheduling, hand-written HIP kernels for gfx950, behind a C ABI
(include/grafx.h) with this thin Python binding."""
from .api import (METHODS, N_PARAMS, TYPE_CODES, GradStep, RenderBuffers,  # noqa: F401
                  Schedule, delay_phasor_regularise, merge_graphs, merge_inputs, mrstft_loss, render, render_noalloc,
                  schedule_many,
                  set_schedule_threads)
from ._lib import EXPORTS, LIB_PATH, GrafxError, load  # noqa: F401
