"""CPU checks of the learned initialiser's C ABI: sizes of the weight, activation and scratch
buffers against the network's shape, and the argument errors every entry point reports before it
enqueues anything (no call here reaches a GPU)."""
import ctypes

import pytest

import synth
from paper_2408_03204_amd import encoder as enc
from paper_2408_03204_amd._lib import STATUS, load


def _status(code):
    return STATUS[code]


def test_sizes_match_the_network():
    n_w, n_act, n_grad = enc.sizes(256, 125)
    assert n_w == synth.encoder_weights(0).size == 64 * 256 * 5 + 64 + 5 * (64 * 64 * 5 + 64) \
        + 11 * 64 + 11
    frames, total = 125, 0
    for _ in range(6):
        frames = (frames + 1) // 2
        total += 256 * 64 * frames
    assert n_act == total + 256 * 64          # six layer outputs and the pooled features
    assert n_grad == total + 256 * 64 + 256 * 11 + 256


@pytest.mark.parametrize("batch,frames", [(0, 10), (4, 0), (-1, 5), (1 << 21, 3)])
def test_sizes_reject_bad_shapes(batch, frames):
    a = ctypes.c_size_t()
    assert _status(load().grafx_encoder_sizes(batch, frames, ctypes.byref(a), None, None)) == \
        "GRAFX_E_SHAPE"


def test_entry_points_reject_null_and_bad_arguments():
    lib = load()
    p = ctypes.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert _status(lib.grafx_logmel(1, 1000, p, p, None)) == "GRAFX_E_SHAPE"  # T < 1024
    assert _status(lib.grafx_logmel(0, 4096, p, p, None)) == "GRAFX_E_SHAPE"
    assert _status(lib.grafx_logmel(1, 4096, None, p, None)) == "GRAFX_E_ARG"
    assert _status(lib.grafx_encoder_forward(2, 9, None, p, 0, p, p, None)) == "GRAFX_E_ARG"
    assert _status(lib.grafx_encoder_forward(0, 9, p, p, 0, p, p, None)) == "GRAFX_E_SHAPE"
    assert _status(lib.grafx_encoder_forward(1 << 20, 600, p, p, 1, p, p, None)) == \
        "GRAFX_E_SHAPE"  # bf16 path: batch x 256 x frames beyond its 2^29 limit
    assert _status(lib.grafx_encoder_backward(2, 9, p, p, p, p, None, p, p, p, None)) == \
        "GRAFX_E_ARG"
    assert _status(lib.grafx_encoder_gather(2, 9, p, p, p, p, p, None, p, None)) == \
        "GRAFX_E_ARG"  # a label table without a labels buffer
    assert _status(lib.grafx_adam(10, p, p, p, p, None, 0, 0.1, 0.9, 0.999, 1e-8, None)) == \
        "GRAFX_E_ARG"  # steps count from 1
    assert _status(lib.grafx_adam(10, None, p, p, p, None, 1, 0.1, 0.9, 0.999, 1e-8, None)) == \
        "GRAFX_E_ARG"
    assert _status(lib.grafx_adam(0, None, None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8,
                                  None)) == "GRAFX_OK"  # nothing to do
    assert _status(lib.grafx_encoder_params(0, p, p, p, p, None)) == "GRAFX_E_SHAPE"
    assert b"batch" in lib.grafx_last_error()  # the failing call's message is kept


def test_binding_requires_contiguous_device_tensors():
    import torch
    with pytest.raises(ValueError):
        enc.logmel(torch.zeros((1, 2, 4096)))  # a host tensor
