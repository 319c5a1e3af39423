"""Pins of the learned-initialiser oracle (oracle/encoder.py): the mel filterbank's triangles,
the frame power spectrum against a direct DFT, a pure tone's log-mel peak, each convolution
layer against a direct sum, the network's gradients against finite differences, Adam's first
steps in closed form, and the normalised-parameter map against the generator's own draws."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import encoder as E

F64 = torch.float64


def test_mel_filters_are_unit_triangles_summing_to_one():
    W = E.mel_filterbank()
    assert W.shape == (128, 513) and W.min() >= 0.0 and W.max() <= 1.0
    edges = E.mel_to_hz(np.linspace(E.hz_to_mel(0.0), E.hz_to_mel(E.FS / 2), 130))
    f = np.arange(513) * E.FS / 1024
    # between the first and the last filter peak, neighbouring triangles sum to one
    inside = (f >= edges[1]) & (f <= edges[128])
    assert np.max(np.abs(W[:, inside].sum(axis=0) - 1.0)) < 1e-12
    # each filter is zero outside its two neighbouring edges and peaks where its centre falls
    for b in (10, 60, 127):
        out = (f <= edges[b]) | (f >= edges[b + 2])
        assert not W[b, out].any()
        k = int(np.argmin(np.abs(f - edges[b + 1])))
        assert abs(W[b, k] - min((f[k] - edges[b]) / (edges[b + 1] - edges[b]),
                                 (edges[b + 2] - f[k]) / (edges[b + 2] - edges[b + 1]))) < 1e-12


def test_power_spectrum_matches_direct_dft():
    x = np.random.default_rng(1).normal(size=3000)
    P = E.power_spectrum(x)
    assert P.shape == ((3000 - 1024) // 256 + 1, 513)
    f, k = 2, 37
    n = np.arange(1024)
    w = 0.5 - 0.5 * np.cos(2 * np.pi * n / 1024)
    X = np.sum(w * x[f * 256:f * 256 + 1024] * np.exp(-2j * np.pi * k * n / 1024))
    assert abs(P[f, k] - abs(X) ** 2) < 1e-9 * abs(X) ** 2


def test_pure_tone_peaks_in_its_mel_band():
    T, f0 = 8192, 3000.0
    t = np.arange(T) / E.FS
    s = np.stack([np.sin(2 * np.pi * f0 * t)] * 2)
    feat = E.log_mel(s)
    edges = E.mel_to_hz(np.linspace(E.hz_to_mel(0.0), E.hz_to_mel(E.FS / 2), 130))
    b = int(np.argmax(feat[:, 3]))
    assert edges[b] < f0 < edges[b + 2]


def test_conv_layer_equals_direct_sum():
    rng = np.random.default_rng(2)
    x = torch.as_tensor(rng.normal(size=(2, 3, 11)))
    W = torch.as_tensor(rng.normal(size=(4, 3, 5)))
    b = torch.as_tensor(rng.normal(size=4))
    y = E.conv_layer(x, W, b).numpy()
    assert y.shape == (2, 4, 6)
    ref = np.zeros((2, 4, 6))
    for bb in range(2):
        for co in range(4):
            for t in range(6):
                acc = float(b[co])
                for ci in range(3):
                    for k in range(5):
                        src = 2 * t + k - 2
                        if 0 <= src < 11:
                            acc += float(W[co, ci, k]) * float(x[bb, ci, src])
                ref[bb, co, t] = max(acc, 0.0)
    assert np.max(np.abs(y - ref)) < 1e-12


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    x = torch.as_tensor(rng.normal(size=(3, E.C_IN, 9)))
    lab = torch.as_tensor(rng.uniform(size=(3, E.N_OUT)))
    ws = [w.clone().requires_grad_(True) for w in E.init_weights(4)]
    for i in range(1, 2 * E.N_LAYERS, 2):  # small positive biases keep most units active
        with torch.no_grad():
            ws[i].fill_(0.05)
    grads = torch.autograd.grad(E.loss(x, lab, ws), ws)
    for which, idx in ((0, (5, 100, 2)), (5, (7,)), (10, (3, 1, 4)), (12, (4, 17)), (13, (6,))):
        h = 1e-6
        base = [w.detach().clone() for w in ws]
        hi = [w.clone() for w in base]
        lo = [w.clone() for w in base]
        hi[which][idx] += h
        lo[which][idx] -= h
        fd = float(E.loss(x, lab, hi) - E.loss(x, lab, lo)) / (2 * h)
        assert abs(fd - float(grads[which][idx])) < 1e-6 * max(1.0, abs(fd)), (which, idx)


def test_adam_first_steps_closed_form():
    p = [torch.tensor([1.0, -2.0], dtype=F64)]
    g = [torch.tensor([0.5, -0.25], dtype=F64)]
    st = {}
    E.adam(p, g, st, lr=0.1)
    # step 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps)
    exp1 = torch.tensor([1.0, -2.0]) - 0.1 * g[0] / (g[0].abs() + 1e-8)
    assert torch.max(torch.abs(p[0] - exp1)) < 1e-15
    E.adam(p, g, st, lr=0.1)  # a constant gradient keeps m_hat = g, v_hat = g^2
    assert torch.max(torch.abs(p[0] - (exp1 - 0.1 * g[0] / (g[0].abs() + 1e-8)))) < 1e-15


def test_parameter_map_matches_the_generator():
    ws, labels = synth.labelled_tiny_consoles(5, 3, T=2048)
    for i, w in enumerate(ws):
        for trk in range(4):
            mine = E.to_params(labels[i, trk])
            assert np.max(np.abs(mine["gain_pan"] - w.params[synth.GAIN_PAN][trk])) < 1e-6
            assert np.max(np.abs(mine["eq"] - w.params[synth.EQ][trk])) < 1e-6
            assert np.max(np.abs(mine["compressor"] - w.params[synth.COMP][trk])) < 1e-6 * 8
    # ranges: 0 and 1 hit the ends
    lo, hi = E.to_params(np.zeros(11)), E.to_params(np.ones(11))
    assert abs(lo["gain_pan"][0] - (-12.0) * math.log(10) / 20) < 1e-12
    assert abs(hi["compressor"][3] - 8.0) < 1e-12
    assert abs(lo["compressor"][0] - math.exp(-1.0 / (1e-3 * E.FS))) < 1e-12


@pytest.mark.parametrize("T", [32768, 2048])
def test_encoder_input_shape(T):
    s = synth.make_sources(synth.rng_for(1, 1), 2, T)
    x = E.encoder_input(s[0], s[1])
    assert x.shape == (256, E.n_frames(T))
    ws = E.init_weights(0)
    y = E.forward(torch.as_tensor(x)[None], ws)
    assert y.shape == (1, 11) and float(y.min()) > 0.0 and float(y.max()) < 1.0
