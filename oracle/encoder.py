"""Oracle of the learned parameter initialiser (the paper's gradient-descent mixing application,
Sec. 4 "Example usage", with a convolutional encoder predicting each track's processor
parameters as the starting point of the optimisation).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes none of this network; the readings (each listed in the design notes):
* features: the mono mix (l + r) / 2 of a signal, frames of 1024 samples at hop 256 while the
  frame fits inside [0, T), periodic Hann window, power spectrum |rFFT|^2 (bins 0..512), 128
  triangular mel filters on the HTK scale mel(f) = 2595 log10(1 + f / 700) with 130 edges evenly
  spaced in mel over [0, fs/2], filter b rising from edge b to edge b + 1 and falling to edge
  b + 2 (peak 1), feature ((ln(mel energy + 1e-6)) + 5) / 5;
* input: the dry track's 128 features stacked over the target mix's 128 features, [256, F];
* six convolution layers, kernel 5, stride 2, zero padding 2, bias, ReLU after each; 256 -> 64
  channels, then 64 -> 64; frames F -> ceil(F / 2) per layer;
* the mean over the remaining frames, one linear head 64 -> 11 and a sigmoid: normalised
  parameters in (0, 1);
* the 11 normalised parameters map affinely onto the generator's ranges: gain/pan dB per channel
  [-12, 6], six EQ band gains dB [-12, 12] (spread over the 1024 log-magnitudes by linear
  interpolation in log-frequency between band centres 20 * 1000^((b + 0.5) / 6) Hz, bin k at
  k fs / 2047 Hz, constant beyond the outer centres), compressor time constant [1, 100] ms
  (alpha = exp(-1 / (tau fs))), threshold dB [-30, -10], ratio [2, 8]; knee 3 dB;
* training loss: the mean squared error between the sigmoid outputs and the normalised
  parameters that drew the rendered example;
* Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Pins (tests): the mel filterbank's triangles (peaks, partition of unity between edges), the
power spectrum against a direct DFT, a pure tone's log-mel peak in the filter that holds its
frequency; each convolution against a direct sum; the whole network's gradients against
finite differences; Adam's first steps against their closed form; the parameter map against
the generator's own draws.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64
FS = 44100
N_FFT, HOP, N_MELS = 1024, 256, 128
N_BINS = N_FFT // 2 + 1
LOG_EPS = 1e-6
C_IN, C_HID, N_LAYERS, KSIZE, STRIDE, PAD = 2 * N_MELS, 64, 6, 5, 2, 2
N_OUT = 11
LN10_20, LN10_10 = math.log(10.0) / 20.0, math.log(10.0) / 10.0


def hz_to_mel(f):
    return 2595.0 * np.log10(1.0 + np.asarray(f, dtype=np.float64) / 700.0)


def mel_to_hz(m):
    return 700.0 * (10.0 ** (np.asarray(m, dtype=np.float64) / 2595.0) - 1.0)


def mel_filterbank() -> np.ndarray:
    """[128, 513] triangular filters (HTK mel scale, peak 1)."""
    edges = mel_to_hz(np.linspace(hz_to_mel(0.0), hz_to_mel(FS / 2.0), N_MELS + 2))
    f = np.arange(N_BINS) * FS / N_FFT
    W = np.zeros((N_MELS, N_BINS))
    for b in range(N_MELS):
        lo, mid, hi = edges[b], edges[b + 1], edges[b + 2]
        up = (f - lo) / (mid - lo)
        down = (hi - f) / (hi - mid)
        W[b] = np.maximum(0.0, np.minimum(up, down))
    return W


def n_frames(T: int) -> int:
    return (T - N_FFT) // HOP + 1 if T >= N_FFT else 0


def power_spectrum(x: np.ndarray) -> np.ndarray:
    """Mono signal [T] -> [F, 513] power spectra of the Hann-windowed frames."""
    F = n_frames(x.shape[-1])
    n = np.arange(N_FFT)
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * n / N_FFT)
    frames = np.stack([x[f * HOP:f * HOP + N_FFT] for f in range(F)]) * w
    X = np.fft.rfft(frames, axis=-1)
    return X.real ** 2 + X.imag ** 2


def log_mel(signal: np.ndarray) -> np.ndarray:
    """Stereo signal [2, T] -> features [128, F]."""
    m = 0.5 * (np.asarray(signal[0], dtype=np.float64) + np.asarray(signal[1], dtype=np.float64))
    E = power_spectrum(m) @ mel_filterbank().T  # [F, 128]
    return ((np.log(E + LOG_EPS) + 5.0) / 5.0).T


def encoder_input(dry: np.ndarray, mix: np.ndarray) -> np.ndarray:
    return np.concatenate([log_mel(dry), log_mel(mix)], axis=0)


def init_weights(seed: int = 0) -> list:
    """He-uniform convolution weights and zero biases, then the head (float64 tensors):
    [W1, b1, ..., W6, b6, Wh, bh]."""
    rng = np.random.default_rng(seed)
    ws = []
    c_in = C_IN
    for _ in range(N_LAYERS):
        bound = math.sqrt(6.0 / (c_in * KSIZE))
        ws.append(torch.as_tensor(rng.uniform(-bound, bound, (C_HID, c_in, KSIZE)), dtype=F64))
        ws.append(torch.zeros(C_HID, dtype=F64))
        c_in = C_HID
    bound = math.sqrt(6.0 / (C_HID + N_OUT))
    ws.append(torch.as_tensor(rng.uniform(-bound, bound, (N_OUT, C_HID)), dtype=F64))
    ws.append(torch.zeros(N_OUT, dtype=F64))
    return ws


def unflatten(flat) -> list:
    """One flat weight vector [W1, b1, ..., W6, b6, Wh, bh] -> the list of float64 tensors."""
    v = torch.as_tensor(np.asarray(flat), dtype=F64)
    out, o, c_in = [], 0, C_IN
    for _ in range(N_LAYERS):
        n = C_HID * c_in * KSIZE
        out += [v[o:o + n].reshape(C_HID, c_in, KSIZE).clone(), v[o + n:o + n + C_HID].clone()]
        o += n + C_HID
        c_in = C_HID
    out += [v[o:o + N_OUT * C_HID].reshape(N_OUT, C_HID).clone(),
            v[o + N_OUT * C_HID:o + N_OUT * C_HID + N_OUT].clone()]
    assert o + N_OUT * C_HID + N_OUT == v.numel()
    return out


def conv_layer(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """x [B, C_in, F] -> ReLU(conv1d(x, W, stride 2, zero padding 2) + b) [B, C_out, ceil(F/2)]."""
    return torch.relu(torch.nn.functional.conv1d(x, W, b, stride=STRIDE, padding=PAD))


def forward(x: torch.Tensor, ws: list) -> torch.Tensor:
    """x [B, 256, F] -> normalised parameters [B, 11] in (0, 1)."""
    h = x
    for layer in range(N_LAYERS):
        h = conv_layer(h, ws[2 * layer], ws[2 * layer + 1])
    pooled = h.mean(dim=-1)
    return torch.sigmoid(pooled @ ws[-2].T + ws[-1])


def loss(x: torch.Tensor, labels: torch.Tensor, ws: list) -> torch.Tensor:
    return ((forward(x, ws) - labels) ** 2).mean()


def adam(params: list, grads: list, state: dict, lr: float, b1=0.9, b2=0.999, eps=1e-8) -> None:
    """One Adam step in place (state holds t, m, v)."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    ms = state.setdefault("m", [torch.zeros_like(p) for p in params])
    vs = state.setdefault("v", [torch.zeros_like(p) for p in params])
    for p, g, m, v in zip(params, grads, ms, vs):
        m.mul_(b1).add_((1 - b1) * g)
        v.mul_(b2).add_((1 - b2) * g * g)
        p.sub_(lr * (m / (1 - b1 ** t)) / (torch.sqrt(v / (1 - b2 ** t)) + eps))


# --- normalised parameters -> a track's processor parameters ----------------------------------

RANGES = [(-12.0, 6.0), (-12.0, 6.0)] + [(-12.0, 12.0)] * 6 + [(1.0, 100.0), (-30.0, -10.0),
                                                             (2.0, 8.0)]
KNEE_DB = 3.0


def eq_log_mags(band_db: np.ndarray) -> np.ndarray:
    """Six band gains (dB) -> 1024 log-magnitudes (linear interpolation in log-frequency)."""
    centres = 20.0 * 1000.0 ** ((np.arange(6) + 0.5) / 6)
    f = np.arange(1024) * FS / 2047.0
    lf = np.log(np.maximum(f, 1e-3))
    return np.interp(lf, np.log(centres), band_db) * LN10_20


def to_params(s: np.ndarray) -> dict:
    """Normalised [11] -> {'gain_pan': [2], 'eq': [1024], 'compressor': [4]} (float64)."""
    v = [lo + (hi - lo) * float(x) for x, (lo, hi) in zip(s, RANGES)]
    return {"gain_pan": np.array(v[0:2]) * LN10_20,
            "eq": eq_log_mags(np.array(v[2:8])),
            "compressor": np.array([math.exp(-1.0 / (v[8] * 1e-3 * FS)), v[9] * LN10_10,
                                    KNEE_DB * LN10_10, v[10]])}
