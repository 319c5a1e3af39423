"""Oracle multi-resolution STFT loss (the loss driving gradient descent in paper Sec. 4,
"Example usage": the rendered output is compared with a target mix).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper only says the output can be used to compute a loss; this is the standard
multi-resolution STFT loss (spectral convergence plus log-magnitude L1), written from its
definition. Reading:
* resolutions r in {512, 1024, 2048}, hop r/4, periodic Hann window of length r, frames at
  0, hop, 2 hop, ... while the frame fits inside [0, T) (no padding); a resolution with no
  frame contributes 0;
* S = sqrt(|rFFT|^2 + 1e-8) over bins 0..r/2, for every output node and channel;
* SC_r = ||S_y - S_t||_F / ||S_t||_F and LM_r = mean |ln S_y - ln S_t|, both over all
  (node, channel, frame, bin) entries;
* L = (SC_512 + LM_512 + SC_1024 + LM_1024 + SC_2048 + LM_2048) / 3.

Parity pins (tests): L(y, y) = 0; each frame's spectrum equals a direct DFT sum; spectral
convergence is invariant to scaling both signals' excess (closed form for y = c * target at
high level); finite-difference gradients away from equality.
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64
RESOLUTIONS = (512, 1024, 2048)
MAG_EPS = 1e-8


def n_frames(T: int, r: int) -> int:
    return (T - r) // (r // 4) + 1 if T >= r else 0


def stft_mag(x: torch.Tensor, r: int) -> torch.Tensor:
    """x [..., T] -> |STFT| [..., F, r/2+1] with the periodic Hann window."""
    hop = r // 4
    frames = x.unfold(-1, r, hop)
    n = torch.arange(r, dtype=F64)
    w = 0.5 - 0.5 * torch.cos(2.0 * math.pi * n / r)
    X = torch.fft.rfft(frames * w, dim=-1)
    return torch.sqrt(X.real ** 2 + X.imag ** 2 + MAG_EPS)


def mrstft(y: torch.Tensor, target: torch.Tensor, resolutions=RESOLUTIONS) -> torch.Tensor:
    total = torch.zeros((), dtype=F64)
    T = y.shape[-1]
    for r in resolutions:
        if n_frames(T, r) == 0:
            continue
        Sy, St = stft_mag(y, r), stft_mag(target, r)
        sc = torch.linalg.vector_norm(Sy - St) / torch.linalg.vector_norm(St)
        lm = torch.mean(torch.abs(torch.log(Sy) - torch.log(St)))
        total = total + sc + lm
    return total / len(resolutions)
