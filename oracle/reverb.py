"""Oracle of the filtered-noise mid/side reverb (paper Sec. 3 "Reverb", Eqs. 6-7) and of the
multitap delay's delay-time surrogate (Sec. 3 "Multitap delay", Eq. 15), in torch float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reverb. Two fixed noise signals u_m (mid) and u_s (side) of L samples (2 s at 44.1 kHz in the
paper) are analysed by an STFT, masked, and brought back to the time domain; the mid/side pair
is turned into a stereo FIR, and each channel of the input is convolved with its FIR:
* STFT: FFT size 384, hop 192, periodic Hann analysis window w[q] = 1/2 - 1/2 cos(2 pi q / 384);
  frame m covers samples [192 m - 192, 192 m + 192) (zero outside [0, L)), m = 0..M-1 with
  M = ceil(L / 192) + 1, so that every sample lies in two frames.
* Mask (Eq. 7): M_x[k, m] = exp(H0_x[k] + m HD_x[k]) for the one-sided bins k = 0..191; the
  paper's frame index starts at 1 and multiplies (m - 1), ours starts at 0. The Nyquist bin 192
  takes the mask of bin 191.
* Inverse: each masked frame goes through a real inverse DFT of size 384 and the frames are
  overlap-added at their positions, with no synthesis window: the periodic Hann window at half
  overlap sums to 1, so an all-ones mask gives back the noise itself. The sum is cropped to
  [0, L).
* Mid/side to stereo as for the imager (Sec. 3 "Stereo imager"): h_l = (h_m + h_s) / 2,
  h_r = (h_m - h_s) / 2.
* Output: causal, channel-wise convolution y_c[t] = sum_{n=0}^{L-1} h_c[n] u_c[t - n], t < T
  (input zero before 0).
Parameters p (768): [x in (mid, side)][f in (H0, HD)][192 log-magnitudes], i.e. index
x * 384 + f * 192 + k.

Delay surrogate. Within each 100 ms slot (N = 4410 samples) the delay d is the integer the
forward pass reads from the phase of the slot's phasor z (z = exp(-2 pi i d / N) on the unit
circle). The surrogate of the unit impulse delta[n - d] is the inverse DFT of the damped
sinusoid z^k: s[n] = Re (1/N) sum_{k=0}^{N-1} z^k exp(2 pi i k n / N), n = 0..N-1, which is
exactly delta[n - d] when z = exp(-2 pi i d / N). Straight-through estimation: the forward pass
keeps the exact integer delay; the gradient with respect to (Re z, Im z) is the one the render
would have if slot m's impulse were s shifted by the slot's start, i.e. with
G[n] = dL/ds[n] = sum_t ybar[t] (c * u)[t - 4410 m - n] and s'(z)[n] = ds/dz (complex):
dL/dRe z = sum_n G[n] Re s'[n],  dL/dIm z = -sum_n G[n] Im s'[n].
The paper also normalises each delay gradient and pulls z towards the unit circle with a
regulariser; it gives neither the normalisation nor the regulariser's weight. The two helpers
below take a unit-norm gradient per phasor and a squared distance to the circle times a caller's
weight: "parity unpinned" for both (their constants are not in the paper).

Parity pins (tests/test_oracle_reverb.py): an all-ones mask returns the noise; a mask that depends
on the frame only has the closed form noise[n] sum_m e^(m d) w[n - 192 m + 192]; Parseval per
frame for a frequency-dependent mask; the mid/side closed form; the convolution against a direct
sum; autograd against finite differences; the surrogate equals delta[n - d] on the unit circle,
matches the geometric-series closed form (1 - z^N) / (N (1 - z e^(2 pi i n / N))) inside the
disk, its derivative matches finite differences, and the straight-through gradient equals the
autograd gradient of a delay whose forward uses the surrogate, at phasors on the unit circle.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64
C128 = torch.complex128

FFT = 384
HOP = 192
BINS = 192          # parameterised one-sided bins 0..191 (bin 192 copies bin 191)
N_PARAMS = 768


def n_frames(L: int) -> int:
    """Frames of the centred STFT that give every sample of [0, L) two frames."""
    return -(-L // HOP) + 1


def hann_periodic() -> torch.Tensor:
    q = torch.arange(FFT, dtype=F64)
    return 0.5 - 0.5 * torch.cos(2.0 * math.pi * q / FFT)


def stft(x: torch.Tensor) -> torch.Tensor:
    """One-sided STFT [FFT/2 + 1, M] of a real signal x [L] (frames centred, zero padded)."""
    L = x.shape[-1]
    M = n_frames(L)
    padded = torch.cat([torch.zeros(HOP, dtype=F64), x.to(F64),
                        torch.zeros((M - 1) * HOP + FFT - HOP - L, dtype=F64)])
    idx = (torch.arange(M) * HOP)[:, None] + torch.arange(FFT)[None, :]
    frames = padded[idx] * hann_periodic()[None, :]
    return torch.fft.rfft(frames, n=FFT, dim=-1).T  # [193, M]


def istft(X: torch.Tensor, L: int) -> torch.Tensor:
    """Inverse of `stft` without a synthesis window: real inverse DFT of each frame,
    overlap-added at its position, cropped to [0, L)."""
    M = X.shape[-1]
    frames = torch.fft.irfft(X.T, n=FFT, dim=-1)  # [M, 384]
    total = (M - 1) * HOP + FFT
    idx = ((torch.arange(M) * HOP)[:, None] + torch.arange(FFT)[None, :]).reshape(-1)
    out = torch.zeros(total, dtype=F64).index_add(0, idx, frames.reshape(-1))
    return out[HOP:HOP + L]


def mask(H0: torch.Tensor, HD: torch.Tensor, M: int) -> torch.Tensor:
    """Eq. 7 on the one-sided bins: exp(H0[k] + m HD[k]), m = 0..M-1, Nyquist bin = bin 191."""
    H0 = torch.cat([H0, H0[-1:]])
    HD = torch.cat([HD, HD[-1:]])
    m = torch.arange(M, dtype=F64)
    return torch.exp(H0[:, None] + m[None, :] * HD[:, None])


def reverb_ir(p: torch.Tensor, noise: torch.Tensor) -> torch.Tensor:
    """Stereo FIR [2, L] of one reverb node from its parameter row p [768] and the noise
    [2, L] (mid, side)."""
    q = p.reshape(2, 2, BINS)
    L = noise.shape[-1]
    M = n_frames(L)
    h = []
    for x in range(2):  # mid, side
        U = stft(torch.as_tensor(noise[x], dtype=F64))
        h.append(istft(U * mask(q[x, 0], q[x, 1], M), L))
    hm, hs = h
    return torch.stack([(hm + hs) / 2, (hm - hs) / 2])


def causal_conv(u: torch.Tensor, h: torch.Tensor) -> torch.Tensor:
    """y_c[t] = sum_n h_c[n] u_c[t - n] for t < T, per channel (float64 FFT convolution)."""
    T, L = u.shape[-1], h.shape[-1]
    n = 1
    while n < T + L:
        n *= 2
    y = torch.fft.irfft(torch.fft.rfft(u, n=n) * torch.fft.rfft(h, n=n), n=n)
    return y[..., :T]


def reverb(u: torch.Tensor, p: torch.Tensor, noise) -> torch.Tensor:
    """The reverb processor: input [2, T], parameter row [768], noise [2, L] (numpy or tensor)."""
    noise = torch.as_tensor(np.asarray(noise) if not torch.is_tensor(noise) else noise,
                            dtype=F64)
    return causal_conv(u, reverb_ir(p, noise))


# ---------------------------------------------------------------------------------------------
# delay-time surrogate (Eq. 15) and the straight-through gradient

SLOT = 4410


def surrogate(z, N: int = SLOT) -> torch.Tensor:
    """(1/N) sum_k z^k exp(2 pi i k n / N), n = 0..N-1 (complex128), as the inverse DFT of the
    damped sinusoid z^k; z is a complex number or a complex (differentiable) tensor."""
    k = torch.arange(N, dtype=F64).to(C128)
    zt = torch.as_tensor(z, dtype=C128)
    return torch.fft.ifft(torch.exp(k * torch.log(zt)))


def surrogate_deriv(z: complex, N: int = SLOT) -> np.ndarray:
    """ds/dz = (1/N) sum_{k>=1} k z^(k-1) exp(2 pi i k n / N), n = 0..N-1."""
    k = np.arange(N, dtype=np.float64)
    return np.fft.ifft(k * z ** np.maximum(k - 1, 0))


def surrogate_closed_form(z: complex, N: int = SLOT) -> np.ndarray:
    """The geometric series of `surrogate`: (1 - z^N) / (N (1 - z e^(2 pi i n / N)))."""
    n = np.arange(N)
    return (1.0 - z ** N) / (N * (1.0 - z * np.exp(2j * np.pi * n / N)))


def phasor_grad(G: np.ndarray, z: complex, N: int = SLOT) -> tuple[float, float]:
    """Straight-through gradient of one slot's phasor from G[n] = dL/ds[n], n = 0..N-1."""
    sp = surrogate_deriv(z, N)
    return float(np.sum(G * sp.real)), float(-np.sum(G * sp.imag))


def normalise_phasor_grads(g: np.ndarray) -> np.ndarray:
    """Unit-norm gradient per phasor: g [..., 2] (d/dRe z, d/dIm z) divided by its length
    (zero stays zero). Parity unpinned: the paper does not give its normalisation."""
    n = np.linalg.norm(g, axis=-1, keepdims=True)
    return np.where(n > 0, g / np.where(n > 0, n, 1.0), 0.0)


def unit_circle_penalty(z: np.ndarray, weight: float) -> tuple[float, np.ndarray]:
    """weight * sum (|z| - 1)^2 and its gradient with respect to (Re z, Im z). Parity unpinned:
    the paper gives neither the regulariser's form nor its weight."""
    r = np.abs(z)
    val = float(weight * np.sum((r - 1.0) ** 2))
    scale = np.where(r > 0, 2.0 * weight * (r - 1.0) / np.where(r > 0, r, 1.0), 0.0)
    return val, np.stack([scale * z.real, scale * z.imag], axis=-1)
