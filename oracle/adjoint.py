"""Oracle adjoints written out by hand, one processor at a time (the backpropagation through the
render that gradient-descent matching needs, paper Sec. 4), in torch float64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function takes a node's aggregated input u [2, T], its parameter row p and the adjoint of
its output ybar [2, T], and returns (ubar [2, T], pbar [N_t]), the adjoints of the input and of
the parameters. They are derived from the forward definitions in `processors` (which follow the
paper's Eqs. 2-5, 8-12 and 14) without autograd, so that a graph too large for autograd's saved
state (the 256-track console at T = 2^20) can be differentiated one node at a time (`streamed`).

Derivations (y the output, rho = sum_c ybar_c y_c where a gain multiplies both channels):
* gain/pan (Eq. 2): ubar_c = e^{p_c} ybar_c;  pbar_c = sum_t ybar_c y_c.
* imager (Eq. 3): with m = l + r, s = e^p (l - r): ubar_l = ((1 + e^p) ybar_l + (1 - e^p) ybar_r)/2,
  ubar_r = ((1 - e^p) ybar_l + (1 + e^p) ybar_r)/2;  pbar = sum_t (ybar_l - ybar_r)/2 * s.
* zero-phase FIR (Eqs. 4-5): y_c[t] = sum_n h[n] u_c[t - n] with h even, so ubar is the same
  filter applied to ybar; hbar[n] = sum_{c,t} ybar_c[t] u_c[t - n]; h = v h0 gives
  h0bar = v hbar; h0[n] = (A_0 + 2 sum_k A_k cos(2 pi k n / N)) / N gives
  Abar_k = (kappa_k / N) sum_n h0bar[n] cos(2 pi k n / N) (kappa_0 = 1, else 2), and A = e^p
  gives pbar = A Abar.
* compressor (Eqs. 8-12) and noisegate (Sec. 3): e = G_y - G_u with G_y = phi(G_u; T, W, R),
  gamma = e^e, y = gamma u, so dy_c/dG_u = gamma u_c (phi' - 1) and
  Gbar_u = rho (phi' - 1); gbar = Gbar_u / (g + eps); the envelope g[t] = a g[t-1] + (1 - a) x[t]
  has the reverse recursion lambda[t] = gbar[t] + a lambda[t+1] (lambda[T] = 0), so
  xbar = (1 - a) lambda and abar = sum_t lambda[t] (g[t-1] - x[t]); x = (l + r)^2 gives
  ubar_c = gamma ybar_c + 2 (l + r) xbar; and (T, W, R)bar = sum_t rho dphi/d(T, W, R).
* multitap delay (Eq. 14): y_c = sum_m c_{c,m} * u_c shifted by d_{c,m}: ubar_c is the
  correlation of ybar_c with the same taps; each slot's tap adjoint is
  cbar_{c,m}[j] = sum_t ybar_c[t] u_c[t - d_{c,m} - j] and reaches its 20 log-magnitudes through
  the FIR chain above with N = 39. The delay times get no gradient (as in `processors.delay`).
* tanh (not in the paper): y = tanh(e^p u): ubar = ybar e^p (1 - y^2);
  pbar = sum ybar (1 - y^2) e^p u.
* mix, out: ubar = ybar.

Parity pins (tests): every function equals torch autograd through the forward processor (to
1e-10 of the largest entry) on random inputs, for each branch of the gain curves; the streamed
adjoint of whole graphs equals autograd through `render`.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.signal
import torch

from . import processors as P

F64 = torch.float64


def xcorr(a: torch.Tensor, b: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    """c[lag] = sum_t a[t] b[t - lag] for lag = lo..hi (both [T] float64, zero outside [0, T)),
    by a float64 FFT long enough that no lag wraps around."""
    T = a.shape[-1]
    n = 1
    while n < T + max(abs(lo), abs(hi)) + 1:
        n *= 2
    c = torch.fft.irfft(torch.fft.rfft(a, n=n) * torch.conj(torch.fft.rfft(b, n=n)), n=n)
    lags = torch.arange(lo, hi + 1)
    return c[lags % n]


def fir_param_adjoint(logmag: torch.Tensor, hbar: torch.Tensor, N: int) -> torch.Tensor:
    """Adjoint of `processors.zero_phase_fir` (windowed): the log-magnitude gradient from the
    gradient hbar of the taps n = -(N-1)/2 .. (N-1)/2."""
    M = (N - 1) // 2
    n = torch.arange(-M, M + 1, dtype=F64)
    window = 0.5 + 0.5 * torch.cos(math.pi * n / M)
    h0bar = window * hbar
    k = torch.arange(0, M + 1, dtype=F64)
    kappa = torch.full((M + 1,), 2.0, dtype=F64)
    kappa[0] = 1.0
    cosmat = torch.cos(2.0 * math.pi * torch.outer(k, n) / N)  # [M+1, N]
    Abar = kappa / N * (cosmat @ h0bar)
    return torch.exp(logmag) * Abar


def gain_pan(u, p, ybar):
    g = torch.exp(p)
    y = g[:, None] * u
    return g[:, None] * ybar, (ybar * y).sum(dim=1)


def imager(u, p, ybar):
    e = torch.exp(p[0])
    ul = ((1 + e) * ybar[0] + (1 - e) * ybar[1]) / 2
    ur = ((1 - e) * ybar[0] + (1 + e) * ybar[1]) / 2
    s = e * (u[0] - u[1])
    return torch.stack([ul, ur]), (((ybar[0] - ybar[1]) / 2) * s).sum().reshape(1)


def eq(u, p, ybar):
    h = P.zero_phase_fir(p, 2047)
    ubar = P.linear_conv_centred(ybar, h, -1023)
    hbar = xcorr(ybar[0], u[0], -1023, 1023) + xcorr(ybar[1], u[1], -1023, 1023)
    return ubar, fir_param_adjoint(p, hbar, 2047)


def _comp_curve_grads(Gu, thr, knee, ratio):
    """phi'(G_u) and dphi/d(T, W, R) of the compressor's quadratic-knee curve (Eqs. 10-11)."""
    one, zero = torch.ones_like(Gu), torch.zeros_like(Gu)
    c = 1.0 / ratio - 1.0
    d = Gu - thr
    if knee <= 0.0:
        above = Gu >= thr
        dG = torch.where(above, one / ratio, one)
        dT = torch.where(above, one * (1.0 - 1.0 / ratio), zero)
        dR = torch.where(above, -d / ratio ** 2, zero)
        return dG, dT, zero, dR
    q = d + knee  # G_u - T + W
    below, inknee = Gu < thr - knee, (Gu >= thr - knee) & (Gu < thr + knee)
    dG = torch.where(below, one, torch.where(inknee, 1.0 + c * q / (2 * knee), one / ratio))
    dT = torch.where(below, zero, torch.where(inknee, -c * q / (2 * knee), one * (1.0 - 1.0 / ratio)))
    dW = torch.where(inknee, c * (2 * q / (4 * knee) - q ** 2 / (4 * knee ** 2)), zero)
    dR = torch.where(below, zero, torch.where(inknee, -q ** 2 / (4 * knee) / ratio ** 2,
                                              -d / ratio ** 2))
    return dG, dT, dW, dR


def _gate_curve_grads(Gu, thr, knee, ratio):
    """phi'(G_u) and dphi/d(T, W, R) of the noisegate's curve (Sec. 3 "Noisegate")."""
    one, zero = torch.ones_like(Gu), torch.zeros_like(Gu)
    d = Gu - thr
    if knee <= 0.0:
        below = Gu < thr
        return (torch.where(below, one * ratio, one), torch.where(below, one * (1.0 - ratio), zero),
                zero, torch.where(below, d, zero))
    q = d - knee  # G_u - T - W
    below, inknee = Gu < thr - knee, (Gu >= thr - knee) & (Gu < thr + knee)
    g1 = 1.0 - ratio
    dG = torch.where(below, one * ratio, torch.where(inknee, 1.0 + g1 * q / (2 * knee), one))
    dT = torch.where(below, one * (1.0 - ratio), torch.where(inknee, -g1 * q / (2 * knee), zero))
    dW = torch.where(inknee, g1 * (-2 * q / (4 * knee) - q ** 2 / (4 * knee ** 2)), zero)
    dR = torch.where(below, d, torch.where(inknee, -q ** 2 / (4 * knee), zero))
    return dG, dT, dW, dR


def _dynamics(u, p, ybar, curve, grads):
    a, thr, knee, ratio = (float(v) for v in p)
    x = (u[0] + u[1]) ** 2
    g = torch.as_tensor(scipy.signal.lfilter([1.0 - a], [1.0, -a], x.numpy()), dtype=F64)
    Gu = torch.log(g + P.EPS_ENV)
    Gy = curve(Gu, torch.tensor(thr, dtype=F64), torch.tensor(knee, dtype=F64),
               torch.tensor(ratio, dtype=F64))
    gamma = torch.exp(Gy - Gu)
    y = gamma[None, :] * u
    rho = (ybar * y).sum(dim=0)
    dG, dT, dW, dR = grads(Gu, thr, knee, ratio)
    gbar = rho * (dG - 1.0) / (g + P.EPS_ENV)
    lam = torch.as_tensor(scipy.signal.lfilter([1.0], [1.0, -a], gbar.numpy()[::-1])[::-1].copy(),
                          dtype=F64)
    gprev = torch.cat([torch.zeros(1, dtype=F64), g[:-1]])
    xbar = (1.0 - a) * lam
    ubar = gamma[None, :] * ybar + (2.0 * (u[0] + u[1]) * xbar)[None, :]
    pbar = torch.stack([(lam * (gprev - x)).sum(), (rho * dT).sum(), (rho * dW).sum(),
                        (rho * dR).sum()])
    return ubar, pbar


def compressor(u, p, ybar):
    return _dynamics(u, p, ybar, P.gain_computer, _comp_curve_grads)


def noisegate(u, p, ybar):
    return _dynamics(u, p, ybar, P.gate_computer, _gate_curve_grads)


def delay(u, p, ybar):
    d = P.delay_offsets(p.numpy())
    M = d.shape[1]
    q = p.reshape(2, M, 2 + P.DELAY_BINS)
    span = int(d.max()) + 39
    ubar, pbar = [], torch.zeros_like(q)
    for c in range(2):
        h = torch.zeros(span, dtype=F64)
        for m in range(M):
            start = int(d[c, m])
            h[start:start + 39] += P.zero_phase_fir(q[c, m, 2:], 39)
        # forward: y[t] = sum_j h[j] u[t - (j - 19)]; adjoint: the reversed filter
        ubar.append(P.linear_conv_centred(ybar[c:c + 1], torch.flip(h, [0]), -(span - 20))[0])
        # hbar[j] = sum_t ybar[t] u[t - (j - 19)] for j = 0..span-1
        hbar = xcorr(ybar[c], u[c], -19, span - 20)
        for m in range(M):
            start = int(d[c, m])
            pbar[c, m, 2:] = fir_param_adjoint(q[c, m, 2:], hbar[start:start + 39], 39)
    return torch.stack(ubar), pbar.reshape(-1)


def tanh_dist(u, p, ybar):
    e = torch.exp(p[0])
    y = torch.tanh(e * u)
    s = ybar * (1.0 - y ** 2)
    return s * e, (s * e * u).sum().reshape(1)


def identity(u, p, ybar):
    return ybar, None


ADJOINT = {1: identity, 2: identity, 3: gain_pan, 4: eq, 5: compressor, 6: imager, 7: delay,
           8: tanh_dist, 9: noisegate, 12: delay}
