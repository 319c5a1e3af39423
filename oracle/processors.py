"""Oracle processors in torch float64 (paper Sec. 3, "Differentiable Audio Processors").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every processor maps an input u of shape [2, T] (left, right; the paper's default is stereo)
and one parameter row p to an output y of shape [2, T]. Gradients come from torch autograd; the
one exception is the one-pole envelope, computed by the textbook recursion (scipy's `lfilter`)
and wrapped with its adjoint recursion (pinned by finite differences and by the convolution
form of Eq. 9).

Readings of passages the paper leaves open (each is listed with its reason in the design notes):
* EQ tap range: 2047 taps centred at 0 (n = -1023..1023); the printed bound would give 2049.
* EQ magnitudes: the 1024 log-magnitudes are the independent bins of a real, even response of
  odd length 2047 (bin N-k mirrors bin k).
* EQ window: symmetric Hann centred at 0, v[n] = 0.5 + 0.5 cos(pi n / 1023).
* EQ alignment: centred ("same") convolution, zero input outside [0, T).
* compressor mid signal: u_l + u_r (a sum, as printed); the envelope starts from g[-1] = 0;
  G_u = ln(g + 1e-8); the FIR of Eq. 9 is untruncated, i.e. equal to the one-pole recursion;
  the gain exp(G_y - G_u) multiplies the amplitude as printed; W <= 0 means a hard knee.
* attack/release ballistics (Eq. 8 unrestricted): the attack coefficient applies while the
  envelope rises, i.e. when x[t] > g[t-1]; a tie counts as release.
* delay (Eq. 14): M 100 ms slots of 4410 samples per channel, M = 20 (2 s, the paper's setting,
  880 parameters: node type delay_long) or M = 5 (500 ms, 220 parameters: node type delay); the
  delay inside slot m is read from the phase of z as rint(-arg(z) * 4410 / 2 pi) mod 4410,
  computed in float32 because it decides an integer; each slot's 39-tap filter follows the EQ
  recipe with N = 39 and 20 log-magnitudes; the output is the wet signal only.
* tanh distortion (not in the paper): y = tanh(exp(p) u).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.signal
import torch

F64 = torch.float64
EPS_ENV = 1e-8


# ---------------------------------------------------------------------------------------------
# gain / panning (Eq. 2) and stereo imager (Eq. 3)

def gain_pan(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """y_c = exp(p_c) u_c, one log-gain per channel."""
    return torch.exp(p)[:, None] * u


def imager(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """Mid = l + r, side = exp(p) (l - r); back to stereo as ((m+s)/2, (m-s)/2)."""
    m = u[0] + u[1]
    s = torch.exp(p[0]) * (u[0] - u[1])
    return torch.stack([(m + s) / 2, (m - s) / 2])


# ---------------------------------------------------------------------------------------------
# zero-phase FIR design (Eq. 4): shared by the EQ (N = 2047) and the delay taps (N = 39)

def zero_phase_fir(logmag: torch.Tensor, N: int, windowed: bool = True) -> torch.Tensor:
    """Length-N (odd) zero-phase FIR from (N+1)/2 log-magnitudes: the inverse DFT of the real,
    even magnitude response exp(logmag) (bin N-k mirrors bin k), times a symmetric Hann window
    (omitted when `windowed` is False). Returns taps for n = -(N-1)/2 .. (N-1)/2."""
    M = (N - 1) // 2
    assert logmag.shape[-1] == M + 1
    A = torch.exp(logmag)
    n = torch.arange(-M, M + 1, dtype=F64)
    k = torch.arange(1, M + 1, dtype=F64)
    # inverse DFT of an even spectrum: (A_0 + 2 sum_k A_k cos(2 pi k n / N)) / N
    cosmat = torch.cos(2.0 * math.pi * torch.outer(n, k) / N)
    h0 = (A[0] + 2.0 * (cosmat @ A[1:])) / N
    if not windowed:
        return h0
    window = 0.5 + 0.5 * torch.cos(math.pi * n / M)
    return window * h0


def linear_conv_centred(u: torch.Tensor, h: torch.Tensor, offset: int) -> torch.Tensor:
    """y[t] = sum_j h[j] u[t - (j + offset)] over a [C, T] input, zero input outside [0, T):
    tap j of `h` sits at lag j + offset. Computed as a float64 FFT linear convolution."""
    C, T = u.shape
    L = h.shape[-1]
    n = 1
    while n < T + L:
        n *= 2
    Uf = torch.fft.rfft(u, n=n)
    Hf = torch.fft.rfft(h, n=n)
    full = torch.fft.irfft(Uf * Hf, n=n)  # full[t'] = sum_j h[j] u[t' - j]
    # y[t] = full[t - offset]
    start = -offset
    if start >= 0:
        return full[..., start:start + T]
    pad = torch.zeros(u.shape[:-1] + (-start,), dtype=u.dtype)
    return torch.cat([pad, full[..., :T + start]], dim=-1)


def eq(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """Zero-phase FIR EQ (Eqs. 4-5): 2047 taps from 1024 log-magnitudes, same FIR on both
    channels, centred convolution."""
    h = zero_phase_fir(p, 2047)
    return linear_conv_centred(u, h, -1023)


def eq_direct(u: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Direct-sum form of the EQ for small inputs (numpy float64), used to cross-check the FFT
    convolution: y_c[t] = sum_{n=-1023}^{1023} h[n] u_c[t - n]."""
    h = zero_phase_fir(torch.as_tensor(p, dtype=F64), 2047).numpy()
    C, T = u.shape
    y = np.zeros((C, T))
    for t in range(T):
        lo, hi = max(0, t - 1023), min(T - 1, t + 1023)
        for s in range(lo, hi + 1):
            y[:, t] += h[t - s + 1023] * u[:, s]
    return y


# ---------------------------------------------------------------------------------------------
# compressor (Eqs. 8-12)

class _OnePole(torch.autograd.Function):
    """g[t] = alpha g[t-1] + (1 - alpha) x[t], g[-1] = 0 (Eq. 8 with equal attack and release),
    by the textbook recursion. Adjoint: lambda[t] = gbar[t] + alpha lambda[t+1];
    xbar = (1 - alpha) lambda; alphabar = sum_t lambda[t] (g[t-1] - x[t])."""

    @staticmethod
    def forward(ctx, x, alpha):
        a = float(alpha)
        g = scipy.signal.lfilter([1.0 - a], [1.0, -a], x.detach().numpy())
        g = torch.as_tensor(g, dtype=F64)
        ctx.save_for_backward(x, alpha, g)
        return g

    @staticmethod
    def backward(ctx, gbar):
        x, alpha, g = ctx.saved_tensors
        a = float(alpha)
        lam = scipy.signal.lfilter([1.0], [1.0, -a], gbar.detach().numpy()[::-1])[::-1].copy()
        lam = torch.as_tensor(lam, dtype=F64)
        gprev = torch.cat([torch.zeros(1, dtype=F64), g[:-1]])
        return (1.0 - alpha) * lam, (lam * (gprev - x)).sum().reshape(alpha.shape)


def one_pole(x: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    return _OnePole.apply(x, alpha)


def one_pole_fir(x: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """Eq. 9 form: the envelope as the convolution of x with h[n] = (1 - alpha) alpha^n, taken
    untruncated (length >= T), by FFT. Used to pin the recursion."""
    T = x.shape[-1]
    n = torch.arange(T, dtype=F64)
    h = (1.0 - alpha) * torch.exp(n * torch.log(alpha))
    return linear_conv_centred(x[None], h, 0)[0]


def gain_computer(Gu, thr, knee, ratio):
    """Quadratic-knee static curve (Eqs. 10-11): returns G_y for log-energy G_u."""
    above = thr + (Gu - thr) / ratio
    if float(torch.as_tensor(knee).detach()) <= 0.0:
        return torch.where(Gu < thr, Gu, above)
    mid = Gu + (1.0 / ratio - 1.0) * (Gu - thr + knee) ** 2 / (4.0 * knee)
    return torch.where(Gu < thr - knee, Gu, torch.where(Gu < thr + knee, mid, above))


def compressor(u: torch.Tensor, p: torch.Tensor, envelope=one_pole) -> torch.Tensor:
    """Feed-forward compressor: x = (u_l + u_r)^2, one-pole energy envelope g, G_u = ln(g+eps),
    quadratic-knee curve, y = exp(G_y - G_u) u (Eq. 12). p = (alpha, T, W, R)."""
    alpha, thr, knee, ratio = p[0], p[1], p[2], p[3]
    x = (u[0] + u[1]) ** 2
    g = envelope(x, alpha)
    Gu = torch.log(g + EPS_ENV)
    Gy = gain_computer(Gu, thr, knee, ratio)
    return torch.exp(Gy - Gu)[None, :] * u


def gate_computer(Gu, thr, knee, ratio):
    """Noisegate static curve (Sec. 3 "Noisegate"): G_y = G_u at or above T + W, a quadratic knee
    G_u + (1 - R)(G_u - T - W)^2 / (4W) on [T - W, T + W), and T + R (G_u - T) below T - W (an
    expander of ratio R). A knee width W <= 0 is read as a hard knee at T."""
    below = thr + ratio * (Gu - thr)
    if float(torch.as_tensor(knee).detach()) <= 0.0:
        return torch.where(Gu < thr, below, Gu)
    mid = Gu + (1.0 - ratio) * (Gu - thr - knee) ** 2 / (4.0 * knee)
    return torch.where(Gu < thr - knee, below, torch.where(Gu < thr + knee, mid, Gu))


def noisegate(u: torch.Tensor, p: torch.Tensor, envelope=one_pole) -> torch.Tensor:
    """Noisegate (Sec. 3 "Noisegate"): the compressor's energy envelope and output rule
    (Eqs. 8, 9, 12) with the gate's static curve. p = (alpha, T, W, R)."""
    alpha, thr, knee, ratio = p[0], p[1], p[2], p[3]
    x = (u[0] + u[1]) ** 2
    g = envelope(x, alpha)
    Gu = torch.log(g + EPS_ENV)
    Gy = gate_computer(Gu, thr, knee, ratio)
    return torch.exp(Gy - Gu)[None, :] * u


class _Ballistics(torch.autograd.Function):
    """Eq. 8 with distinct attack and release coefficients: alpha[t] = alpha_a while the envelope
    rises (x[t] > g[t-1]) and alpha_r otherwise (an unchanged envelope, x[t] = g[t-1], counts as
    release; both branches give the same g there); g[-1] = 0. Literal per-sample loop in float64.
    With the branch pattern fixed the recursion is linear, so the adjoint is the one-pole adjoint
    with a per-sample coefficient: lambda[t] = gbar[t] + alpha[t+1] lambda[t+1];
    xbar[t] = (1 - alpha[t]) lambda[t]; the gradient of each coefficient sums
    lambda[t] (g[t-1] - x[t]) over the samples that use it (the switch itself has zero
    derivative almost everywhere)."""

    @staticmethod
    def forward(ctx, x, alpha_a, alpha_r):
        xs = x.detach().numpy()
        aa, ar = float(alpha_a), float(alpha_r)
        g = np.empty_like(xs)
        attack = np.zeros(xs.shape[0], dtype=bool)
        prev = 0.0
        for t in range(xs.shape[0]):
            up = xs[t] > prev
            a = aa if up else ar
            prev = a * prev + (1.0 - a) * xs[t]
            g[t] = prev
            attack[t] = up
        g = torch.as_tensor(g, dtype=F64)
        att = torch.as_tensor(attack)
        ctx.save_for_backward(x, alpha_a, alpha_r, g, att)
        return g

    @staticmethod
    def backward(ctx, gbar):
        x, alpha_a, alpha_r, g, att = ctx.saved_tensors
        a = np.where(att.numpy(), float(alpha_a), float(alpha_r))
        gb = gbar.detach().numpy()
        lam = np.empty_like(gb)
        nxt = 0.0  # alpha[t+1] lambda[t+1]
        for t in range(gb.shape[0] - 1, -1, -1):
            lam[t] = gb[t] + nxt
            nxt = a[t] * lam[t]
        lam = torch.as_tensor(lam, dtype=F64)
        gprev = torch.cat([torch.zeros(1, dtype=F64), g[:-1]])
        d = lam * (gprev - x)
        xbar = torch.as_tensor(1.0 - a, dtype=F64) * lam
        return (xbar, d[att].sum().reshape(alpha_a.shape),
                d[~att].sum().reshape(alpha_r.shape))


def ballistics(x: torch.Tensor, alpha_a: torch.Tensor, alpha_r: torch.Tensor) -> torch.Tensor:
    return _Ballistics.apply(x, alpha_a, alpha_r)


def compressor_ar(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """Compressor with distinct attack and release ballistics (Eq. 8 unrestricted, then
    Eqs. 10-12 as for the compressor). p = (alpha_a, alpha_r, T, W, R)."""
    return compressor(u, torch.stack([p[0], p[2], p[3], p[4]]),
                      envelope=lambda x, _a: ballistics(x, p[0], p[1]))


def envelope_loop(x: np.ndarray, alpha: float) -> np.ndarray:
    """Literal per-sample loop of Eq. 8 (pure Python; small inputs only)."""
    g = np.zeros_like(x, dtype=np.float64)
    prev = 0.0
    for t in range(x.shape[0]):
        prev = alpha * prev + (1.0 - alpha) * float(x[t])
        g[t] = prev
    return g


# ---------------------------------------------------------------------------------------------
# multitap delay (Eq. 14), limited to five 100 ms slots

DELAY_SLOT = 4410
DELAY_TAPS = 5          # slots of the 500 ms delay (node type delay)
DELAY_TAPS_LONG = 20    # slots of the 2 s delay (node type delay_long)
DELAY_BINS = 20


def delay_slots(p) -> int:
    """Slots per channel of a delay parameter row: 220 values -> 5, 880 -> 20."""
    m = int(np.prod(np.shape(p))) // (2 * (2 + DELAY_BINS))
    if m not in (DELAY_TAPS, DELAY_TAPS_LONG) or m * 2 * (2 + DELAY_BINS) != int(np.prod(np.shape(p))):
        raise ValueError(f"a delay row has 220 or 880 values, not {int(np.prod(np.shape(p)))}")
    return m


def delay_offsets(p: np.ndarray) -> np.ndarray:
    """Integer delay per (channel, slot), decided in float32 from the phase of z."""
    M = delay_slots(p)
    q = np.asarray(p, dtype=np.float32).reshape(2, M, 2 + DELAY_BINS)
    ph = np.arctan2(q[..., 1], q[..., 0]).astype(np.float32)
    frac = np.rint(-ph * np.float32(DELAY_SLOT / (2.0 * math.pi))).astype(np.int64)
    d = np.mod(frac, DELAY_SLOT)
    return d + DELAY_SLOT * np.arange(M)[None, :]


def delay(u: torch.Tensor, p: torch.Tensor, surrogate: bool = False) -> torch.Tensor:
    """y_c[t] = sum_m sum_{j=-19}^{19} c_{c,m}[j] u_c[t - d_{c,m} - j]: per channel, M (5 or 20)
    integer delays, each followed by its own 39-tap zero-phase FIR. The integer delays carry no
    gradient; with `surrogate`, the phasors get the straight-through gradient of Eq. 15 (the
    value is unchanged: see `_delay_surrogate_term`)."""
    y = _delay_exact(u, p)
    if surrogate:
        s = _delay_surrogate_term(u.detach(), p)
        y = y + (s - s.detach())
    return y


def _delay_surrogate_term(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """The delay with each slot's integer delay replaced by the real part of the surrogate
    impulse of its phasor (oracle.reverb.surrogate; 4410 lags from the slot's start), filter
    taps and input held constant: its gradient with respect to the phasors is the
    straight-through gradient."""
    from .reverb import surrogate as surr  # the surrogate lives with the other Eq. 15 helpers
    M = delay_slots(p)
    q = p.reshape(2, M, 2 + DELAY_BINS)
    span = M * DELAY_SLOT + 38
    ys = []
    for c in range(2):
        K = torch.zeros(span, dtype=F64)
        for m in range(M):
            z = torch.complex(q[c, m, 0], q[c, m, 1])
            s = surr(z, DELAY_SLOT).real  # impulse at lag n within the slot, n = 0..4409
            taps = zero_phase_fir(q[c, m, 2:].detach(), 39)
            cs = torch.nn.functional.conv1d(s.view(1, 1, -1), taps.flip(0).view(1, 1, -1),
                                            padding=38).view(-1)  # (taps * s)[0 .. 4410 + 37]
            K = K + torch.nn.functional.pad(cs, (m * DELAY_SLOT, span - m * DELAY_SLOT - cs.shape[0]))
        ys.append(linear_conv_centred(u[c:c + 1], K, -19)[0])  # index i at lag i - 19
    return torch.stack(ys)


def _delay_exact(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    d = delay_offsets(p.detach().numpy())
    M = d.shape[1]
    q = p.reshape(2, M, 2 + DELAY_BINS)
    span = int(d.max()) + 39
    ys = []
    for c in range(2):
        h = torch.zeros(span, dtype=F64)
        for m in range(M):
            taps = zero_phase_fir(q[c, m, 2:], 39)
            start = int(d[c, m])  # tap j=-19 sits at lag d - 19 -> index d
            h = h + torch.nn.functional.pad(taps, (start, span - start - 39))
        ys.append(linear_conv_centred(u[c:c + 1], h, -19)[0])
    return torch.stack(ys)


# ---------------------------------------------------------------------------------------------
# tanh distortion (not in the paper; drive in natural-log amplitude units)

def tanh_dist(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    return torch.tanh(torch.exp(p[0]) * u)


def identity(u: torch.Tensor, p=None) -> torch.Tensor:
    return u


PROCESS = {2: identity, 3: gain_pan, 4: eq, 5: compressor, 6: imager, 7: delay, 8: tanh_dist,
           9: noisegate, 10: compressor_ar, 1: identity, 12: delay}
N_PARAMS = {0: 0, 1: 0, 2: 0, 3: 2, 4: 1024, 5: 4, 6: 1, 7: 220, 8: 1, 9: 4, 10: 5, 11: 768,
            12: 880}
REVERB = 11  # the reverb takes its noise realisation besides u and p (oracle.reverb.reverb)
