"""Pins of the oracle processors against closed forms, special cases, library routines and brute
force (paper Sec. 3: Eqs. 2-5, 8-12, 14; tanh distortion is not in the paper)."""
import math

import numpy as np
import pytest
import scipy.signal
import torch

from oracle import processors as P

F64 = torch.float64


def _rand(shape, seed=0):
    return torch.as_tensor(np.random.default_rng(seed).uniform(-0.5, 0.5, size=shape), dtype=F64)


# --- EQ (Eqs. 4-5) -----------------------------------------------------------------------------

def test_flat_eq_is_identity():
    # p = 0: the inverse DFT of a flat unit response is a unit impulse; the window is 1 at n=0
    u = _rand((2, 5000))
    y = P.eq(u, torch.zeros(1024, dtype=F64))
    assert torch.max(torch.abs(y - u)) < 1e-12


def test_eq_spectrum_is_exp_logmag():
    # the unwindowed FIR's DFT at the N = 2047 design frequencies is exp(p_k) (bin N-k = bin k)
    p = torch.as_tensor(np.random.default_rng(1).uniform(-1.4, 1.4, 1024), dtype=F64)
    h0 = P.zero_phase_fir(p, 2047, windowed=False).numpy()
    n = np.arange(-1023, 1024)
    for k in (0, 1, 7, 500, 1023):
        Hk = np.sum(h0 * np.exp(-2j * np.pi * k * n / 2047))
        assert abs(Hk - math.exp(float(p[k]))) < 1e-12
        assert abs(Hk.imag) < 1e-12


def test_single_bin_eq_closed_form():
    # p_j = a, others 0 -> h0[n] = delta[n] + (2/N)(e^a - 1) cos(2 pi j n / N)
    N, j, a = 2047, 37, 0.8
    p = torch.zeros(1024, dtype=F64)
    p[j] = a
    h0 = P.zero_phase_fir(p, N, windowed=False).numpy()
    n = np.arange(-1023, 1024)
    ref = (n == 0).astype(float) + (2.0 / N) * (math.exp(a) - 1.0) * np.cos(2 * np.pi * j * n / N)
    assert np.max(np.abs(h0 - ref)) < 1e-13
    h = P.zero_phase_fir(p, N).numpy()
    win = h / np.where(np.abs(h0) > 0, h0, 1.0)
    assert abs(h[1023] - h0[1023]) < 1e-15  # window is 1 at the centre
    assert h[0] == 0.0 and h[-1] == 0.0  # and 0 at both ends (symmetric Hann)
    assert np.allclose(win[1:-1][::-1], win[1:-1])  # even


def test_eq_fft_equals_direct_sum():
    rng = np.random.default_rng(2)
    u = rng.uniform(-0.5, 0.5, (2, 2500))
    p = rng.uniform(-1.0, 1.0, 1024)
    y = P.eq(torch.as_tensor(u), torch.as_tensor(p)).numpy()
    y_direct = P.eq_direct(u, p)
    assert np.max(np.abs(y - y_direct)) < 1e-12


def test_eq_matches_numpy_convolve():
    rng = np.random.default_rng(3)
    u = rng.uniform(-0.5, 0.5, (2, 7000))
    p = rng.uniform(-1.0, 1.0, 1024)
    h = P.zero_phase_fir(torch.as_tensor(p), 2047).numpy()
    y = P.eq(torch.as_tensor(u), torch.as_tensor(p)).numpy()
    for c in range(2):
        ref = np.convolve(u[c], h, mode="same")  # "same" centres the odd-length kernel
        assert np.max(np.abs(y[c] - ref)) < 1e-12


# --- compressor (Eqs. 8-12) --------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [0.5, 0.99, 0.99977])
def test_envelope_step_response(alpha):
    c, T = 0.3, 3000
    g = P.one_pole(torch.full((T,), c, dtype=F64), torch.tensor(alpha, dtype=F64)).numpy()
    t = np.arange(T)
    assert np.max(np.abs(g - c * (1 - alpha ** (t + 1)))) < 1e-13


def test_envelope_recursion_forms_agree():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, 1500) ** 2
    a = 0.997
    loop = P.envelope_loop(x, a)
    lf = P.one_pole(torch.as_tensor(x), torch.tensor(a, dtype=F64)).numpy()
    fir = P.one_pole_fir(torch.as_tensor(x), torch.tensor(a, dtype=F64)).numpy()
    assert np.max(np.abs(lf - loop)) < 1e-13
    assert np.max(np.abs(fir - loop)) < 1e-12


def test_envelope_gradient_matches_fd_and_fir_form():
    rng = np.random.default_rng(5)
    x = torch.as_tensor(rng.uniform(0, 1, 300) ** 2).requires_grad_(True)
    a = torch.tensor(0.95, dtype=F64, requires_grad=True)
    assert torch.autograd.gradcheck(P.one_pole, (x, a), eps=1e-6, atol=1e-8)
    w = torch.as_tensor(rng.normal(size=300))
    gx1, ga1 = torch.autograd.grad((P.one_pole(x, a) * w).sum(), (x, a))
    gx2, ga2 = torch.autograd.grad((P.one_pole_fir(x, a) * w).sum(), (x, a))
    assert torch.max(torch.abs(gx1 - gx2)) < 1e-10 and abs(float(ga1 - ga2)) < 1e-8


def test_compressor_below_threshold_is_identity():
    u = _rand((2, 4000))
    p = torch.tensor([0.99, 10.0, 0.69, 4.0], dtype=F64)  # T far above any ln(g)
    y = P.compressor(u, p)
    assert torch.equal(y, u)


def test_compressor_ratio_one_is_identity():
    u = _rand((2, 4000), 1) * 8
    p = torch.tensor([0.99, -3.0, 0.69, 1.0], dtype=F64)
    assert torch.max(torch.abs(P.compressor(u, p) - u)) < 1e-15 * 8


def test_knee_continuity():
    thr, knee, ratio = -2.0, 0.7, 4.0
    Gu = torch.tensor([thr - knee, thr + knee], dtype=F64)
    eps = 1e-9
    lo = P.gain_computer(Gu - eps, thr, knee, ratio)
    hi = P.gain_computer(Gu + eps, thr, knee, ratio)
    assert torch.max(torch.abs(hi - lo)) < 1e-8
    assert abs(float(P.gain_computer(Gu[1:], thr, knee, ratio)) - (thr + knee / ratio)) < 1e-12
    # slopes: 1 below, 1/R above, continuous at both knee edges
    for edge, left_slope, right_slope in ((thr - knee, 1.0, 1.0), (thr + knee, 1 / ratio, 1 / ratio)):
        x = torch.tensor([edge - 2e-6, edge - 1e-6, edge + 1e-6, edge + 2e-6], dtype=F64)
        y = P.gain_computer(x, thr, knee, ratio)
        sl = float((y[1] - y[0]) / 1e-6)
        sr = float((y[3] - y[2]) / 1e-6)
        assert abs(sl - left_slope) < 1e-5 and abs(sr - right_slope) < 1e-5


def test_compressor_static_gain_closed_form():
    # constant input far beyond the envelope's settling time: g -> x, so the gain is the static
    # curve above the knee: y/u = exp((1/R - 1)(ln(x + eps) - T))
    T_, c = 20000, 0.4
    u = torch.full((2, T_), c, dtype=F64)
    alpha, thr, knee, ratio = 0.9, -3.0, 0.5, 3.0
    y = P.compressor(u, torch.tensor([alpha, thr, knee, ratio], dtype=F64))
    x = (2 * c) ** 2
    expect = math.exp((1 / ratio - 1) * (math.log(x + 1e-8) - thr))
    assert abs(float(y[0, -1]) / c - expect) < 1e-12


# --- attack/release ballistics (Eq. 8 with distinct coefficients) ------------------------------

def _bal(x, aa, ar):
    return P.ballistics(torch.as_tensor(x, dtype=F64), torch.tensor(aa, dtype=F64),
                        torch.tensor(ar, dtype=F64))


def test_ballistics_equal_coefficients_is_one_pole():
    x = np.random.default_rng(11).uniform(0, 1, 4000) ** 2
    g = _bal(x, 0.993, 0.993).numpy()
    ref = scipy.signal.lfilter([1 - 0.993], [1, -0.993], x)
    assert np.max(np.abs(g - ref)) < 1e-14


@pytest.mark.parametrize("aa,ar", [(0.9, 0.999), (0.999, 0.95)])
def test_ballistics_attack_then_release_closed_form(aa, ar):
    """A step up from zero is all attack: g = c (1 - aa^(n+1)); after the step down to 0 it is
    all release: g = g_end ar^(n+1)."""
    c, n1, n2 = 0.25, 700, 900
    x = np.concatenate([np.full(n1, c), np.zeros(n2)])
    g = _bal(x, aa, ar).numpy()
    t = np.arange(n1)
    up = c * (1 - aa ** (t + 1))
    assert np.max(np.abs(g[:n1] - up)) < 1e-15
    t2 = np.arange(n2)
    assert np.max(np.abs(g[n1:] - up[-1] * ar ** (t2 + 1))) < 1e-15


@pytest.mark.parametrize("aa,ar", [(0.95, 0.999), (0.999, 0.9), (0.99, 0.99)])
def test_ballistics_is_max_or_min_of_two_affine_maps(aa, ar):
    """Since g_a - g_r = (ar - aa)(x - g_prev), the branch rule picks the larger of the two
    one-pole updates when attack is the faster one (aa <= ar) and the smaller otherwise."""
    x = np.random.default_rng(12).uniform(0, 1, 3000) ** 3
    g = _bal(x, aa, ar).numpy()
    pick = max if aa <= ar else min
    prev, ref = 0.0, np.empty_like(x)
    for t in range(x.shape[0]):
        prev = pick(aa * prev + (1 - aa) * x[t], ar * prev + (1 - ar) * x[t])
        ref[t] = prev
    assert np.max(np.abs(g - ref)) < 1e-15


def test_ballistics_adjoint_matches_autograd_of_the_loop_and_fd():
    """The hand-written adjoint against torch autograd through the per-sample recursion written
    with torch ops (where the branch is a comparison, not differentiated), and against central
    finite differences in both coefficients."""
    rng = np.random.default_rng(13)
    x = torch.as_tensor(rng.uniform(0, 1, 400) ** 2).requires_grad_(True)
    aa = torch.tensor(0.93, dtype=F64, requires_grad=True)
    ar = torch.tensor(0.985, dtype=F64, requires_grad=True)
    w = torch.as_tensor(rng.normal(size=400))
    g1 = torch.autograd.grad((P.ballistics(x, aa, ar) * w).sum(), (x, aa, ar))
    prev, out = torch.zeros((), dtype=F64), []
    for t in range(400):
        a = aa if bool(x[t] > prev) else ar
        prev = a * prev + (1 - a) * x[t]
        out.append(prev)
    g2 = torch.autograd.grad((torch.stack(out) * w).sum(), (x, aa, ar))
    for a_, b_ in zip(g1, g2):
        assert torch.max(torch.abs(a_ - b_)) < 1e-11
    for which in (1, 2):
        h = 1e-7
        args = [x.detach(), aa.detach(), ar.detach()]
        hi = list(args); hi[which] = args[which] + h
        lo = list(args); lo[which] = args[which] - h
        fd = float(((P.ballistics(*hi) - P.ballistics(*lo)) * w).sum()) / (2 * h)
        assert abs(fd - float(g1[which])) < 1e-5 * max(1.0, abs(fd))


def test_compressor_ar_with_equal_coefficients_is_compressor():
    u = _rand((2, 3000), 3) * 4
    p5 = torch.tensor([0.995, 0.995, -3.0, 0.6, 4.0], dtype=F64)
    p4 = torch.tensor([0.995, -3.0, 0.6, 4.0], dtype=F64)
    assert torch.max(torch.abs(P.compressor_ar(u, p5) - P.compressor(u, p4))) < 1e-14


def test_compressor_ar_parameter_gradients_match_fd():
    u = _rand((2, 600), 4) * 4
    p = torch.tensor([0.97, 0.995, -3.0, 0.6, 4.0], dtype=F64, requires_grad=True)
    w = torch.as_tensor(np.random.default_rng(14).normal(size=(2, 600)))
    (gp,) = torch.autograd.grad((P.compressor_ar(u, p) * w).sum(), (p,))
    for i in range(5):
        h = 1e-7
        e = torch.zeros(5, dtype=F64)
        e[i] = h
        fd = float(((P.compressor_ar(u, p.detach() + e) - P.compressor_ar(u, p.detach() - e))
                    * w).sum()) / (2 * h)
        assert abs(fd - float(gp[i])) < 1e-5 * max(1.0, abs(fd)), (i, fd, float(gp[i]))


# --- noisegate (Sec. 3 "Noisegate": the compressor's envelope, a downward-expander curve) ------

def test_noisegate_above_threshold_is_identity():
    u = _rand((2, 4000), 11)
    p = torch.tensor([0.99, -60.0, 0.69, 4.0], dtype=F64)  # T + W far below any ln(g)
    assert torch.equal(P.noisegate(u, p), u)


def test_noisegate_ratio_one_is_identity():
    u = _rand((2, 4000), 12) * 1e-3
    p = torch.tensor([0.99, 5.0, 0.69, 1.0], dtype=F64)  # everything below T, but R = 1
    assert torch.max(torch.abs(P.noisegate(u, p) - u)) < 1e-15 * 1e-3


def test_gate_knee_continuity():
    thr, knee, ratio = -8.0, 0.7, 4.0
    eps = 1e-9
    Gu = torch.tensor([thr - knee, thr + knee], dtype=F64)
    lo = P.gate_computer(Gu - eps, thr, knee, ratio)
    hi = P.gate_computer(Gu + eps, thr, knee, ratio)
    assert torch.max(torch.abs(hi - lo)) < 1e-8
    assert abs(float(P.gate_computer(Gu[:1], thr, knee, ratio)) - (thr - ratio * knee)) < 1e-12
    # slopes: R below, 1 above, continuous at both knee edges
    for edge, slope in ((thr - knee, ratio), (thr + knee, 1.0)):
        x = torch.tensor([edge - 2e-6, edge - 1e-6, edge + 1e-6, edge + 2e-6], dtype=F64)
        y = P.gate_computer(x, thr, knee, ratio)
        sl = float((y[1] - y[0]) / 1e-6)
        sr = float((y[3] - y[2]) / 1e-6)
        assert abs(sl - slope) < 1e-5 and abs(sr - slope) < 1e-5
    # hard knee (W = 0): expander below T, identity above
    y = P.gate_computer(torch.tensor([thr - 1.0, thr + 1.0], dtype=F64), thr, 0.0, ratio)
    assert abs(float(y[0]) - (thr - ratio)) < 1e-12 and abs(float(y[1]) - (thr + 1.0)) < 1e-12


def test_noisegate_static_gain_closed_form():
    # constant input long after the envelope settled (g -> x) and below the knee: the gain is
    # exp(G_y - G_u) = exp((R - 1)(ln(x + eps) - T))
    T_, c = 20000, 0.01
    u = torch.full((2, T_), c, dtype=F64)
    alpha, thr, knee, ratio = 0.9, -2.0, 0.5, 3.0
    y = P.noisegate(u, torch.tensor([alpha, thr, knee, ratio], dtype=F64))
    x = (2 * c) ** 2
    expect = math.exp((ratio - 1) * (math.log(x + 1e-8) - thr))
    assert abs(float(y[0, -1]) / c - expect) < 1e-12 * max(1.0, expect)


# --- gain/pan, imager, tanh (Eqs. 2-3) ----------------------------------------------------------

def test_gain_pan_and_imager_closed_forms():
    u = _rand((2, 100), 6)
    y = P.gain_pan(u, torch.tensor([math.log(2.0), math.log(0.5)], dtype=F64))
    assert torch.allclose(y[0], 2 * u[0], atol=0, rtol=1e-15)
    assert torch.allclose(y[1], 0.5 * u[1], atol=0, rtol=1e-15)
    assert torch.max(torch.abs(P.imager(u, torch.zeros(1, dtype=F64)) - u)) < 1e-16
    y = P.imager(u, torch.tensor([math.log(3.0)], dtype=F64))
    m, s = y[0] + y[1], y[0] - y[1]
    assert torch.max(torch.abs(m - (u[0] + u[1]))) < 1e-15
    assert torch.max(torch.abs(s - 3 * (u[0] - u[1]))) < 1e-15
    y = P.imager(u, torch.tensor([-60.0], dtype=F64))  # side removed: mono
    assert torch.max(torch.abs(y[0] - y[1])) < 1e-15


def test_tanh():
    u = _rand((2, 100), 7)
    y = P.tanh_dist(u, torch.tensor([math.log(3.0)], dtype=F64)).numpy()
    assert np.max(np.abs(y - np.tanh(3 * u.numpy()))) < 1e-15
    small = u * 1e-3
    y = P.tanh_dist(small, torch.zeros(1, dtype=F64))
    assert torch.max(torch.abs(y - (small - small ** 3 / 3))) < 1e-15


# --- delay (Eq. 14) ------------------------------------------------------------------------------

def _delay_p(d, logmags):
    """d [2,M] integer delays inside their slots, logmags [2,M,20] (M = 5 or 20)."""
    M = np.shape(d)[1]
    p = np.zeros((2, M, 22))
    ph = -2 * np.pi * np.asarray(d) / 4410
    p[..., 0], p[..., 1] = np.cos(ph), np.sin(ph)
    p[..., 2:] = logmags
    return p.reshape(2 * M * 22).astype(np.float32)


@pytest.mark.parametrize("M", [5, 20])
def test_delay_offsets_from_phasor(M):
    rng = np.random.default_rng(8)
    d = rng.integers(0, 4410, (2, M))
    d[0, 0], d[0, 1], d[1, 0] = 0, 2205, 4409
    off = P.delay_offsets(_delay_p(d, np.zeros((2, M, 20))))
    assert np.array_equal(off, d + 4410 * np.arange(M)[None, :])


@pytest.mark.parametrize("M,slot0,T", [(5, 2, 30000), (20, 17, 90000)])
def test_delay_single_flat_tap_is_pure_shift(M, slot0, T):
    rng = np.random.default_rng(9)
    d = rng.integers(0, 4410, (2, M))
    lm = np.full((2, M, 20), -1000.0)  # exp(-1000) = 0 to double precision
    lm[0, slot0] = 0.0
    lm[1, 0] = math.log(0.5)
    p32 = _delay_p(d, lm)
    p = torch.as_tensor(p32, dtype=F64)
    u = _rand((2, T), 10)
    y = P.delay(u, p).numpy()
    sh0 = int(d[0, slot0]) + slot0 * 4410
    sh1 = int(d[1, 0])
    half = math.exp(float(p32.reshape(2, M, 22)[1, 0, 2]))  # float32-rounded ln(0.5)
    assert np.max(np.abs(y[0, sh0:] - u.numpy()[0, :T - sh0])) < 1e-12
    assert np.max(np.abs(y[0, :sh0])) < 1e-12
    assert np.max(np.abs(y[1, sh1:] - half * u.numpy()[1, :T - sh1])) < 1e-12


@pytest.mark.parametrize("M,T,points", [(5, 23000, (0, 5, 4500, 13000, 22999)),
                                        (20, 90000, (3, 20000, 70000, 86000, 89999))])
def test_delay_direct_sum(M, T, points):
    rng = np.random.default_rng(11)
    d = rng.integers(0, 4410, (2, M))
    lm = rng.uniform(-2, 0, (2, M, 20))
    p32 = _delay_p(d, lm)
    p = torch.as_tensor(p32, dtype=F64)
    u = _rand((2, T), 12).numpy()
    y = P.delay(torch.as_tensor(u), p).numpy()
    off = P.delay_offsets(p32)
    q = p.reshape(2, M, 22)
    for c in range(2):
        for t in points:
            acc = 0.0
            for m in range(M):
                taps = P.zero_phase_fir(q[c, m, 2:], 39).numpy()
                for j in range(-19, 20):
                    s = t - int(off[c, m]) - j
                    if 0 <= s < T:
                        acc += taps[j + 19] * u[c, s]
            assert abs(acc - y[c, t]) < 1e-12


def test_delay_row_sizes():
    assert P.delay_slots(np.zeros(220)) == 5 and P.delay_slots(np.zeros(880)) == 20
    with pytest.raises(ValueError):
        P.delay_slots(np.zeros(440))


def test_lfilter_reference_for_delay_free_compressor_path():
    # scipy's lfilter with the same one-pole coefficients as an independent library routine
    rng = np.random.default_rng(13)
    x = rng.uniform(0, 1, 500)
    g = P.envelope_loop(x, 0.9)
    assert np.max(np.abs(g - scipy.signal.lfilter([0.1], [1, -0.9], x))) < 1e-14
