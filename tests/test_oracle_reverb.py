"""Pins of the oracle's reverb (paper Sec. 3 "Reverb", Eqs. 6-7) and delay-time surrogate
(Sec. 3 "Multitap delay", Eq. 15), each against something other than the oracle itself:
closed forms written out with explicit loops, the STFT's constant-overlap-add property, a direct
convolution sum, and finite differences."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import processors as OP
from oracle import render as OR
from oracle import reverb as RV

F64 = torch.float64


def hann(q):
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * q / 384.0)


def params(h0_m, hd_m, h0_s, hd_s):
    p = np.zeros((2, 2, 192))
    p[0, 0], p[0, 1], p[1, 0], p[1, 1] = h0_m, hd_m, h0_s, hd_s
    return torch.as_tensor(p.reshape(768), dtype=F64)


@pytest.mark.parametrize("L", [3000, 4800, synth.REVERB_LEN])
def test_all_ones_mask_gives_back_the_noise(L):
    """H0 = HD = 0: the periodic Hann window at hop N/2 sums to one, so the STFT round trip
    returns each noise signal, and mid/side to stereo gives ((m + s) / 2, (m - s) / 2)."""
    noise = synth.reverb_noise(3, L).astype(np.float64)
    h = RV.reverb_ir(params(0, 0, 0, 0), torch.as_tensor(noise)).numpy()
    assert np.max(np.abs(h[0] - (noise[0] + noise[1]) / 2)) < 1e-12
    assert np.max(np.abs(h[1] - (noise[0] - noise[1]) / 2)) < 1e-12


def test_frame_only_mask_closed_form():
    """A mask exp(c + m d) that does not depend on k scales each windowed frame by its own
    factor, so h[n] = noise[n] e^c sum_m e^(m d) w[n - 192 m + 192] (frames m = 0..M-1)."""
    L, c, d = 2500, -0.7, -0.05
    noise = synth.reverb_noise(4, L).astype(np.float64)
    h = RV.reverb_ir(params(c, d, c, d), torch.as_tensor(noise)).numpy()
    M = -(-L // 192) + 1
    scale = np.zeros(L)
    for n in range(L):
        for m in range(M):
            q = n - 192 * m + 192
            if 0 <= q < 384:
                scale[n] += math.exp(c + m * d) * hann(q)
    hm, hs = noise[0] * scale, noise[1] * scale
    assert np.max(np.abs(h[0] - (hm + hs) / 2)) < 1e-12
    assert np.max(np.abs(h[1] - (hm - hs) / 2)) < 1e-12


@pytest.mark.parametrize("k0", [1, 37, 191])
def test_single_bin_mask_closed_form(k0):
    """A mask that keeps one bin 0 < k0 < 192 (every other bin at exp(-60)) turns each frame
    into the real sinusoid (2 / 384) Re(X[k0] e^(2 pi i k0 q / 384)), X[k0] the DFT of the
    windowed frame at k0 written out as a sum; the frames overlap-add into h. Checks the bin
    index of the mask and the one-sided inverse. For k0 = 191 the Nyquist bin 192 shares the
    mask of bin 191 and adds its own term (1 / 384) X[192] (-1)^q."""
    L = 1500
    noise = synth.reverb_noise(5, L).astype(np.float64)
    h0 = np.full(192, -60.0)
    h0[k0] = 0.0
    h = RV.reverb_ir(params(h0, 0, h0, 0), torch.as_tensor(noise)).numpy()
    M = -(-L // 192) + 1
    q = np.arange(384)
    ref = []
    for x in range(2):
        out = np.zeros((M - 1) * 192 + 384)
        for m in range(M):
            seg = np.zeros(384)
            for qq in range(384):
                n = 192 * m - 192 + qq
                if 0 <= n < L:
                    seg[qq] = noise[x][n] * hann(qq)
            X = sum(seg[qq] * np.exp(-2j * np.pi * k0 * qq / 384) for qq in range(384))
            out[192 * m:192 * m + 384] += (2.0 / 384.0) * np.real(
                X * np.exp(2j * np.pi * k0 * q / 384))
            if k0 == 191:
                Xn = sum(seg[qq] * (-1.0) ** qq for qq in range(384))
                out[192 * m:192 * m + 384] += (1.0 / 384.0) * Xn * (-1.0) ** q
        ref.append(out[192:192 + L])
    hl, hr = (ref[0] + ref[1]) / 2, (ref[0] - ref[1]) / 2
    tol = 1e-9 * np.max(np.abs(hl))
    assert np.max(np.abs(h[0] - hl)) < tol and np.max(np.abs(h[1] - hr)) < tol


def test_side_mask_off_gives_identical_channels():
    L = 2000
    noise = synth.reverb_noise(6, L).astype(np.float64)
    rng = np.random.default_rng(1)
    h = RV.reverb_ir(params(rng.uniform(-1, 0, 192), rng.uniform(-0.05, 0, 192), -200.0, 0.0),
                     torch.as_tensor(noise)).numpy()
    assert np.array_equal(h[0], h[1])


def test_causal_convolution_against_direct_sum():
    rng = np.random.default_rng(2)
    u = rng.normal(size=(2, 700))
    h = rng.normal(size=(2, 300))
    y = RV.causal_conv(torch.as_tensor(u), torch.as_tensor(h)).numpy()
    for c in range(2):
        ref = np.array([sum(h[c][n] * u[c][t - n] for n in range(min(t + 1, 300)))
                        for t in range(700)])
        assert np.max(np.abs(y[c] - ref)) < 1e-10


def test_reverb_gradients_against_finite_differences():
    L, T = 600, 900
    noise = synth.reverb_noise(7, L)
    rng = np.random.default_rng(3)
    p0 = synth.reverb_params(rng, 1)[0].astype(np.float64)
    u0 = rng.normal(size=(2, T))
    w = rng.normal(size=(2, T))

    def loss(p, u):
        return torch.sum(torch.as_tensor(w) * RV.reverb(u, p, noise))

    p = torch.as_tensor(p0).requires_grad_(True)
    u = torch.as_tensor(u0).requires_grad_(True)
    gp, gu = torch.autograd.grad(loss(p, u), [p, u])
    eps = 1e-6
    for i in [0, 5, 191, 192, 250, 383, 384, 500, 600, 767]:
        dp = np.zeros(768)
        dp[i] = eps
        fd = (loss(torch.as_tensor(p0 + dp), torch.as_tensor(u0)) -
              loss(torch.as_tensor(p0 - dp), torch.as_tensor(u0))).item() / (2 * eps)
        assert abs(fd - gp[i].item()) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gp[i].item())
    for c, t in [(0, 0), (1, 450), (0, 899)]:
        du = np.zeros((2, T))
        du[c, t] = eps
        fd = (loss(torch.as_tensor(p0), torch.as_tensor(u0 + du)) -
              loss(torch.as_tensor(p0), torch.as_tensor(u0 - du))).item() / (2 * eps)
        assert abs(fd - gu[c, t].item()) <= 1e-6 * max(1.0, abs(fd))


def test_reverb_node_in_a_graph():
    """A reverb node renders through the graph evaluator like any processor."""
    b = synth.GraphBuilder()
    i0 = b.add(synth.IN)
    r = b.add(synth.REVERB)
    o = b.add(synth.OUT)
    b.connect(i0, r)
    b.connect(r, o)
    g = b.build()
    T, L = 1200, 900
    S = synth.make_sources(synth.rng_for(1, 1), 1, T)
    P = synth.draw_params(synth.rng_for(1, 2), g)
    noise = synth.reverb_noise(1, L)
    Y = OR.render(g.node_type, g.edges, S, OR.as_params64(P), reverb_noise=noise)
    ref = RV.reverb(torch.as_tensor(S[0], dtype=F64), torch.as_tensor(P[synth.REVERB][0], dtype=F64),
                    noise)
    assert torch.equal(Y[0], ref)
    with pytest.raises(ValueError):
        OR.render(g.node_type, g.edges, S, OR.as_params64(P))


# ---- delay-time surrogate ----------------------------------------------------------------------

@pytest.mark.parametrize("d", [0, 1, 2205, 4409])
def test_surrogate_is_the_delayed_impulse_on_the_unit_circle(d):
    z = np.exp(-2j * np.pi * d / RV.SLOT)
    s = RV.surrogate(z).numpy()
    ref = np.zeros(RV.SLOT)
    ref[d] = 1.0
    assert np.max(np.abs(s - ref)) < 1e-10  # z^k for k < 4410 as exp(k log z): ~1e-12 rounding


@pytest.mark.parametrize("z", [0.9 * np.exp(-2j * np.pi * 100.4 / 4410), 0.5 + 0.3j, 0.999j])
def test_surrogate_geometric_series(z):
    assert np.max(np.abs(RV.surrogate(z).numpy() - RV.surrogate_closed_form(z))) < 1e-12


def test_surrogate_derivative_against_finite_differences():
    z = 0.95 * np.exp(-2j * np.pi * 777.2 / 4410)
    h = 1e-6
    fd = (RV.surrogate_closed_form(z + h) - RV.surrogate_closed_form(z - h)) / (2 * h)
    fdi = (RV.surrogate_closed_form(z + 1j * h) - RV.surrogate_closed_form(z - 1j * h)) / (2j * h)
    sp = RV.surrogate_deriv(z)
    scale = np.max(np.abs(sp))
    assert np.max(np.abs(fd - sp)) < 1e-6 * scale
    assert np.max(np.abs(fdi - sp)) < 1e-6 * scale  # holomorphic: same derivative along i


def _delay_case(T, seed, unit=True):
    rng = np.random.default_rng(seed)
    p = synth.delay_params(rng, 1)[0].astype(np.float64)
    if not unit:  # phasors pulled inside the disk, angles unchanged
        q = p.reshape(2, 5, 22)
        q[:, :, 0:2] *= 0.97
    u = synth.make_sources(synth.rng_for(seed, 1), 1, T)[0].astype(np.float64)
    w = rng.normal(size=(2, T))
    return p, u, w


def test_straight_through_value_and_non_phasor_gradients_are_exact():
    """With the surrogate the forward value is the exact delay bit for bit, and the gradients of
    the input and of the filter magnitudes are those of the exact delay."""
    p0, u0, w = _delay_case(9000, 11)
    out = {}
    for sur in (False, True):
        p = torch.as_tensor(p0).requires_grad_(True)
        u = torch.as_tensor(u0).requires_grad_(True)
        y = OP.delay(u, p, surrogate=sur)
        gp, gu = torch.autograd.grad(torch.sum(torch.as_tensor(w) * y), [p, u])
        out[sur] = (y.detach().numpy(), gp.numpy().reshape(2, 5, 22), gu.numpy())
    assert np.array_equal(out[False][0], out[True][0])
    assert np.max(np.abs(out[False][1][..., 2:] - out[True][1][..., 2:])) < 1e-12
    assert np.max(np.abs(out[False][2] - out[True][2])) < 1e-12
    assert np.all(out[False][1][..., :2] == 0)
    assert np.max(np.abs(out[True][1][..., :2])) > 0


def test_surrogate_delay_matches_exact_delay_on_the_unit_circle():
    """The delay whose slot impulses are the surrogates equals the exact delay when every phasor
    sits on the unit circle at its integer angle (the surrogate's orientation matches the delay
    the forward pass reads from the phase)."""
    p0, u0, _ = _delay_case(30000, 12)
    # phasors exactly on the circle at the decoded delays (float32-rounded phasors leave
    # |z| - 1 and angle errors of ~1e-7, whose surrogate leaks ~1e-4 off the impulse)
    d = OP.delay_offsets(p0) % RV.SLOT
    q = p0.reshape(2, 5, 22)
    q[:, :, 0] = np.cos(-2.0 * np.pi * d / RV.SLOT)
    q[:, :, 1] = np.sin(-2.0 * np.pi * d / RV.SLOT)
    assert np.array_equal(OP.delay_offsets(p0) % RV.SLOT, d)
    u = torch.as_tensor(u0)
    p = torch.as_tensor(p0)
    ys = OP._delay_surrogate_term(u, p).numpy()
    ye = OP.delay(u, p).numpy()
    assert np.max(np.abs(ys - ye)) < 1e-10 * np.max(np.abs(ye))


def test_surrogate_delay_matches_exact_delay_on_the_unit_circle_2s():
    """The same for the 2 s delay (20 slots): every slot's surrogate is its delayed impulse."""
    rng = np.random.default_rng(14)
    p0 = synth.delay_params(rng, 1, 2000.0, 20)[0].astype(np.float64)
    d = OP.delay_offsets(p0) % RV.SLOT
    q = p0.reshape(2, 20, 22)
    q[:, :, 0] = np.cos(-2.0 * np.pi * d / RV.SLOT)
    q[:, :, 1] = np.sin(-2.0 * np.pi * d / RV.SLOT)
    assert np.array_equal(OP.delay_offsets(p0) % RV.SLOT, d)
    u = torch.as_tensor(synth.make_sources(synth.rng_for(14, 1), 1, 90000)[0].astype(np.float64))
    p = torch.as_tensor(p0)
    ys = OP._delay_surrogate_term(u, p).numpy()
    ye = OP.delay(u, p).numpy()
    assert np.max(np.abs(ys - ye)) < 1e-10 * np.max(np.abs(ye))


@pytest.mark.parametrize("unit", [True, False])
def test_phasor_gradient_against_finite_differences(unit):
    """The straight-through phasor gradient equals central differences of the surrogate delay's
    loss sum(w * y) in Re z and Im z."""
    T = 12000
    p0, u0, w = _delay_case(T, 13, unit)
    wt = torch.as_tensor(w)
    u = torch.as_tensor(u0)
    p = torch.as_tensor(p0).requires_grad_(True)
    g = torch.autograd.grad(torch.sum(wt * OP.delay(u, p, surrogate=True)), p)[0].numpy()
    eps = 1e-6
    for c, m, j in [(0, 0, 0), (0, 2, 1), (1, 4, 0), (1, 1, 1)]:
        i = (c * 5 + m) * 22 + j
        dp = np.zeros(220)
        dp[i] = eps
        lp = torch.sum(wt * OP._delay_surrogate_term(u, torch.as_tensor(p0 + dp))).item()
        lm = torch.sum(wt * OP._delay_surrogate_term(u, torch.as_tensor(p0 - dp))).item()
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (c, m, j, fd, g[i])


def test_unpinned_helpers_behave():
    """Normalisation and the unit-circle penalty (constants not in the paper): unit length,
    zero stays zero; the penalty vanishes on the circle and its gradient matches differences."""
    g = np.array([[3.0, 4.0], [0.0, 0.0]])
    ng = RV.normalise_phasor_grads(g)
    assert np.allclose(ng[0], [0.6, 0.8]) and np.all(ng[1] == 0)
    z = np.array([0.8 + 0.1j, np.exp(0.3j)])
    val, grad = RV.unit_circle_penalty(z, 2.0)
    assert abs(val - 2.0 * (abs(z[0]) - 1) ** 2) < 1e-15
    h = 1e-7
    fd = (RV.unit_circle_penalty(z + h, 2.0)[0] - RV.unit_circle_penalty(z - h, 2.0)[0]) / (2 * h)
    assert abs(fd - grad[:, 0].sum()) < 1e-6
