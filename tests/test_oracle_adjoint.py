"""Pins of the hand-written FP64 adjoints (`oracle.adjoint`) and of the streamed renderer
(`oracle.streamed`): each processor's adjoint equals torch autograd through its forward
definition (paper Eqs. 2-5, 8-12, 14; the noisegate of Sec. 3; tanh), on random inputs that
reach every branch of the gain curves; the streamed forward equals the node-by-node renderer bit
for bit, and the streamed adjoint equals autograd through the whole graph."""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as A
from oracle import processors as P
from oracle import render as R
from oracle import streamed as ST

F64 = torch.float64
TOL = 1e-10


def _autograd(fn, u, p, ybar):
    u = u.clone().requires_grad_(True)
    wrt = [u]
    if p is not None:
        p = p.clone().requires_grad_(True)
        wrt.append(p)
    y = fn(u, p)
    g = torch.autograd.grad(y, wrt, ybar, allow_unused=True)
    gp = None
    if p is not None:
        gp = g[1] if g[1] is not None else torch.zeros_like(p)
    return g[0], gp


def _close(a, b):
    scale = max(float(b.abs().max()), 1e-300)
    return float((a - b).abs().max()) / scale


def _signal(rng, T, level=0.3):
    env = np.exp(-np.arange(T) / (0.3 * T))[None, :]
    return torch.as_tensor(rng.uniform(-1, 1, (2, T)) * level * env, dtype=F64)


@pytest.mark.parametrize("seed", range(3))
def test_pointwise_adjoints_equal_autograd(seed):
    rng = np.random.default_rng(seed)
    T = 1500
    u, ybar = _signal(rng, T), torch.as_tensor(rng.standard_normal((2, T)), dtype=F64)
    for fn, adj, p in ((P.gain_pan, A.gain_pan, rng.uniform(-1, 1, 2)),
                       (P.imager, A.imager, rng.uniform(-1, 1, 1)),
                       (P.tanh_dist, A.tanh_dist, rng.uniform(0, 2.5, 1))):
        p = torch.as_tensor(p, dtype=F64)
        gu, gp = _autograd(fn, u, p, ybar)
        hu, hp = adj(u, p, ybar)
        assert _close(hu, gu) <= TOL and _close(hp, gp) <= TOL, fn.__name__


@pytest.mark.parametrize("T", [700, 5000])
def test_eq_adjoint_equals_autograd(T):
    rng = np.random.default_rng(T)
    u, ybar = _signal(rng, T), torch.as_tensor(rng.standard_normal((2, T)), dtype=F64)
    p = torch.as_tensor(synth.eq_params(rng, 1)[0], dtype=F64)
    gu, gp = _autograd(P.eq, u, p, ybar)
    hu, hp = A.eq(u, p, ybar)
    assert _close(hu, gu) <= TOL
    assert _close(hp, gp) <= TOL


def _dyn_params(rng, gate, knee):
    a = float(np.exp(-1.0 / (rng.uniform(1, 5) * 1e-3 * 44100)))
    if gate:
        return torch.tensor([a, np.log(10) / 10 * -25, knee, 4.0], dtype=F64)
    return torch.tensor([a, np.log(10) / 10 * -18, knee, 4.0], dtype=F64)


@pytest.mark.parametrize("gate", [False, True])
@pytest.mark.parametrize("knee", [0.0, 1.5])
def test_dynamics_adjoints_equal_autograd(gate, knee):
    """Ramped sources so that the envelope crosses below, inside and above the knee."""
    rng = np.random.default_rng(7 + int(gate))
    T = 6000
    ramp = np.logspace(-3.5, 0, T)[None, :]
    u = torch.as_tensor(rng.uniform(-1, 1, (2, T)) * 0.5 * ramp, dtype=F64)
    ybar = torch.as_tensor(rng.standard_normal((2, T)), dtype=F64)
    p = _dyn_params(rng, gate, knee)
    fwd, adj = (P.noisegate, A.noisegate) if gate else (P.compressor, A.compressor)
    x = (u[0] + u[1]) ** 2
    Gu = torch.log(P.one_pole(x, p[0]) + P.EPS_ENV)
    lo, hi = float(p[1] - max(knee, 1e-9)), float(p[1] + knee)
    assert (Gu < lo).any() and (Gu >= hi).any()  # both outer regions are reached
    if knee > 0:
        assert ((Gu >= lo) & (Gu < hi)).any()
    gu, gp = _autograd(fwd, u, p, ybar)
    hu, hp = adj(u, p, ybar)
    assert _close(hu, gu) <= TOL
    for j in range(4):
        if float(gp[j].abs()) == 0.0:
            assert float(hp[j].abs()) == 0.0
        else:
            assert abs(float(hp[j] - gp[j])) <= TOL * abs(float(gp[j])) * 10, j


@pytest.mark.parametrize("slots,T", [(5, 23000), (20, 89000)])
def test_delay_adjoint_equals_autograd(slots, T):
    rng = np.random.default_rng(3)
    u, ybar = _signal(rng, T), torch.as_tensor(rng.standard_normal((2, T)), dtype=F64)
    p = torch.as_tensor(synth.delay_params(rng, 1, 100.0 * slots, slots)[0], dtype=F64)
    assert P.delay_offsets(p.numpy()).max() + 20 < T
    gu, gp = _autograd(P.delay, u, p, ybar)
    hu, hp = A.delay(u, p, ybar)
    assert _close(hu, gu) <= TOL
    assert _close(hp, gp) <= TOL


def _check_streamed(w, seed):
    g = w.graph
    Y0 = R.render(g.node_type, g.edges, w.sources, R.as_params64(w.params))
    Yf = ST.render_and_adjoint(g.node_type, g.edges, w.sources, w.params)
    assert torch.equal(Y0, Yf)  # same arithmetic, same order
    dY = np.random.default_rng(seed).standard_normal(tuple(Y0.shape))
    Ys, dS, dP = ST.render_and_adjoint(g.node_type, g.edges, w.sources, w.params, dY)
    assert torch.equal(Ys, Y0)
    S = torch.as_tensor(w.sources, dtype=F64).requires_grad_(True)
    P64 = R.as_params64(w.params, requires_grad=True)
    L = (R.render(g.node_type, g.edges, S, P64) * torch.as_tensor(dY, dtype=F64)).sum()
    keys = [t for t in sorted(P64) if P64[t].shape[0] > 0]
    gr = torch.autograd.grad(L, [S] + [P64[t] for t in keys], allow_unused=True)
    assert _close(dS, gr[0]) <= TOL
    for t, ref in zip(keys, gr[1:]):
        ref = torch.zeros_like(P64[t]) if ref is None else ref
        for j in range(ref.shape[1]):
            scale = float(ref[:, j].abs().max())
            err = float((dP[t][:, j] - ref[:, j]).abs().max())
            assert err <= TOL * max(scale, float(ref.abs().max()) * 1e-6), (t, j, err, scale)


@pytest.mark.parametrize("seed", range(4))
def test_streamed_equals_autograd_random_dags(seed):
    types = (synth.MIX, synth.GAIN_PAN, synth.EQ, synth.COMP, synth.IMAGER, synth.TANH,
             synth.GATE)
    w = synth.random_workload(900 + seed, 12, 3000 + 517 * seed, types=types, edge_p=0.35,
                              n_out=1 + seed % 2)
    _check_streamed(w, seed)


def test_streamed_equals_autograd_with_delays():
    w = synth.random_workload(950, 8, 23500, types=(synth.MIX, synth.DELAY, synth.GAIN_PAN),
                              edge_p=0.4)
    assert (w.graph.node_type == synth.DELAY).any()
    _check_streamed(w, 1)


def test_streamed_equals_autograd_console():
    _check_streamed(synth.mixing_console(T=4096, n_tracks=16, n_bus=4), 2)


def test_streamed_forward_frees_intermediate_outputs():
    """Without an adjoint, the forward keeps only what later nodes still read (checked through
    the result only: it must still equal the renderer's)."""
    w = synth.tiny_console(T=2048)
    g = w.graph
    Y0 = R.render(g.node_type, g.edges, w.sources, R.as_params64(w.params))
    assert torch.equal(ST.render_and_adjoint(g.node_type, g.edges, w.sources, w.params), Y0)
