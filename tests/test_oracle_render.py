"""Pins of the oracle renderer (paper Sec. 2 "Definitions", Eq. 1) and of the MRSTFT loss:
path-sum closed forms, topological-order invariance, finite-difference gradients."""
import itertools
import math

import numpy as np
import pytest
import torch

import synth
from oracle import mrstft as M
from oracle import render as R

F64 = torch.float64


def _paths(graph, src):
    """All edge paths from node `src` to each output node (parallel edges counted)."""
    succ = [[] for _ in range(graph.num_nodes)]
    for s, d in graph.edges.T:
        succ[int(s)].append(int(d))
    out = []

    def rec(v, path):
        if graph.node_type[v] == synth.OUT:
            out.append(path + [v])
            return
        for w in succ[v]:
            rec(w, path + [v])

    rec(src, [])
    return out


@pytest.mark.parametrize("seed", range(12))
def test_gain_pan_graph_equals_path_sum(seed):
    w = synth.random_workload(seed, int(np.random.default_rng(seed).integers(5, 12)), T=64,
                              types=(synth.MIX, synth.GAIN_PAN), edge_p=0.4,
                              n_out=1 + seed % 2)
    g = w.graph
    Y = R.render(g.node_type, g.edges, w.sources, R.as_params64(w.params)).numpy()
    rows = R.param_rows(g.node_type)
    outs = [v for v in range(g.num_nodes) if g.node_type[v] == synth.OUT]
    expect = np.zeros_like(Y)
    for v in range(g.num_nodes):
        if g.node_type[v] != synth.IN:
            continue
        for path in _paths(g, v):
            gain = np.ones(2)
            for n in path:
                if g.node_type[n] == synth.GAIN_PAN:
                    gain = gain * np.exp(w.params[synth.GAIN_PAN][rows[n]].astype(np.float64))
            expect[outs.index(path[-1])] += gain[:, None] * w.sources[rows[v]]
    assert np.max(np.abs(Y - expect)) <= 1e-13 * max(1.0, np.max(np.abs(expect)))


@pytest.mark.parametrize("seed", range(6))
def test_gain_imager_graph_equals_matrix_path_sum(seed):
    w = synth.random_workload(50 + seed, 9, T=48, types=(synth.MIX, synth.GAIN_PAN, synth.IMAGER),
                              edge_p=0.4)
    g = w.graph
    Y = R.render(g.node_type, g.edges, w.sources, R.as_params64(w.params)).numpy()
    rows = R.param_rows(g.node_type)
    expect = np.zeros_like(Y)
    for v in np.flatnonzero(g.node_type == synth.IN):
        for path in _paths(g, int(v)):
            Mx = np.eye(2)
            for n in path:
                t = g.node_type[n]
                if t == synth.GAIN_PAN:
                    Mx = np.diag(np.exp(w.params[t][rows[n]].astype(np.float64))) @ Mx
                elif t == synth.IMAGER:
                    e = math.exp(float(w.params[t][rows[n]][0]))
                    Mx = 0.5 * np.array([[1 + e, 1 - e], [1 - e, 1 + e]]) @ Mx
            expect[0] += Mx @ w.sources[rows[int(v)]]
    assert np.max(np.abs(Y - expect)) <= 1e-13 * max(1.0, np.max(np.abs(expect)))


def _all_topo_orders(g, limit=200):
    V = g.num_nodes
    preds = [set() for _ in range(V)]
    for s, d in g.edges.T:
        preds[int(d)].add(int(s))
    out = []

    def rec(done, order):
        if len(out) >= limit:
            return
        if len(order) == V:
            out.append(list(order))
            return
        for v in range(V):
            if v not in done and preds[v] <= done:
                rec(done | {v}, order + [v])

    rec(set(), [])
    return out


@pytest.mark.parametrize("seed", range(3))
def test_every_topological_order_is_bit_identical(seed):
    w = synth.random_workload(70 + seed, 7, T=3000, edge_p=0.45)
    g = w.graph
    p = R.as_params64(w.params)
    ref = R.render(g.node_type, g.edges, w.sources, p)
    orders = _all_topo_orders(g, limit=30)
    assert len(orders) > 1
    for order in orders:
        assert torch.equal(R.render(g.node_type, g.edges, w.sources, p, order=order), ref)


def _directional_check(fn, tensors, seed, eps=1e-6, rtol=2e-5, scales=None):
    """Central finite difference along random directions vs autograd. `scales` (optional, one
    per tensor) shrinks the direction where the loss is strongly curved."""
    rng = np.random.default_rng(seed)
    loss = fn(*tensors)
    grads = torch.autograd.grad(loss, tensors, allow_unused=True)
    grads = [torch.zeros_like(t) if g is None else g for t, g in zip(tensors, grads)]
    scales = scales or [1.0] * len(tensors)
    for _ in range(3):
        dirs = [torch.as_tensor(rng.normal(size=t.shape), dtype=F64) * sc
                for t, sc in zip(tensors, scales)]
        with torch.no_grad():
            lp = fn(*[t + eps * d for t, d in zip(tensors, dirs)])
            lm = fn(*[t - eps * d for t, d in zip(tensors, dirs)])
        fd = float(lp - lm) / (2 * eps)
        an = sum(float((g * d).sum()) for g, d in zip(grads, dirs))
        assert abs(fd - an) <= rtol * max(1.0, abs(an)), (fd, an)


GATE_TYPES = (synth.MIX, synth.GAIN_PAN, synth.EQ, synth.COMP, synth.GATE, synth.IMAGER, synth.TANH)
AR_TYPES = (synth.MIX, synth.GAIN_PAN, synth.EQ, synth.COMP_AR, synth.IMAGER, synth.TANH)


@pytest.mark.parametrize("seed", range(8))
def test_render_gradients_match_finite_differences(seed):
    # cases 4 and 5 draw graphs with noisegates (seeds 105, 115: 3 and 2 of them), cases 6 and 7
    # graphs with attack/release compressors (seeds 131, 138: 4 and 3 of them)
    if seed < 4:
        w = synth.random_workload(90 + seed, 9, T=5000, edge_p=0.35)
    elif seed < 6:
        w = synth.random_workload((105, 115)[seed - 4], 9, T=5000, edge_p=0.35, types=GATE_TYPES)
        assert w.graph.count(synth.GATE) >= 2
    else:
        w = synth.random_workload((131, 138)[seed - 6], 9, T=5000, edge_p=0.35, types=AR_TYPES)
        assert w.graph.count(synth.COMP_AR) >= 3
    g = w.graph
    types = sorted(t for t in w.params if w.params[t].shape[0] > 0)
    # the delay's offsets are piecewise constant in z: keep them out of the perturbation
    S = torch.as_tensor(w.sources, dtype=F64).requires_grad_(True)
    weights = torch.as_tensor(np.random.default_rng(seed).normal(size=(g.count(synth.OUT), 2, w.T)))
    ps = [torch.as_tensor(w.params[t], dtype=F64).requires_grad_(True) for t in types]
    mask = {t: torch.ones_like(p) for t, p in zip(types, ps)}
    if synth.DELAY in mask:
        mask[synth.DELAY].reshape(-1, 2, 5, 22)[..., :2] = 0

    def fn(S_, *ps_):
        pd = {t: ps[i] + (ps_[i] - ps[i]) * mask[t] for i, t in enumerate(types)}
        pd.update({t: torch.as_tensor(w.params[t], dtype=F64) for t in w.params if t not in pd})
        return (R.render(g.node_type, g.edges, S_, pd) * weights).sum()

    # the compressor's alpha sits near 1 where the output is strongly curved in it
    scales = [1.0] + [torch.tensor([1e-2, 1, 1, 1], dtype=F64) if t in (synth.COMP, synth.GATE)
                      else torch.tensor([1e-2, 1e-2, 1, 1, 1], dtype=F64) if t == synth.COMP_AR
                      else 1.0 for t in types]
    _directional_check(fn, [S] + ps, seed, scales=scales)


def test_mrstft_zero_for_equal_and_frame_dft():
    rng = np.random.default_rng(20)
    y = torch.as_tensor(rng.normal(size=(1, 2, 6000)))
    assert float(M.mrstft(y, y)) == 0.0
    S = M.stft_mag(y, 512)
    f, k = 3, 17
    n = np.arange(512)
    w = 0.5 - 0.5 * np.cos(2 * np.pi * n / 512)
    seg = y[0, 1, f * 128:f * 128 + 512].numpy()
    X = np.sum(w * seg * np.exp(-2j * np.pi * k * n / 512))
    assert abs(float(S[0, 1, f, k]) - math.sqrt(abs(X) ** 2 + 1e-8)) < 1e-10
    assert S.shape[-2] == (6000 - 512) // 128 + 1


def test_mrstft_spectral_convergence_scale():
    # y = c * t with |t| large: every magnitude scales by c (the 1e-8 floor is negligible), so
    # SC = |c - 1| and LM = |ln c| for every resolution
    rng = np.random.default_rng(21)
    t = torch.as_tensor(rng.normal(size=(1, 2, 9000))) * 100
    for c in (0.5, 2.0):
        L = float(M.mrstft(c * t, t))
        assert abs(L - (abs(c - 1) + abs(math.log(c)))) < 1e-9


def test_mrstft_gradient_fd():
    rng = np.random.default_rng(22)
    t = torch.as_tensor(rng.normal(size=(1, 2, 3000)))
    y = (t + 0.3 * torch.as_tensor(rng.normal(size=(1, 2, 3000)))).requires_grad_(True)
    _directional_check(lambda a: M.mrstft(a, t), [y], 23, eps=1e-6, rtol=1e-4)
