"""GPU parity at the benchmark's full size: the 64-track mixing console at T = 2^18, in the launch
configuration bench.py times (beam schedule, autograd path, MRSTFT loss against a target mix).

* the whole gradient step (render, loss, adjoint) against the FP64 oracle: output within 1e-5 of
  its peak, loss value, every parameter gradient within 1e-3 of its tensor's largest entry;
* every processed node's row against the single-node oracle fed with the GPU's own input rows
  (so each kernel is checked at full length without error accumulation along the graph).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, RENDER_TOL, grad_err, rel_err, say
from oracle import mrstft as OM
from oracle import render as OR
from paper_2408_03204_amd import Schedule, mrstft_loss, render

pytestmark = pytest.mark.gpu
F64 = torch.float64


@pytest.fixture(scope="module")
def console():
    w = synth.mixing_console(T=2 ** 18)
    sched = Schedule(w.graph.node_type, w.graph.edges, "beam")
    return w, sched


def test_console_full_step_against_oracle(console):
    w, sched = console
    g = w.graph
    say(f"[fullsize step] {w.name} T={w.T} nodes={g.num_nodes}")
    dev = torch.device("cuda")
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev).requires_grad_(True)
         for t, p in w.params.items() if p.shape[0] > 0}
    with torch.no_grad():
        tgt = render(sched, S, {t: torch.as_tensor(p, device=dev)
                                for t, p in w.target_params.items() if p.shape[0] > 0}).clone()
    Y = render(sched, S, P)
    L = mrstft_loss(Y, tgt)
    keys = list(P)
    grads = torch.autograd.grad(L, [P[t] for t in keys])
    torch.cuda.synchronize()
    # oracle: same float32 inputs (target taken from the GPU render, so both sides see the same
    # target), FP64 throughout
    tgt64 = torch.as_tensor(tgt.cpu().numpy(), dtype=F64)
    P64 = OR.as_params64(w.params, requires_grad=True)
    Y64 = OR.render(g.node_type, g.edges, w.sources, P64)
    L64 = OM.mrstft(Y64, tgt64)
    g64 = torch.autograd.grad(L64, [P64[t] for t in keys])
    e_y = rel_err(Y.detach().cpu().numpy().astype(np.float64), Y64.detach().numpy())
    loss, loss64 = float(L.detach()), float(L64.detach())
    say(f"   Y rel err {e_y:.3e}; loss {loss:.8f} vs {loss64:.8f}")
    assert e_y <= RENDER_TOL
    assert abs(loss - loss64) <= 1e-5 * abs(loss64)
    for t, a, b in zip(keys, grads, g64):
        e = grad_err(a.cpu().numpy(), b.numpy())
        say(f"   dP[{t}] rel err {e:.3e}")
        assert e <= GRAD_TOL, (t, e)


def test_console_every_node_locally(console):
    w, sched = console
    g = w.graph
    say("[fullsize nodes] local single-node parity for every processed node")
    dev = torch.device("cuda")
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    with torch.no_grad():
        _, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    Uh = U.cpu().numpy()
    rows = OR.param_rows(g.node_type)
    P64 = OR.as_params64(w.params)
    pos = np.empty(g.num_nodes, dtype=np.int64)
    pos[sched.perm] = np.arange(g.num_nodes)
    in_edges = [[] for _ in range(g.num_nodes)]
    for e in range(g.num_edges):
        in_edges[int(g.edges[1, e])].append(int(g.edges[0, e]))
    worst = {}
    for v in range(g.num_nodes):
        t = int(g.node_type[v])
        if t == synth.IN:
            continue
        u = torch.zeros((2, w.T), dtype=F64)
        for s in in_edges[v]:
            src = w.sources[rows[s]] if g.node_type[s] == synth.IN else Uh[pos[s]]
            u = u + torch.as_tensor(src, dtype=F64)
        p = P64[t][rows[v]] if t in P64 else None
        y64 = OR.node_forward(t, u, p).numpy()
        e = rel_err(Uh[pos[v]].astype(np.float64), y64)
        worst[t] = max(worst.get(t, 0.0), e)
        assert e <= RENDER_TOL, (v, t, e)
    say("   worst per type", {synth.TYPE_NAMES[k]: f"{x:.2e}" for k, x in worst.items()})
