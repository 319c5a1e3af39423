"""GPU parity of processors with no incoming edge and of processors whose output no node reads,
against the FP64 oracle, for every processor type. A node without inputs processes a zero signal
(paper Eq. 1: its input is an empty sum), and a node without consumers receives a zero output
adjoint, so its parameters get zero gradients. These are the rows for which the kernels' gathers
find no edge at all (the transforms' and the dynamics' first-row paths, the delay's and the
reverb's staging). The tolerances are the render's (1e-5 of the peak output) and the gradients'
(1e-3 of each parameter column's largest entry)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, RENDER_TOL, grad_err, rel_err, say
from oracle import render as OR
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

F64 = torch.float64
TYPES = (synth.MIX, synth.GAIN_PAN, synth.EQ, synth.COMP, synth.IMAGER, synth.DELAY, synth.TANH,
         synth.GATE, synth.COMP_AR, synth.REVERB, synth.DELAY_LONG)


def unconnected_graph(T, seed, noise_len):
    """Per type: one node without inputs feeding the output and one node fed by an input whose
    output nobody reads; a gain on the first input and the second input straight to the output
    keep the output non-trivial."""
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    o = b.add(synth.OUT)
    gp = b.add(synth.GAIN_PAN)
    b.connect(i0, gp)
    b.connect(gp, o)
    b.connect(i1, o)
    for t in TYPES:
        orphan, dangling = b.add(t), b.add(t)
        b.connect(orphan, o)
        b.connect(i0, dangling)
    g = b.build()
    w = synth.Workload("unconnected", g, synth.make_sources(synth.rng_for(seed, 1), 2, T),
                       synth.draw_params(synth.rng_for(seed, 2), g), None, T, seed)
    return w, synth.reverb_noise(seed, noise_len)


def oracle(w, noise, dY):
    g = w.graph
    S = torch.as_tensor(w.sources, dtype=F64).requires_grad_(True)
    P = OR.as_params64(w.params, requires_grad=True)
    Y = OR.render(g.node_type, g.edges, S, P, reverb_noise=noise)
    keys = [t for t in sorted(P) if P[t].shape[0] > 0]
    gr = torch.autograd.grad((Y * torch.as_tensor(dY, dtype=F64)).sum(), [S] + [P[t] for t in keys],
                             allow_unused=True)
    out = {"S": gr[0].numpy()}
    for t, x in zip(keys, gr[1:]):
        out[t] = np.zeros(tuple(P[t].shape)) if x is None else x.detach().numpy()
    return Y.detach().numpy(), out


@pytest.mark.parametrize("T", [3 * 2048 + 555, 2 ** 14])
def test_unconnected_processors(T):
    say(f"[unconnected] every type, T={T}")
    w, noise = unconnected_graph(T, 71, 5000)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    sched.set_reverb_noise(torch.as_tensor(noise).cuda())
    S = torch.as_tensor(w.sources).cuda().requires_grad_(True)
    P = {t: torch.as_tensor(p).cuda().requires_grad_(True) for t, p in w.params.items()
         if p.shape[0] > 0}
    Y = render(sched, S, P)
    dY = np.random.default_rng(72).normal(size=tuple(Y.shape)).astype(np.float32)
    Y.backward(torch.as_tensor(dY).cuda())
    torch.cuda.synchronize()
    Yr, ref = oracle(w, noise, dY)
    Yh = Y.detach().cpu().numpy().astype(np.float64)
    errs = {"Y": max(rel_err(Yh[k], Yr[k]) for k in range(Yh.shape[0])),
            "S": grad_err(S.grad.cpu().numpy(), ref["S"])}
    for t, p in P.items():
        errs[synth.TYPE_NAMES[t]] = grad_err(p.grad.cpu().numpy(), ref[t])
    say("   errs", {k: f"{e:.2e}" for k, e in errs.items()})
    g = w.graph
    assert errs["Y"] <= RENDER_TOL, errs
    for k, e in errs.items():
        if k != "Y":
            assert e <= GRAD_TOL, (k, e)
    # every node's own output row, those nobody reads included
    with torch.no_grad():
        _, U = render(sched, S.detach(), {t: p.detach() for t, p in P.items()}, return_U=True)
        _, ys = OR.render(g.node_type, g.edges, w.sources, OR.as_params64(w.params), keep_all=True,
                          reverb_noise=noise)
    torch.cuda.synchronize()
    K = sched.num_inputs
    Uh = U[K:].cpu().numpy().astype(np.float64)  # the input rows are never written
    for i in range(K, sched.num_nodes):
        v = int(sched.perm[i])
        e = rel_err(Uh[i - K], ys[v].numpy())
        assert e <= RENDER_TOL, (v, synth.TYPE_NAMES[g.node_type[v]], e)
    # rows of the nodes nobody reads get exactly zero parameter gradients
    for t, p in P.items():
        nodes = [v for v in range(g.num_nodes) if g.node_type[v] == t]
        consumers = set(int(s) for s in g.edges[0])
        rows = [r for r, v in enumerate(nodes) if v not in consumers]
        assert rows, t
        assert np.all(p.grad.cpu().numpy()[rows] == 0.0), synth.TYPE_NAMES[t]
