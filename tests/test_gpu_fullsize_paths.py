"""GPU parity on the code paths that only full-size signals reach.

* Multitap delay (Eq. 14, five 100 ms slots): at T >= 2^16 every slot, including delays of
  17,640-22,049 samples, lands inside the signal, and the tap-gradient reduction runs over several
  8-tile groups. Forward, input adjoint and tap gradients against the FP64 oracle.
* Attack/release compressors (Eq. 8 unrestricted) on the 64-track console at T = 2^18 (86 chunks
  per node, several branch-pattern passes): every node's output, input adjoint and parameter
  gradients against the single-node oracle (the literal per-sample loop) fed with the GPU's rows,
  with the default pass limit and with the pass limit lowered to 2 (most chunks then take the
  serial fallback). Also reports how many passes the console needs: the smallest pass limit whose
  render is bit-identical to the default one.
* The 128-graph batch at full size (per-graph T in {2^16, 2^17, 2^18}, merged into one schedule):
  one render and one adjoint of a seeded output adjoint, and for a fixed sample of graphs (each
  with delays and tanh nodes, one per length) the outputs, source adjoints and parameter
  gradients against the whole-graph FP64 oracle.
"""
import concurrent.futures
import functools
import os

import numpy as np
import pytest
import torch

import synth
from gpu_common import (GRAD_TOL, RENDER_TOL, check_nodes_locally, fmt_worst, grad_err,
                        oracle_grads, rel_err, say)
from oracle import processors as OP
from oracle import render as OR
from paper_2408_03204_amd import RenderBuffers, Schedule, merge_graphs, merge_inputs

pytestmark = pytest.mark.gpu
F64 = torch.float64


def delay_graph(T, seed):
    """Three delay nodes in one step, fed by different source sums, into a mix."""
    b = synth.GraphBuilder()
    i0, i1, i2 = b.add(synth.IN), b.add(synth.IN), b.add(synth.IN)
    d = [b.add(synth.DELAY) for _ in range(3)]
    m = b.add(synth.MIX)
    o = b.add(synth.OUT)
    for s, n in ((i0, d[0]), (i1, d[0]), (i1, d[1]), (i2, d[2]), (i0, d[2])):
        b.connect(s, n)
    for n in d:
        b.connect(n, m)
    b.connect(m, o)
    b.connect(d[1], o)
    g = b.build()
    return synth.Workload("delays", g, synth.make_sources(synth.rng_for(seed, 1), 3, T),
                          synth.draw_params(synth.rng_for(seed, 2), g), None, T, seed)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("T", [2 ** 16 + 1234, 2 ** 18])
def test_delay_full_length(T):
    w = delay_graph(T, 91)
    offs = np.stack([OP.delay_offsets(p) for p in w.params[synth.DELAY]])
    say(f"[delay full] T={T} delays {offs.min()}..{offs.max()} samples")
    # every slot of every node lands inside the signal, the last slot beyond 17,640 samples
    assert offs.max() + 19 < T and (offs[:, :, 4] >= 4 * 4410).all()
    sched = Schedule(w.graph.node_type, w.graph.edges)
    dev = torch.device("cuda")
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    rb = RenderBuffers(sched, T, dev, with_backward=True)
    rb.forward(S, P)
    dY = np.random.default_rng(17).standard_normal((sched.num_outputs, 2, T)).astype(np.float32)
    dP = {t: torch.empty_like(p) for t, p in P.items()}
    dS = torch.zeros_like(S)
    rb.backward(S, P, torch.as_tensor(dY, device=dev), dP, dS=dS)
    torch.cuda.synchronize()
    Uh, dUh = rb.U.cpu().numpy(), rb.dU.cpu().numpy()
    worst = check_nodes_locally(w, sched, Uh, dUh, dY, {t: d.cpu().numpy() for t, d in dP.items()})
    say("   local worst (y, ubar, dp):", fmt_worst(worst))
    # whole graph: outputs, source adjoint and tap gradients against FP64 autograd
    Y64 = OR.render(w.graph.node_type, w.graph.edges, w.sources, OR.as_params64(w.params))
    e_y = rel_err(rb.Y.cpu().numpy().astype(np.float64), Y64.numpy())
    ref = oracle_grads(w, dY)
    e_s = grad_err(dS.cpu().numpy(), ref["S"])
    e_p = grad_err(dP[synth.DELAY].cpu().numpy(), ref[synth.DELAY])
    say(f"   whole graph: Y {e_y:.2e}, dS {e_s:.2e}, dP[delay] {e_p:.2e}")
    assert e_y <= RENDER_TOL and e_s <= GRAD_TOL and e_p <= GRAD_TOL
    # the tap gradients are not trivially small: every slot's taps see the signal
    g = np.abs(ref[synth.DELAY].reshape(3, 2, 5, 22)[..., 2:]).max(axis=-1)
    assert (g > 1e-3 * g.max()).all()


@pytest.fixture(scope="module")
def console_ar():
    w = synth.mixing_console(T=2 ** 18, attack_release=True)
    return w, Schedule(w.graph.node_type, w.graph.edges, "beam")


def _render_and_adjoint(w, sched, passes=None):
    dev = torch.device("cuda")
    if passes is not None:
        sched.set_tuning(Schedule.TUNE_AR_MAX_PASSES, passes)
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    rb = RenderBuffers(sched, w.T, dev, with_backward=True)
    rb.forward(S, P)
    dY = np.random.default_rng(23).standard_normal(
        (sched.num_outputs, 2, w.T)).astype(np.float32)
    dP = {t: torch.empty_like(p) for t, p in P.items()}
    rb.backward(S, P, torch.as_tensor(dY, device=dev), dP)
    torch.cuda.synchronize()
    assert rb.error_word() == 0
    out = (rb.U.cpu().numpy(), rb.dU.cpu().numpy(), dY, {t: d.cpu().numpy() for t, d in dP.items()})
    sched.set_tuning(Schedule.TUNE_AR_MAX_PASSES, 16)
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("passes", [16, 2])
def test_console_ar_every_node_full_length(console_ar, passes):
    w, sched = console_ar
    n_ar = int((w.graph.node_type == synth.COMP_AR).sum())
    say(f"[console_ar full] T={w.T}, {n_ar} attack/release compressors, pass limit {passes}")
    Uh, dUh, dY, dP = _render_and_adjoint(w, sched, passes)
    types = None if passes == 16 else {synth.COMP_AR}
    worst = check_nodes_locally(w, sched, Uh, dUh, dY, dP, types=types, log_every=40)
    say("   worst (y, ubar, dp):", fmt_worst(worst))


def test_console_ar_passes_needed(console_ar):
    w, sched = console_ar
    dev = torch.device("cuda")
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    rb = RenderBuffers(sched, w.T, dev, with_backward=False)
    rb.forward(S, P)
    ref = rb.Y.clone()
    need = None
    for k in range(1, 17):
        sched.set_tuning(Schedule.TUNE_AR_MAX_PASSES, k)
        rb.forward(S, P)
        if torch.equal(rb.Y, ref):
            need = k
            break
    sched.set_tuning(Schedule.TUNE_AR_MAX_PASSES, 16)
    torch.cuda.synchronize()
    say(f"[console_ar passes] smallest pass limit with the default bits: {need}")
    assert need is not None and need <= 16


SAMPLE = (84, 102, 120)  # one graph per length (2^16, 2^17, 2^18), each with delay and tanh nodes


@pytest.fixture(scope="module")
def batch():
    workers = min(16, os.cpu_count() or 1)
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers) as ex:
        ws = list(ex.map(functools.partial(synth.batched_graph, 7), range(128)))
    return ws


@pytest.mark.timeout(900)
def test_batch_full_size_sampled_graphs(batch):
    ws = batch
    m = merge_graphs([(w.graph.node_type, w.graph.edges, w.T) for w in ws])
    say(f"[batch full] 128 graphs, {len(m['node_type'])} nodes, stride {m['T']}")
    S_h, P_h = merge_inputs(m, [w.sources for w in ws], [w.params for w in ws])
    sched = Schedule(m["node_type"], m["edges"], "beam", lengths=m["lengths"])
    dev = torch.device("cuda")
    S = torch.as_tensor(S_h, device=dev)
    del S_h
    P = {t: torch.as_tensor(p, device=dev) for t, p in P_h.items()}
    T = m["T"]
    rng = np.random.default_rng(29)
    dY = torch.zeros((sched.num_outputs, 2, T), dtype=torch.float32, device=dev)
    dY_g = {}
    for i, w in enumerate(ws):
        n_out, o0 = w.graph.count(synth.OUT), m["output_offset"][i]
        d = rng.standard_normal((n_out, 2, w.T)).astype(np.float32)
        if i in SAMPLE:
            dY_g[i] = d
        dY[o0:o0 + n_out, :, :w.T] = torch.as_tensor(d, device=dev)
    rb = RenderBuffers(sched, T, dev, with_backward=True)
    rb.forward(S, P)
    dP = {t: torch.empty_like(p) for t, p in P.items()}
    dS = torch.zeros_like(S)
    rb.backward(S, P, dY, dP, dS=dS)
    torch.cuda.synchronize()
    assert rb.error_word() == 0
    say("   merged render and adjoint done")
    for i in SAMPLE:
        w = ws[i]
        g = w.graph
        nt = g.node_type
        assert (nt == synth.DELAY).any() and (nt == synth.TANH).any()
        n_out, o0, k0 = g.count(synth.OUT), m["output_offset"][i], m["input_offset"][i]
        K = g.count(synth.IN)
        Y = rb.Y[o0:o0 + n_out, :, :w.T].cpu().numpy().astype(np.float64)
        Y64 = OR.render(nt, g.edges, w.sources, OR.as_params64(w.params)).numpy()
        e_y = rel_err(Y, Y64)
        ref = oracle_grads(w, dY_g[i])
        e_s = grad_err(dS[k0:k0 + K, :, :w.T].cpu().numpy(), ref["S"])
        errs = {}
        for t, r in ref.items():
            if t == "S":
                continue
            r0 = int(m["param_offset"][i][t])
            errs[synth.TYPE_NAMES[t]] = grad_err(dP[t][r0:r0 + r.shape[0]].cpu().numpy(), r)
        say(f"   graph {i} (T={w.T}, {g.num_nodes} nodes): Y {e_y:.2e}, dS {e_s:.2e}, dP",
            {k: f"{e:.1e}" for k, e in errs.items()})
        assert e_y <= RENDER_TOL, (i, e_y)
        assert e_s <= GRAD_TOL, (i, e_s)
        for k, e in errs.items():
            assert e <= GRAD_TOL, (i, k, e)
