"""GPU parity of the noisegate (paper Sec. 3 "Noisegate": the compressor's envelope with a
downward-expander curve) against the FP64 oracle, forward and adjoint. The sources fall from
0 dB to -90 dB along the signal so that the gate's envelope crosses all three regions of its
curve (above the knee, inside it, below it); graphs that mix compressors and noisegates check
that the two types keep apart in their shared chunk state. The one-pole envelope cannot fall
faster than its own time constant allows, so the gates here get short ones (2-5 ms)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, check_render, device_inputs, grad_err, oracle_grads, say
from oracle import processors as OP
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

T_RAGGED = [3 * 2048 + 555, 4 * 3072 + 1024 + 4]


def ramped(sources: np.ndarray, top_db=0.0, bottom_db=-90.0) -> np.ndarray:
    T = sources.shape[-1]
    ramp = 10.0 ** (np.linspace(top_db, bottom_db, T) / 20.0)
    return (sources * ramp[None, None, :]).astype(np.float32)


def short_alpha(n):
    tau = np.linspace(2e-3, 5e-3, n)
    return np.exp(-1.0 / (tau * synth.FS)).astype(np.float32)


def gate_workload(T, seed, knee_db=3.0):
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    n = b.add(synth.GATE)
    o = b.add(synth.OUT)
    b.connect(i0, n)
    b.connect(i1, n)
    b.connect(i0, n)
    b.connect(n, o)
    g = b.build()
    S = ramped(synth.make_sources(synth.rng_for(seed, 1), 2, T))
    P = synth.draw_params(synth.rng_for(seed, 2), g)
    P[synth.GATE][:, 2] = knee_db * synth.LN10_10
    P[synth.GATE][:, 0] = short_alpha(1)
    return synth.Workload("single_gate", g, S, P, None, T, seed)


def regions(w):
    """Samples of the single gate's envelope below, inside and above the knee (oracle FP64)."""
    S = torch.as_tensor(w.sources, dtype=torch.float64)
    u = S[0] + S[1] + S[0]
    p = torch.as_tensor(w.params[synth.GATE][0], dtype=torch.float64)
    Gu = torch.log(OP.one_pole((u[0] + u[1]) ** 2, p[0]) + OP.EPS_ENV)
    thr, knee = float(p[1]), float(p[2])
    lo, hi = thr - max(knee, 0.0), thr + max(knee, 0.0)
    return int((Gu < lo).sum()), int(((Gu >= lo) & (Gu < hi)).sum()), int((Gu >= hi).sum())


def run_backward(w, seed):
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    S.requires_grad_(True)
    for p in P.values():
        p.requires_grad_(True)
    Y = render(sched, S, P)
    dY = np.random.default_rng(seed).normal(size=tuple(Y.shape)).astype(np.float32)
    Y.backward(torch.as_tensor(dY).cuda())
    torch.cuda.synchronize()
    ref = oracle_grads(w, dY)
    errs = {"S": grad_err(S.grad.cpu().numpy(), ref["S"])}
    for t, p in P.items():
        errs[t] = grad_err(p.grad.cpu().numpy(), ref[t])
    return errs


@pytest.mark.parametrize("knee_db", [3.0, 0.0])
@pytest.mark.parametrize("T", T_RAGGED)
def test_gate_forward(T, knee_db):
    say(f"[gate fwd] T={T} knee={knee_db} dB")
    w = gate_workload(T, 41, knee_db)
    below, inside, above = regions(w)
    assert below > 0 and above > 0 and (inside > 0 or knee_db == 0.0), (below, inside, above)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)


@pytest.mark.parametrize("knee_db", [3.0, 0.0])
@pytest.mark.parametrize("T", T_RAGGED)
def test_gate_backward(T, knee_db):
    say(f"[gate bwd] T={T} knee={knee_db} dB")
    w = gate_workload(T, 43, knee_db)
    errs = run_backward(w, 5)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def mixed_dynamics(seed, T):
    """Random DAG with compressors and noisegates (at least one of each), sources ramped down."""
    for s in range(seed, seed + 100):
        w = synth.random_workload(s, 14, T, types=(synth.MIX, synth.GAIN_PAN, synth.COMP,
                                                   synth.GATE, synth.EQ), edge_p=0.3)
        nt = w.graph.node_type
        if (nt == synth.COMP).sum() >= 1 and (nt == synth.GATE).sum() >= 2:
            w.sources = ramped(w.sources, 0.0, -70.0)
            w.params[synth.GATE][:, 0] = short_alpha(int((nt == synth.GATE).sum()))
            return w
    raise AssertionError("no workload with both dynamics types")


@pytest.mark.parametrize("seed", [700, 800])
def test_mixed_dynamics_forward_backward(seed):
    T = T_RAGGED[(seed // 100) % 2]
    w = mixed_dynamics(seed, T)
    say(f"[mixed dynamics] seed={w.seed} T={T} comp={(w.graph.node_type == synth.COMP).sum()} "
        f"gate={(w.graph.node_type == synth.GATE).sum()}")
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)
    errs = run_backward(w, seed)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def test_gate_schedule_invariance():
    """Every schedule gives the same bits with noisegates and compressors in one graph."""
    w = mixed_dynamics(900, 5 * 2048 + 77)
    S, P = device_inputs(w)
    ref = None
    for m in ("one_by_one", "greedy", "beam"):
        Y = render(Schedule(w.graph.node_type, w.graph.edges, m), S, P)
        torch.cuda.synchronize()
        if ref is None:
            ref = Y.clone()
        else:
            assert torch.equal(Y, ref), m
