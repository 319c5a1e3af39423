"""GPU parity of the batched render and its adjoint against the FP64 oracle (paper Algorithm 1;
processors of Sec. 3). Sizes span several tiles with ragged tails (T % 2048 != 0, both T % 4 == 0
and T % 4 != 0) so every kernel's edge handling runs."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import (GRAD_TOL, check_render, device_inputs, grad_err, oracle_grads,
                        rel_err, say)
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

T_RAGGED = [3 * 2048 + 555, 4 * 2048 + 1024 + 4]
SINGLE_TYPES = [synth.MIX, synth.GAIN_PAN, synth.IMAGER, synth.TANH, synth.EQ, synth.COMP,
                synth.DELAY]


def single_node_workload(t, T, seed):
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    n = b.add(t)
    o = b.add(synth.OUT)
    b.connect(i0, n)
    b.connect(i1, n)
    b.connect(i0, n)  # parallel edge: counted twice
    b.connect(n, o)
    g = b.build()
    return synth.Workload(f"single_{t}", g, synth.make_sources(synth.rng_for(seed, 1), 2, T),
                          synth.draw_params(synth.rng_for(seed, 2), g), None, T, seed)


@pytest.mark.parametrize("T", T_RAGGED)
@pytest.mark.parametrize("t", SINGLE_TYPES)
def test_single_processor_forward(t, T):
    say(f"[single fwd] type={t} T={T}")
    w = single_node_workload(t, T, 10 + t)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)


@pytest.mark.parametrize("seed", range(4))
def test_random_dag_forward(seed):
    T = T_RAGGED[seed % 2]
    say(f"[random fwd] seed={seed} T={T}")
    w = synth.random_workload(500 + seed, 14, T, edge_p=0.3, n_out=1 + seed % 2)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)


def test_tiny_console_forward():
    say("[tiny console fwd] T=2^15")
    w = synth.tiny_console(T=2 ** 15)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)


def test_schedule_invariance_and_determinism():
    """All four schedules give bit-identical renders (each node's arithmetic is fixed), and two
    runs give identical bits."""
    say("[invariance] random dag, 4 methods")
    w = synth.random_workload(77, 12, 5 * 2048 + 77, edge_p=0.35)
    S, P = device_inputs(w)
    ref = None
    for m in ("one_by_one", "greedy", "beam", "optimal"):
        sched = Schedule(w.graph.node_type, w.graph.edges, m)
        Y = render(sched, S, P)
        torch.cuda.synchronize()
        if ref is None:
            ref = Y.clone()
            Y2 = render(sched, S, P)
            assert torch.equal(Y2, ref)
        else:
            assert torch.equal(Y, ref), m


def test_empty_and_trivial_graphs():
    say("[trivial] in->out, orphan processor, T=1 and T=5")
    for T in (1, 5, 2048):
        g = synth.Graph(np.array([0, 3, 1, 1, 0], dtype=np.int32),
                        np.array([[0, 0, 1], [2, 1, 3]], dtype=np.int32))
        w = synth.Workload("trivial", g, synth.make_sources(synth.rng_for(1, 1), 2, T),
                           synth.draw_params(synth.rng_for(1, 2), g), None, T, 1)
        sched = Schedule(g.node_type, g.edges)
        S, P = device_inputs(w)
        Y, U = render(sched, S, P, return_U=True)
        torch.cuda.synchronize()
        check_render(w, sched, Y, U)


# ---- adjoint -------------------------------------------------------------------------------


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


@pytest.mark.parametrize("T", T_RAGGED)
@pytest.mark.parametrize("t", SINGLE_TYPES)
def test_single_processor_backward(t, T):
    say(f"[single bwd] type={t} T={T}")
    w = single_node_workload(t, T, 30 + t)
    errs = run_backward(w, t)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


@pytest.mark.parametrize("seed", range(4))
def test_random_dag_backward(seed):
    T = T_RAGGED[seed % 2]
    say(f"[random bwd] seed={seed} T={T}")
    w = synth.random_workload(600 + seed, 14, T, edge_p=0.3, n_out=1 + seed % 2)
    errs = run_backward(w, seed)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def test_tiny_console_backward():
    say("[tiny console bwd]")
    errs = run_backward(synth.tiny_console(T=2 ** 15), 3)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


@pytest.mark.parametrize("a", [0.0, 0.999999])
def test_compressor_alpha_edge_values(a):
    """alpha at the ends of its domain [0, 1): 0 (no smoothing, g = x) and a time constant of
    about 23 s, across several 3072-sample chunks, forward and adjoint against the oracle. With
    a = 0 the chunk carry weights A^d (A = a^3072) must be 1 for the adjacent chunk and 0 beyond;
    near 1 every earlier chunk's total reaches the carry."""
    T = 5 * 3072 + 77
    say(f"[compressor alpha={a}] T={T}")
    w = single_node_workload(synth.COMP, T, 41)
    w.params[synth.COMP][:, 0] = a
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)
    errs = run_backward(w, 5)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)
