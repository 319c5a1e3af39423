"""GPU parity of the compressor with distinct attack and release ballistics (Eq. 8 unrestricted)
against the FP64 oracle's literal per-sample loop, forward and adjoint. The kernel iterates on
the attack/release branch pattern and falls back to a serial recursion for any chunk that has
not settled after a given number of passes. That number is the schedule's
GRAFX_TUNE_AR_MAX_PASSES setting, lowered here through the C ABI so that the fallback runs
(1 pass: almost every chunk falls back; 2-3: some do)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, check_render, device_inputs, grad_err, oracle_grads, say
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

T_RAGGED = [3 * 2048 + 555, 6 * 3072 + 1024 + 4]
FS = synth.FS


def alpha(ms):
    return float(np.exp(-1.0 / (ms * 1e-3 * FS)))


def ar_workload(T, seed, attack_ms, release_ms):
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    n = b.add(synth.COMP_AR)
    o = b.add(synth.OUT)
    b.connect(i0, n)
    b.connect(i1, n)
    b.connect(i0, n)
    b.connect(n, o)
    g = b.build()
    P = synth.draw_params(synth.rng_for(seed, 2), g)
    P[synth.COMP_AR][:, 0] = alpha(attack_ms)
    P[synth.COMP_AR][:, 1] = alpha(release_ms)
    return synth.Workload("single_comp_ar", g, synth.make_sources(synth.rng_for(seed, 1), 2, T),
                          P, None, T, seed)


def make_schedule(w, passes=None):
    sched = Schedule(w.graph.node_type, w.graph.edges)
    if passes is not None:
        sched.set_tuning(Schedule.TUNE_AR_MAX_PASSES, passes)
    return sched


def run_forward(w, passes=None):
    sched = make_schedule(w, passes)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)
    return Y


def run_backward(w, seed, passes=None):
    sched = make_schedule(w, passes)
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


CASES = [(2.0, 80.0), (90.0, 1.0), (10.0, 10.0)]


@pytest.mark.parametrize("ms", CASES)
@pytest.mark.parametrize("T", T_RAGGED)
def test_comp_ar_forward(T, ms):
    say(f"[comp_ar fwd] T={T} attack/release={ms} ms")
    run_forward(ar_workload(T, 51, *ms))


@pytest.mark.parametrize("ms", CASES)
@pytest.mark.parametrize("T", T_RAGGED)
def test_comp_ar_backward(T, ms):
    say(f"[comp_ar bwd] T={T} attack/release={ms} ms")
    errs = run_backward(ar_workload(T, 53, *ms), 7)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_comp_ar_serial_fallback(passes):
    """With few passes allowed, unsettled chunks take the serial fallback: the results stay
    within tolerance of the oracle, forward and adjoint."""
    T = T_RAGGED[1]
    say(f"[comp_ar fallback] max passes {passes} T={T}")
    run_forward(ar_workload(T, 55, 2.0, 60.0), passes)
    errs = run_backward(ar_workload(T, 57, 70.0, 2.0), 9, passes)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def mixed_ar(seed, T):
    types = (synth.MIX, synth.GAIN_PAN, synth.COMP, synth.COMP_AR, synth.EQ, synth.GATE)
    for s in range(seed, seed + 200):
        w = synth.random_workload(s, 14, T, types=types, edge_p=0.3)
        nt = w.graph.node_type
        if (nt == synth.COMP_AR).sum() >= 2 and (nt == synth.COMP).sum() >= 1:
            return w
    raise AssertionError("no workload with two attack/release compressors")


@pytest.mark.parametrize("seed", [1000, 1100])
def test_comp_ar_random_dags(seed):
    T = T_RAGGED[(seed // 100) % 2]
    w = mixed_ar(seed, T)
    say(f"[comp_ar dag] seed={w.seed} T={T} ar={(w.graph.node_type == synth.COMP_AR).sum()}")
    Y1 = run_forward(w)
    Y2 = render(Schedule(w.graph.node_type, w.graph.edges, "one_by_one"), *device_inputs(w))
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)  # schedule-independent bits
    errs = run_backward(w, seed)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def test_tiny_console_with_attack_release():
    say("[comp_ar tiny console] T=2^15")
    w = synth.tiny_console(T=2 ** 15, attack_release=True)
    run_forward(w)
    errs = run_backward(w, 3)
    say("   grad errs", errs)
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)


def test_comp_ar_merged_graphs_equal_alone():
    """Graphs of different lengths with attack/release compressors merged into one schedule give
    each graph the bits it gets alone."""
    from test_gpu_batch import _check_merged
    ws = [mixed_ar(1200 + 50 * i, T) for i, T in enumerate((6699, 9220, 3001))]
    _check_merged(ws, "attack/release")
