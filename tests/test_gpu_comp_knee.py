"""GPU parity of the compressor's gain curve over all of its regions (paper Sec. 3
"Compressor", Eqs. 10-11: below the knee, inside the quadratic knee, above it), with a soft
knee and with a hard one (W = 0), for the compressor with one ballistics constant and the one
with attack and release constants, forward and adjoint against the FP64 oracle. The sources fall
from 0 dB to -60 dB along the signal, so each compressor's envelope passes through every region
of its curve; short time constants (2-5 ms) let the envelope follow the fall."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, check_render, device_inputs, grad_err, oracle_grads, say
from oracle import processors as OP
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

T_CASES = [3 * 3072 + 555, 2 ** 15]


def ramped(sources: np.ndarray, top_db=0.0, bottom_db=-60.0) -> np.ndarray:
    T = sources.shape[-1]
    ramp = 10.0 ** (np.linspace(top_db, bottom_db, T) / 20.0)
    return (sources * ramp[None, None, :]).astype(np.float32)


def comp_workload(t, T, seed, knee_db):
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    n = b.add(t)
    o = b.add(synth.OUT)
    b.connect(i0, n)
    b.connect(i1, n)
    b.connect(n, o)
    g = b.build()
    S = ramped(synth.make_sources(synth.rng_for(seed, 1), 2, T))
    P = synth.draw_params(synth.rng_for(seed, 2), g)
    p = P[t]
    tau = np.array([2e-3, 5e-3])
    alpha = np.exp(-1.0 / (tau * synth.FS)).astype(np.float32)
    if t == synth.COMP:
        p[:, 0] = alpha[1]
        p[:, 1] = -20.0 * synth.LN10_10  # threshold
        p[:, 2] = knee_db * synth.LN10_10
    else:  # attack faster than release
        p[:, 0], p[:, 1] = alpha[0], alpha[1]
        p[:, 2] = -20.0 * synth.LN10_10
        p[:, 3] = knee_db * synth.LN10_10
    return synth.Workload(f"single_{synth.TYPE_NAMES[t]}", g, S, P, None, T, seed)


def regions(w, t):
    """Samples of the envelope below, inside and above the knee (oracle FP64)."""
    S = torch.as_tensor(w.sources, dtype=torch.float64)
    u = S[0] + S[1]
    x = (u[0] + u[1]) ** 2
    p = torch.as_tensor(w.params[t][0], dtype=torch.float64)
    if t == synth.COMP:
        env, thr, knee = OP.one_pole(x, p[0]), float(p[1]), float(p[2])
    else:
        env, thr, knee = OP.ballistics(x, p[0], p[1]), float(p[2]), float(p[3])
    Gu = torch.log(env + OP.EPS_ENV)
    lo, hi = thr - knee, thr + knee
    return int((Gu < lo).sum()), int(((Gu >= lo) & (Gu < hi)).sum()), int((Gu >= hi).sum())


@pytest.mark.parametrize("knee_db", [3.0, 0.0])
@pytest.mark.parametrize("t", [synth.COMP, synth.COMP_AR])
@pytest.mark.parametrize("T", T_CASES)
def test_compressor_curve_regions(T, t, knee_db):
    name = synth.TYPE_NAMES[t]
    say(f"[{name} curve] T={T} knee={knee_db} dB")
    w = comp_workload(t, T, 51, knee_db)
    below, inside, above = regions(w, t)
    assert below > 0 and above > 0 and (inside > 0 or knee_db == 0.0), (below, inside, above)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S, P = device_inputs(w)
    Y, U = render(sched, S, P, return_U=True)
    torch.cuda.synchronize()
    check_render(w, sched, Y, U)
    S.requires_grad_(True)
    for p in P.values():
        p.requires_grad_(True)
    Y = render(sched, S, P)
    dY = np.random.default_rng(52).normal(size=tuple(Y.shape)).astype(np.float32)
    Y.backward(torch.as_tensor(dY).cuda())
    torch.cuda.synchronize()
    ref = oracle_grads(w, dY)
    errs = {"S": grad_err(S.grad.cpu().numpy(), ref["S"])}
    for k, p in P.items():
        errs[synth.TYPE_NAMES[k]] = grad_err(p.grad.cpu().numpy(), ref[k])
    say("   regions", (below, inside, above), "grad errs", {k: f"{e:.2e}" for k, e in errs.items()})
    for k, e in errs.items():
        assert e <= GRAD_TOL, (k, e)
