"""GPU parity of the filtered-noise mid/side reverb (paper Sec. 3 "Reverb", Eqs. 6-7) against the
FP64 oracle (oracle/reverb.py): outputs, source adjoints and the gradients of the mask
parameters (H0, HD per bin, mid and side), on single reverbs and on graphs where reverbs sit in
several steps, next to other processors and in chains. Cases cover a response longer than the
signal (two seconds of noise on a shorter signal), a response shorter than the signal, lengths
that are not multiples of the 2048-sample block or partition, a noise shorter than one
partition, and one node per row at the paper's full noise length. The tolerances are the
render's (1e-5 of the peak output) and the gradients' (1e-3 of each parameter column's largest
entry)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, RENDER_TOL, grad_err, rel_err, say
from oracle import render as OR
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

F64 = torch.float64


def single_reverb(T, L, seed, n_in=2):
    b = synth.GraphBuilder()
    ins = [b.add(synth.IN) for _ in range(n_in)]
    r = b.add(synth.REVERB)
    o = b.add(synth.OUT)
    for i in ins:
        b.connect(i, r)
    b.connect(r, o)
    g = b.build()
    w = synth.Workload("single_reverb", g, synth.make_sources(synth.rng_for(seed, 1), n_in, T),
                       synth.draw_params(synth.rng_for(seed, 2), g), None, T, seed)
    return w, synth.reverb_noise(seed, L)


def reverb_graph(T, L, seed):
    """Reverbs in three steps: two parallel track reverbs (one after a gain), a reverb on their
    mix and, in series, a reverb behind an EQ, all summed at the output."""
    b = synth.GraphBuilder()
    i0, i1, i2 = b.add(synth.IN), b.add(synth.IN), b.add(synth.IN)
    gp = b.add(synth.GAIN_PAN)
    r0, r1 = b.add(synth.REVERB), b.add(synth.REVERB)
    m = b.add(synth.MIX)
    r2 = b.add(synth.REVERB)
    eq = b.add(synth.EQ)
    r3 = b.add(synth.REVERB)
    o = b.add(synth.OUT)
    for s, d in ((i0, gp), (gp, r0), (i1, r1), (i1, r1), (r0, m), (r1, m), (m, r2), (i2, eq),
                 (eq, r3), (r2, o), (r3, o), (i0, o)):
        b.connect(s, d)
    g = b.build()
    w = synth.Workload("reverb_graph", g, synth.make_sources(synth.rng_for(seed, 1), 3, T),
                       synth.draw_params(synth.rng_for(seed, 2), g), None, T, seed)
    return w, synth.reverb_noise(seed, L)


def oracle(w, noise, dY=None):
    g = w.graph
    S = torch.as_tensor(w.sources, dtype=F64).requires_grad_(dY is not None)
    P = OR.as_params64(w.params, requires_grad=dY is not None)
    Y = OR.render(g.node_type, g.edges, S, P, reverb_noise=noise)
    if dY is None:
        return Y.detach().numpy(), None
    keys = [t for t in sorted(P) if P[t].shape[0] > 0]
    gr = torch.autograd.grad((Y * torch.as_tensor(dY, dtype=F64)).sum(), [S] + [P[t] for t in keys],
                             allow_unused=True)
    out = {"S": gr[0].numpy()}
    for t, x in zip(keys, gr[1:]):
        out[t] = np.zeros(tuple(P[t].shape)) if x is None else x.detach().numpy()
    return Y.detach().numpy(), out


def run(w, noise, seed, backward=True):
    sched = Schedule(w.graph.node_type, w.graph.edges)
    sched.set_reverb_noise(torch.as_tensor(noise).cuda())
    S = torch.as_tensor(w.sources).cuda().requires_grad_(backward)
    P = {t: torch.as_tensor(p).cuda().requires_grad_(backward) for t, p in w.params.items()
         if p.shape[0] > 0}
    Y = render(sched, S, P)
    dY = np.random.default_rng(seed).normal(size=tuple(Y.shape)).astype(np.float32)
    if backward:
        Y.backward(torch.as_tensor(dY).cuda())
    torch.cuda.synchronize()
    Yr, ref = oracle(w, noise, dY if backward else None)
    Yh = Y.detach().cpu().numpy().astype(np.float64)
    errs = {"Y": max(rel_err(Yh[o], Yr[o]) for o in range(Yh.shape[0]))}
    if backward:
        errs["S"] = grad_err(S.grad.cpu().numpy(), ref["S"])
        for t, p in P.items():
            errs[synth.TYPE_NAMES[t]] = grad_err(p.grad.cpu().numpy(), ref[t])
    return errs


def check(errs):
    say("   errs", {k: f"{e:.2e}" for k, e in errs.items()})
    assert errs["Y"] <= RENDER_TOL, errs
    for k, e in errs.items():
        if k != "Y":
            assert e <= GRAD_TOL, (k, e)


# (T, L): response longer than the signal; shorter; both ragged; noise below one partition
CASES = [(2 ** 15, synth.REVERB_LEN), (9 * 2048 + 777, 5000), (3 * 2048 + 5, 1500),
         (2048, 2048), (1, 700)]


@pytest.mark.parametrize("T,L", CASES)
def test_single_reverb(T, L):
    say(f"[reverb single] T={T} L={L}")
    w, noise = single_reverb(T, L, 61)
    check(run(w, noise, 3))


@pytest.mark.parametrize("T,L", [(5 * 2048 + 300, 7000), (2 ** 14, synth.REVERB_LEN)])
def test_reverb_graph(T, L):
    say(f"[reverb graph] T={T} L={L}")
    w, noise = reverb_graph(T, L, 62)
    check(run(w, noise, 4))


def test_reverb_full_length():
    """One reverb on a 2^18-sample signal (about 6 s) with the paper's 2 s noise: every partition
    and block of the product and of the FIR gradient in play."""
    T = 2 ** 18
    say(f"[reverb full] T={T} L={synth.REVERB_LEN}")
    w, noise = single_reverb(T, synth.REVERB_LEN, 63)
    check(run(w, noise, 5))


def test_reverb_requires_noise():
    w, _ = single_reverb(4096, 1000, 64)
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S = torch.as_tensor(w.sources).cuda()
    P = {t: torch.as_tensor(p).cuda() for t, p in w.params.items() if p.shape[0] > 0}
    with pytest.raises(Exception, match="noise"):
        render(sched, S, P)


def test_reverb_at_the_largest_length():
    """One reverb at the large console's length, T = 2^20 (512 blocks, every partition of the
    2 s response in play over the whole signal), forward and adjoint against the oracle."""
    T = 2 ** 20
    say(f"[reverb 2^20] T={T} L={synth.REVERB_LEN}")
    w, noise = single_reverb(T, synth.REVERB_LEN, 65, n_in=1)
    check(run(w, noise, 6))
