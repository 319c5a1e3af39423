"""GPU parity on seeded random DAGs drawn from every processing type the library has (gain/pan,
EQ, compressor, imager, 500 ms and 2 s delays, tanh, noisegate, attack/release compressor,
reverb, mix), with parallel edges, several outputs, shuffled ids and the delay-time surrogate
on: outputs, source adjoints and every parameter gradient against the FP64 oracle, at lengths
that are not multiples of any tile or chunk. Tolerances as everywhere: 1e-5 of each output's
peak, 1e-3 of each parameter column's largest entry (column groups as in gpu_common)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import GRAD_TOL, RENDER_TOL, grad_err, rel_err, say
from oracle import render as OR
from paper_2408_03204_amd import Schedule, render

pytestmark = pytest.mark.gpu

F64 = torch.float64
ALL = (synth.MIX, synth.GAIN_PAN, synth.EQ, synth.COMP, synth.IMAGER, synth.DELAY, synth.TANH,
       synth.GATE, synth.COMP_AR, synth.REVERB, synth.DELAY_LONG)
NOISE_LEN = 6000


@pytest.mark.parametrize("seed", range(6))
def test_random_graph_every_type(seed):
    T = (5 * 2048 + 333, 4 * 3072 + 5, 23000)[seed % 3]
    w = synth.random_workload(1600 + seed, 16, T, types=ALL, edge_p=0.3, n_out=1 + seed % 2)
    g = w.graph
    noise = synth.reverb_noise(1600 + seed, NOISE_LEN)
    counts = {synth.TYPE_NAMES[t]: int((g.node_type == t).sum()) for t in ALL
              if (g.node_type == t).any()}
    say(f"[all types] seed={seed} T={T} nodes={g.num_nodes} {counts}")
    dev = torch.device("cuda")
    sched = Schedule(g.node_type, g.edges, "beam")
    sched.set_reverb_noise(torch.as_tensor(noise, device=dev))
    sched.set_delay_surrogate(True)
    S = torch.as_tensor(w.sources, device=dev).requires_grad_(True)
    P = {t: torch.as_tensor(p, device=dev).requires_grad_(True) for t, p in w.params.items()
         if p.shape[0] > 0}
    Y = render(sched, S, P)
    dY = np.random.default_rng(seed).standard_normal(tuple(Y.shape)).astype(np.float32)
    Y.backward(torch.as_tensor(dY, device=dev))
    torch.cuda.synchronize()
    S64 = torch.as_tensor(w.sources, dtype=F64).requires_grad_(True)
    P64 = OR.as_params64(w.params, requires_grad=True)
    Yr = OR.render(g.node_type, g.edges, S64, P64, reverb_noise=noise, delay_surrogate=True)
    keys = [t for t in sorted(P64) if P64[t].shape[0] > 0]
    gr = torch.autograd.grad((Yr * torch.as_tensor(dY, dtype=F64)).sum(),
                             [S64] + [P64[t] for t in keys], allow_unused=True)
    Yh = Y.detach().cpu().numpy().astype(np.float64)
    Yr = Yr.detach().numpy()
    errs = {"Y": max(rel_err(Yh[o], Yr[o]) for o in range(Yh.shape[0])),
            "S": grad_err(S.grad.cpu().numpy(), gr[0].numpy())}
    for t, x in zip(keys, gr[1:]):
        ref = np.zeros(tuple(P64[t].shape)) if x is None else x.numpy()
        errs[synth.TYPE_NAMES[t]] = grad_err(P[t].grad.cpu().numpy(), ref)
    say("   errs", {k: f"{e:.2e}" for k, e in errs.items()})
    assert errs["Y"] <= RENDER_TOL, errs
    for k, e in errs.items():
        if k != "Y":
            assert e <= GRAD_TOL, (k, e)
