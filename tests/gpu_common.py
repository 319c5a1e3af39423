"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the same
seeded float32 inputs and compare them at the tolerances the target sets (renders within 1e-5
of the peak output, gradients within 1e-3 of the largest gradient entry, per tensor)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import synth
from oracle import mrstft as OM
from oracle import render as OR

RENDER_TOL = 1e-5
GRAD_TOL = 1e-3
F64 = torch.float64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_inputs(w: synth.Workload):
    S = torch.as_tensor(w.sources).cuda()
    P = {t: torch.as_tensor(p).cuda() for t, p in w.params.items() if p.shape[0] > 0}
    return S, P


def oracle_forward(w: synth.Workload, keep_all=True):
    g = w.graph
    with torch.no_grad():
        return OR.render(g.node_type, g.edges, w.sources, OR.as_params64(w.params),
                         keep_all=keep_all)


def rel_err(a: np.ndarray, ref: np.ndarray) -> float:
    scale = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(a - ref))) / (scale if scale > 0 else 1.0)


def check_render(w, sched, Y, U, node_tol=RENDER_TOL):
    """Output rows within RENDER_TOL of their peak; every processed node's row too."""
    Y64, ys = oracle_forward(w)
    Y = Y.detach().cpu().numpy().astype(np.float64)
    for o in range(Y.shape[0]):
        e = rel_err(Y[o], Y64[o].numpy())
        assert e <= RENDER_TOL, f"output {o}: rel err {e:.3e}"
    Uh = U.detach().cpu().numpy().astype(np.float64)
    worst = 0.0
    for i in range(sched.num_inputs, sched.num_nodes):
        v = int(sched.perm[i])
        e = rel_err(Uh[i], ys[v].numpy())
        worst = max(worst, e)
        assert e <= node_tol, f"node {v} (type {w.graph.node_type[v]}): rel err {e:.3e}"
    return worst


def oracle_grads(w: synth.Workload, dY: np.ndarray):
    """Gradients of sum(dY * Y) w.r.t. sources and every parameter tensor (FP64 autograd)."""
    g = w.graph
    S = torch.as_tensor(w.sources, dtype=F64).requires_grad_(True)
    P = OR.as_params64(w.params, requires_grad=True)
    Y = OR.render(g.node_type, g.edges, S, P)
    L = (Y * torch.as_tensor(dY, dtype=F64)).sum()
    keys = [t for t in sorted(P) if P[t].shape[0] > 0]
    grads = torch.autograd.grad(L, [S] + [P[t] for t in keys], allow_unused=True)
    out = {"S": grads[0]}
    for t, gr in zip(keys, grads[1:]):
        out[t] = torch.zeros_like(P[t]) if gr is None else gr
    return {k: v.detach().numpy() for k, v in out.items()}


def grad_err(a: np.ndarray, ref: np.ndarray) -> float:
    return rel_err(a.astype(np.float64), ref)
