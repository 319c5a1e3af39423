"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the same
seeded float32 inputs and compare them at the tolerances the target sets (renders within 1e-5
of the peak output; gradients within 1e-3 of the largest entry of the same parameter column,
i.e. per node type and parameter index, so that a small-valued parameter such as a compressor
threshold is not judged against a large-valued one such as its time constant)."""
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
    Uh = U[sched.num_inputs:].detach().cpu().numpy().astype(np.float64)  # input rows unwritten
    worst = 0.0
    for i in range(sched.num_inputs, sched.num_nodes):
        v = int(sched.perm[i])
        e = rel_err(Uh[i - sched.num_inputs], ys[v].numpy())
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


# A parameter column whose largest oracle entry is below this fraction of the tensor's largest
# entry is structurally zero (e.g. the taps of a delay slot that lies wholly past the end of the
# signal): the FP64 FFT convolution of the oracle leaves rounding residue of about 1e-16 there,
# where the exact value, and the GPU's, is 0. Such a column is judged against the floor instead.
ZERO_COLUMN_FLOOR = 1e-9

# Columns that hold one kind of parameter, in the same units, form a group: the EQ's 1024 bin
# log-magnitudes; each of the reverb's four 192-bin masks (mid H0, mid HD, side H0, side HD); the
# two coordinates (re z, im z) of each delay phasor, whose gradient is a 2-vector (the paper
# normalises it per delay, so its direction is what the optimiser uses). Within a group a column's
# scale is floored at GROUP_FLOOR times the group's largest entry. A gradient entry that crosses
# zero (e.g. one EQ bin of a single EQ node, 4e-5 of the tensor's largest entry; the real part of
# a phasor gradient that points along the imaginary axis) cannot be computed to 1e-3 of itself in
# FP32, whose rounding of the neighbouring large entries is already of that size; judged against
# its group it must still be within 1e-6 of the group's largest entry. Groups are keyed by the
# tensor's width, which is unique for these types (N_t = 1024, 768, 220). Every other column is
# its own group.
GROUP_FLOOR = 1e-3


def _groups(width: int):
    """Group id of every column of a parameter tensor of this width, or None (no groups)."""
    if width == 1024:  # EQ
        return np.zeros(1024, dtype=np.int64)
    if width == 768:  # reverb: [mid, side][H0, HD][192]
        return np.arange(768) // 192
    if width == 220:  # delay: [channel 2][slot 5][re z, im z, 20 log-magnitudes]
        i = np.arange(220)
        return np.where(i % 22 < 2, i // 22, 1000 + i)
    return None


def column_scales(ref: np.ndarray) -> np.ndarray:
    """Per-column judging scale of a parameter-gradient tensor [nodes, N_t] (or of per-column
    maxima [N_t]): the column's largest absolute oracle entry, floored by its group and by
    ZERO_COLUMN_FLOOR times the whole tensor's largest entry."""
    col = np.abs(np.asarray(ref, dtype=np.float64))
    col = col.max(axis=0) if col.ndim == 2 else col
    whole = float(col.max()) if col.size else 0.0
    scale = np.maximum(col, ZERO_COLUMN_FLOOR * whole if whole > 0 else 1.0)
    gid = _groups(col.shape[0])
    if gid is not None:
        for g in np.unique(gid):
            sel = gid == g
            scale[sel] = np.maximum(scale[sel], GROUP_FLOOR * col[sel].max())
    return np.maximum(scale, 1e-300)


def grad_err(a: np.ndarray, ref: np.ndarray) -> float:
    """Worst gradient error. A parameter tensor [nodes, N_t] is judged column by column: each
    column's largest absolute error over the column's scale (column_scales). Any other array (a
    source adjoint, one node's row) is judged against its own largest entry."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if a.ndim != 2:
        return rel_err(a, ref)
    # per-column judgement is for parameter tensors (at most 1024 columns, the EQ's); a signal
    # row [2, T] judged per column would be judged per time sample
    assert ref.shape[1] <= 1024, "judge a signal with rel_err, not per column"
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(a - ref).max(axis=0) / column_scales(ref)))


def row_grad_err(a: np.ndarray, ref: np.ndarray, col_scale: np.ndarray) -> float:
    """Error of one node's parameter-gradient row against per-column scales (the largest
    oracle entry of each column over the nodes checked), floored as in grad_err."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    return float(np.max(np.abs(a - ref) / column_scales(col_scale)))


def check_nodes_locally(w, sched, Uh, dUh=None, dYh=None, dPh=None, types=None, log_every=0):
    """Every processed node (of `types`, if given) against the single-node FP64 oracle fed with
    the GPU's own rows, so that each kernel is checked at full length without error accumulation
    along the graph:
    * its output row from its aggregated input (sum of its sources' rows): within 1e-5 of the
      row's peak;
    * with `dUh` (input adjoints, sigma order), `dYh` (output adjoint) and `dPh` (parameter
      gradients): its input-adjoint row from its output adjoint (the sum of its successors' input
      adjoints) within 1e-3 of that row's largest entry, and its parameter-gradient row, per
      column, within 1e-3 of the largest oracle entry of that column over the nodes of its type.
    Returns the worst errors per type name: (output, input adjoint, parameter gradient)."""
    g = w.graph
    rows = OR.param_rows(g.node_type)
    P64 = OR.as_params64(w.params)
    pos = np.empty(g.num_nodes, dtype=np.int64)
    pos[sched.perm] = np.arange(g.num_nodes)
    ins = [[] for _ in range(g.num_nodes)]
    outs = [[] for _ in range(g.num_nodes)]
    for e in range(g.num_edges):
        s, d = int(g.edges[0, e]), int(g.edges[1, e])
        ins[d].append(s)
        outs[s].append(d)
    out_begin = sched.out_begin

    def y_row(v):
        if g.node_type[v] == synth.IN:
            return torch.as_tensor(w.sources[rows[v]], dtype=F64)
        return torch.as_tensor(Uh[pos[v]], dtype=F64)

    def ybar_row(v):
        a = torch.zeros((2, w.T), dtype=F64)
        for d in outs[v]:
            a += torch.as_tensor(dYh[pos[d] - out_begin] if pos[d] >= out_begin else dUh[pos[d]],
                                 dtype=F64)
        return a

    worst = {}
    prow = []
    nodes = [v for v in range(g.num_nodes) if g.node_type[v] not in (synth.IN,)
             and (types is None or int(g.node_type[v]) in types)]
    for i, v in enumerate(nodes):
        t = int(g.node_type[v])
        u = torch.zeros((2, w.T), dtype=F64)
        for s in ins[v]:
            u = u + y_row(s)
        adj = dUh is not None and t != synth.OUT
        u.requires_grad_(adj)
        p = P64[t][rows[v]].clone().requires_grad_(adj) if t in P64 else None
        y = OR.node_forward(t, u, p)
        e_y = rel_err(Uh[pos[v]].astype(np.float64), y.detach().numpy())
        e_u = 0.0
        if adj:
            wrt = [u] + ([p] if p is not None else [])
            gr = torch.autograd.grad(y, wrt, ybar_row(v), allow_unused=True)
            e_u = rel_err(dUh[pos[v]].astype(np.float64), gr[0].numpy())
            if p is not None and dPh is not None:
                gp = gr[1] if gr[1] is not None else torch.zeros_like(p)
                prow.append((v, t, dPh[t][rows[v]], gp.numpy()))
        name = synth.TYPE_NAMES[t]
        a = worst.get(name, (0.0, 0.0, 0.0))
        worst[name] = (max(a[0], e_y), max(a[1], e_u), a[2])
        assert e_y <= RENDER_TOL, (v, name, "y", e_y)
        assert e_u <= GRAD_TOL, (v, name, "ubar", e_u)
        if log_every and (i + 1) % log_every == 0:
            say(f"   {i + 1}/{len(nodes)} nodes checked")
    scale = {}
    for _, t, _, ref in prow:
        scale[t] = np.maximum(scale.get(t, 0.0), np.abs(ref))
    for v, t, got, ref in prow:
        e_p = row_grad_err(got, ref, scale[t])
        name = synth.TYPE_NAMES[t]
        a = worst[name]
        worst[name] = (a[0], a[1], max(a[2], e_p))
        assert e_p <= GRAD_TOL, (v, name, "dp", e_p)
    return worst


def fmt_worst(worst):
    return {k: tuple(f"{x:.1e}" for x in e) for k, e in worst.items()}
