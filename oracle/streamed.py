"""Streamed oracle: the render and its adjoint of a graph too large for whole-graph autograd (the
256-track console at T = 2^20 would hold on the order of 10^11 bytes of autograd state), one node
at a time in float64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward: exactly `render.render` (Eq. 1: each node's input is the sum of its sources' outputs in
original edge order, then its processor), visiting nodes in the same Kahn order; each output is
kept only while a later node or the adjoint needs it.

Adjoint (the backpropagation through the render, paper Sec. 4): nodes in the reverse of that
order. A node's output adjoint is the sum, over its outgoing edges in original edge order, of the
input adjoints of their destinations (the adjoint of Eq. 1b: a sum distributes its adjoint to
every summand), or the given output adjoint for an `out` node; its input is re-formed from its
sources' outputs, and the hand-written adjoint of its processor (`adjoint`) gives its input
adjoint and its parameter gradient. A source's adjoint is its input node's output adjoint. Each
output is freed once the adjoints that re-form inputs from it are done, each input adjoint once
every predecessor of its node has read it.

Parity pins (tests): the forward equals `render.render` bit for bit; the adjoint equals torch
autograd through `render.render` on small graphs of every processor type it covers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import adjoint as A
from . import processors
from .render import IN, OUT, kahn_order, param_rows

F64 = torch.float64


def _structure(node_type, edges):
    node_type = np.asarray(node_type)
    edges = np.asarray(edges).reshape(2, -1)
    V = node_type.shape[0]
    ins = [[] for _ in range(V)]
    outs = [[] for _ in range(V)]
    for e in range(edges.shape[1]):  # original edge order
        s, d = int(edges[0, e]), int(edges[1, e])
        ins[d].append(s)
        outs[s].append(d)
    return node_type, edges, ins, outs


def render_and_adjoint(node_type, edges, sources, params: dict, dY=None, progress=None):
    """Y [n_out, 2, T] and, if `dY` ([n_out, 2, T], output nodes in node order) is given, the
    adjoints of the sources dS [K, 2, T] and of every parameter tensor dP[t] [n_t, N_t] for the
    loss sum(dY * Y). `sources`: float32 numpy [K, 2, T]; `params`: type -> float32 numpy
    [n_t, N_t] (upcast exactly). `progress(stage, i, n)` is called every 64 nodes."""
    node_type, edges, ins, outs = _structure(node_type, edges)
    V = node_type.shape[0]
    S = torch.as_tensor(np.asarray(sources), dtype=F64)
    T = S.shape[-1]
    P64 = {int(t): torch.as_tensor(np.asarray(p), dtype=F64) for t, p in params.items()}
    rows = param_rows(node_type)
    order = kahn_order(node_type, edges)
    out_nodes = [v for v in range(V) if int(node_type[v]) == OUT]

    def node_input(v, y):
        u = None
        for s in ins[v]:
            u = y[s] if u is None else u + y[s]
        return torch.zeros((2, T), dtype=F64) if u is None else u

    # forward; with an adjoint to follow, every output is kept for the inputs it re-forms
    y: list = [None] * V
    readers = [len(set(outs[v])) for v in range(V)]  # distinct consumers still to run
    for i, v in enumerate(order):
        t = int(node_type[v])
        if t == IN:
            y[v] = S[rows[v]]
        else:
            u = node_input(v, y)
            p = P64[t][rows[v]] if processors.N_PARAMS[t] else None
            with torch.no_grad():
                y[v] = processors.PROCESS[t](u, p)
            if dY is None:
                for s in set(ins[v]):
                    readers[s] -= 1
                    if readers[s] == 0 and int(node_type[s]) != OUT:
                        y[s] = None
        if progress and (i + 1) % 64 == 0:
            progress("forward", i + 1, V)
    Y = torch.stack([y[v] for v in out_nodes])
    if dY is None:
        return Y

    dY64 = torch.as_tensor(np.asarray(dY), dtype=F64)
    ubar: list = [None] * V
    pending = [len(set(ins[v])) for v in range(V)]  # predecessors that still read ubar[v]
    dS = torch.zeros_like(S)
    dP = {t: torch.zeros_like(p) for t, p in P64.items()}
    for i, v in enumerate(reversed(order)):
        t = int(node_type[v])
        if t == OUT:
            ybar = dY64[out_nodes.index(v)]
        else:
            ybar = torch.zeros((2, T), dtype=F64)
            for d in outs[v]:
                ybar = ybar + ubar[d]
            for d in set(outs[v]):
                pending[d] -= 1
                if pending[d] == 0:
                    ubar[d] = None
        if t == IN:
            dS[rows[v]] = ybar
        else:
            u = node_input(v, y)
            p = P64[t][rows[v]] if processors.N_PARAMS[t] else None
            ub, pb = A.ADJOINT[t](u, p, ybar)
            ubar[v] = ub
            if pb is not None:
                dP[t][rows[v]] = pb
            if pending[v] == 0:
                ubar[v] = None
        y[v] = None if t != IN else y[v]
        if progress and (i + 1) % 64 == 0:
            progress("adjoint", i + 1, V)
    return Y, dS, dP
