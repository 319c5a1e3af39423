"""Oracle renderer: the graph evaluated one node at a time (paper Sec. 2 "Definitions", Eq. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each node's input is the sum of the outputs of its predecessors over its incoming edges
(Eq. 1b; parallel edges count once per edge), summed in original edge order; the node's output
is its processor applied to that sum with the node's parameter row (Eq. 1a). Input nodes emit
their source (the k-th input node takes the k-th source, Sec. 2 "Graph representations");
mix and output nodes emit their input sum. Nodes are visited in a topological order (Kahn's
algorithm, ready nodes by smallest id) from the inputs to the outputs. A node with no incoming
edge gets a zero input.

Everything is torch float64 on the CPU; parameters and sources are the same float32 arrays the
GPU receives, upcast exactly. Gradients: torch autograd.

Parity pins (tests): gain/pan-only graphs equal the sum over source-to-output paths of the
product of per-node gains; flat EQs, below-threshold compressors and zero-width imagers are the
identity; every topological order gives bit-identical output; autograd gradients match central
finite differences.
"""
from __future__ import annotations

import numpy as np
import torch

from . import processors, reverb

F64 = torch.float64
IN, OUT = 0, 1


def kahn_order(node_type, edges) -> list[int]:
    node_type = np.asarray(node_type)
    edges = np.asarray(edges).reshape(2, -1)
    V = node_type.shape[0]
    indeg = [0] * V
    succ = [[] for _ in range(V)]
    for e in range(edges.shape[1]):
        succ[int(edges[0, e])].append(int(edges[1, e]))
        indeg[int(edges[1, e])] += 1
    import heapq
    ready = [v for v in range(V) if indeg[v] == 0]
    heapq.heapify(ready)
    order = []
    while ready:
        v = heapq.heappop(ready)
        order.append(v)
        for w in succ[v]:
            indeg[w] -= 1
            if indeg[w] == 0:
                heapq.heappush(ready, w)
    if len(order) != V:
        raise ValueError("graph has a cycle")
    return order


def param_rows(node_type) -> list[int]:
    """Row of each node within its type, in node order."""
    seen: dict[int, int] = {}
    rows = []
    for t in np.asarray(node_type).tolist():
        rows.append(seen.get(t, 0))
        seen[t] = seen.get(t, 0) + 1
    return rows


def as_params64(params: dict, requires_grad: bool = False) -> dict:
    out = {}
    for t, p in params.items():
        q = torch.as_tensor(np.asarray(p), dtype=F64).clone()
        if requires_grad:
            q.requires_grad_(True)
        out[int(t)] = q
    return out


def node_forward(t: int, u: torch.Tensor, p: torch.Tensor | None, reverb_noise=None,
                 delay_surrogate: bool = False) -> torch.Tensor:
    """One processor call on one node (Eq. 1a). A reverb needs the noise realisation
    [2, L] (mid, side); `delay_surrogate` gives delay phasors their straight-through gradient."""
    if t == processors.REVERB:
        if reverb_noise is None:
            raise ValueError("a reverb node needs the reverb noise realisation")
        return reverb.reverb(u, p, reverb_noise)
    if t in (7, 12) and delay_surrogate:  # delay, delay_long
        return processors.delay(u, p, surrogate=True)
    return processors.PROCESS[t](u, p)


def render(node_type, edges, sources, params: dict, order=None, keep_all: bool = False,
           reverb_noise=None, delay_surrogate: bool = False):
    """Returns Y [n_out, 2, T] (output nodes in node order) and, if `keep_all`, the list of
    every node's output (None for unreachable entries is impossible: all nodes are visited).

    `sources` may be a numpy float32 array or a float64 tensor (possibly requiring grad);
    `params` maps type code -> float64 tensor [n_t, N_t] (see `as_params64`)."""
    node_type = np.asarray(node_type)
    edges = np.asarray(edges).reshape(2, -1)
    V = node_type.shape[0]
    S = sources if torch.is_tensor(sources) else torch.as_tensor(np.asarray(sources), dtype=F64)
    T = S.shape[-1]
    if order is None:
        order = kahn_order(node_type, edges)
    rows = param_rows(node_type)
    in_edges = [[] for _ in range(V)]
    for e in range(edges.shape[1]):  # original edge order
        in_edges[int(edges[1, e])].append(int(edges[0, e]))
    y: list = [None] * V
    for v in order:
        t = int(node_type[v])
        if t == IN:
            y[v] = S[rows[v]]
            continue
        u = None
        for s in in_edges[v]:
            if y[s] is None:
                raise ValueError("order is not topological")
            u = y[s] if u is None else u + y[s]
        if u is None:
            u = torch.zeros((2, T), dtype=F64)
        p = params[t][rows[v]] if processors.N_PARAMS[t] else None
        y[v] = node_forward(t, u, p, reverb_noise, delay_surrogate)
    outs = [v for v in range(V) if int(node_type[v]) == OUT]
    Y = torch.stack([y[v] for v in outs])
    return (Y, y) if keep_all else Y
