"""Oracle type scheduler (paper Sec. 2, "Batched processing" and "Type scheduling";
Algorithm 1, preprocessing steps ScheduleBatchedProcessing, OptimizeNodeOrder, Reorder and
GetReadWriteIndex; "Implementation details").

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes:
* the node subsets V_0..V_N form a partition, are causal and each holds one type;
* each subset is maximal for its type, so a schedule is a string of types;
* V_0 holds every input node and V_N every output node;
* the shortest string is found by exhaustive search ("optimal"), approximately by choosing the
  type with the most computable nodes ("greedy"), or by a beam search keeping several
  candidates (32 in the benchmark); one-by-one processing is the baseline.
* After scheduling, nodes are reordered so that each step's nodes are contiguous, and index
  lists for reading inputs, parameters and writing outputs are built.

Readings where the paper is silent (tie-breaks):
* greedy ties go to the smallest type code;
* a beam expands every state by every available type, keeps, for each reachable computed set,
  the lexicographically smallest type string that reaches it, ranks states by (more nodes
  computed first, then smaller string) and keeps the best `beam_width`; it stops at the first
  depth where some state has computed every non-output node and takes the smallest string
  among those; optimal is the same search without the width cap;
* one-by-one takes the ready node with the smallest id;
* an output node is never scheduled before the last step;
* the reordering sorts nodes by (step, original id);
* each node's inputs are listed in original edge order (parallel edges counted each time).

Parity pins (tests): the partition/causality/homogeneity invariants on random DAGs; optimal
equals brute-force enumeration of every maximal-subset type string on small graphs; beam(1)
equals greedy; an unbounded beam equals optimal; optimal <= beam, greedy <= one-by-one; a
21-node graph built to have an optimal schedule of N = 9 processing calls as in the paper's
Fig. 1 example.
"""
from __future__ import annotations

import dataclasses

import numpy as np

IN, OUT = 0, 1
NUM_TYPES = 13  # in, out, mix, gain_pan, eq, compressor, imager, delay, tanh, noisegate,
#                  compressor_ar, reverb, delay_long

ONE_BY_ONE, GREEDY, BEAM, OPTIMAL = 0, 1, 2, 3
METHOD_NAMES = {"one_by_one": ONE_BY_ONE, "greedy": GREEDY, "beam": BEAM, "optimal": OPTIMAL}


class ScheduleError(Exception):
    """`kind` is one of 'arg', 'graph', 'cycle', 'type', 'limit'."""

    def __init__(self, kind: str, msg: str):
        super().__init__(f"{kind}: {msg}")
        self.kind = kind


@dataclasses.dataclass
class Schedule:
    step_type: np.ndarray  # int32 [N+1]
    step_ptr: np.ndarray  # int32 [N+2]
    perm: np.ndarray  # int32 [V]   perm[i] = original id at reordered position i
    in_ptr: np.ndarray  # int32 [V+1]
    in_src: np.ndarray  # int32 [E]   reordered positions of sources, by original edge id
    out_ptr: np.ndarray  # int32 [V+1]
    out_dst: np.ndarray  # int32 [E]
    param_row: np.ndarray  # int32 [V]  row of the node among its type, in original node order

    @property
    def num_steps(self) -> int:
        return int(self.step_type.shape[0]) - 1

    def type_string(self) -> tuple:
        return tuple(int(t) for t in self.step_type)


def validate(node_type, edges, edge_type=None) -> None:
    node_type = np.asarray(node_type)
    edges = np.asarray(edges).reshape(2, -1)
    V = node_type.shape[0]
    if V < 1:
        raise ScheduleError("arg", "graph has no nodes")
    for v in range(V):
        if not 0 <= int(node_type[v]) < NUM_TYPES:
            raise ScheduleError("type", f"node {v} has unknown type {int(node_type[v])}")
    for e in range(edges.shape[1]):
        s, d = int(edges[0, e]), int(edges[1, e])
        if not (0 <= s < V and 0 <= d < V):
            raise ScheduleError("graph", f"edge {e} references a missing node")
    if edge_type is not None:
        et = np.asarray(edge_type).reshape(2, -1)
        if np.any(et != 0):
            raise ScheduleError("type", "multi-port edge types are not supported (SISO only)")
    for e in range(edges.shape[1]):
        s, d = int(edges[0, e]), int(edges[1, e])
        if int(node_type[d]) == IN:
            raise ScheduleError("graph", f"edge {e} enters input node {d}")
        if int(node_type[s]) == OUT:
            raise ScheduleError("graph", f"edge {e} leaves output node {s}")
    if not np.any(node_type == OUT):
        raise ScheduleError("graph", "graph has no output node")
    # cycle check: Kahn's algorithm must consume every node
    indeg = [0] * V
    succ = [[] for _ in range(V)]
    for e in range(edges.shape[1]):
        s, d = int(edges[0, e]), int(edges[1, e])
        succ[s].append(d)
        indeg[d] += 1
    stack = [v for v in range(V) if indeg[v] == 0]
    seen = 0
    while stack:
        v = stack.pop()
        seen += 1
        for w in succ[v]:
            indeg[w] -= 1
            if indeg[w] == 0:
                stack.append(w)
    if seen != V:
        raise ScheduleError("cycle", "graph has a cycle")


class _Graph:
    def __init__(self, node_type, edges):
        self.node_type = [int(t) for t in node_type]
        self.V = len(self.node_type)
        self.edges = np.asarray(edges).reshape(2, -1)
        self.pred_mask = [0] * self.V
        for e in range(self.edges.shape[1]):
            s, d = int(self.edges[0, e]), int(self.edges[1, e])
            self.pred_mask[d] |= 1 << s
        self.proc = [v for v in range(self.V) if self.node_type[v] not in (IN, OUT)]
        self.start = 0
        for v in range(self.V):
            if self.node_type[v] == IN:
                self.start |= 1 << v
        self.full = self.start
        for v in self.proc:
            self.full |= 1 << v

    def ready(self, C: int) -> list[int]:
        """Non-input, non-output nodes not yet computed whose predecessors all are."""
        return [v for v in self.proc if not (C >> v) & 1 and (self.pred_mask[v] & ~C) == 0]

    def ready_by_type(self, C: int) -> dict[int, int]:
        out: dict[int, int] = {}
        for v in self.ready(C):
            t = self.node_type[v]
            out[t] = out.get(t, 0) | (1 << v)
        return out


def _popcount(x: int) -> int:
    return bin(x).count("1")


def _one_by_one(g: _Graph) -> list[int]:
    steps, C = [], g.start
    while C != g.full:
        v = min(g.ready(C))
        steps.append(g.node_type[v])
        C |= 1 << v
    return steps


def _greedy(g: _Graph) -> list[int]:
    steps, C = [], g.start
    while C != g.full:
        by_t = g.ready_by_type(C)
        best = min(by_t, key=lambda t: (-_popcount(by_t[t]), t))
        steps.append(best)
        C |= by_t[best]
    return steps


def _beam(g: _Graph, width: int | None, state_limit: int) -> list[int]:
    states = [(g.start, ())]
    while True:
        done = [s for C, s in states if C == g.full]
        if done:
            return list(min(done))
        children: dict[int, tuple] = {}
        for C, s in states:
            by_t = g.ready_by_type(C)
            for t in sorted(by_t):
                C2, s2 = C | by_t[t], s + (t,)
                if C2 not in children or s2 < children[C2]:
                    children[C2] = s2
        ranked = sorted(children.items(), key=lambda kv: (-_popcount(kv[0]), kv[1]))
        if width is None:
            if len(ranked) > state_limit:
                raise ScheduleError("limit", f"optimal search exceeded {state_limit} states")
            states = ranked
        else:
            states = ranked[:width]


def type_string(node_type, edges, method: int, beam_width: int = 32,
                state_limit: int = 1 << 20) -> list[int]:
    """Processing-step types only (without the leading input and trailing output steps)."""
    g = _Graph(node_type, edges)
    if method == ONE_BY_ONE:
        return _one_by_one(g)
    if method == GREEDY:
        return _greedy(g)
    if method == BEAM:
        if beam_width < 1:
            raise ScheduleError("arg", "beam width must be positive")
        return _beam(g, beam_width, state_limit)
    if method == OPTIMAL:
        if state_limit < 1:
            raise ScheduleError("arg", "state limit must be positive")
        return _beam(g, None, state_limit)
    raise ScheduleError("arg", f"unknown method {method}")


def steps_from_string(node_type, edges, types: list[int]) -> list[list[int]]:
    """Replay a type string: each step takes every ready node of its type (maximal subset)."""
    g = _Graph(node_type, edges)
    C = g.start
    steps = [[v for v in range(g.V) if g.node_type[v] == IN]]
    for t in types:
        nodes = [v for v in g.ready(C) if g.node_type[v] == t]
        if not nodes:
            raise ValueError(f"type {t} has no ready node")
        steps.append(nodes)
        for v in nodes:
            C |= 1 << v
    if C != g.full:
        raise ValueError("type string does not cover the graph")
    steps.append([v for v in range(g.V) if g.node_type[v] == OUT])
    return steps


def schedule(node_type, edges, method: int = BEAM, beam_width: int = 32,
             state_limit: int = 1 << 20, edge_type=None) -> Schedule:
    validate(node_type, edges, edge_type)
    node_type = np.asarray(node_type, dtype=np.int64)
    edges = np.asarray(edges, dtype=np.int64).reshape(2, -1)
    V, E = node_type.shape[0], edges.shape[1]
    types = type_string(node_type, edges, method, beam_width, state_limit)
    if method == ONE_BY_ONE:
        # one node per step (not a maximal subset): replay the smallest-ready-id rule
        g = _Graph(node_type, edges)
        C, steps = g.start, [[v for v in range(V) if int(node_type[v]) == IN]]
        for _ in types:
            v = min(g.ready(C))
            steps.append([v])
            C |= 1 << v
        steps.append([v for v in range(V) if int(node_type[v]) == OUT])
    else:
        steps = steps_from_string(node_type, edges, types)
    step_of = np.empty(V, dtype=np.int64)
    for n, nodes in enumerate(steps):
        for v in nodes:
            step_of[v] = n
    perm = sorted(range(V), key=lambda v: (int(step_of[v]), v))
    pos = [0] * V
    for i, v in enumerate(perm):
        pos[v] = i
    step_ptr = [0]
    for nodes in steps:
        step_ptr.append(step_ptr[-1] + len(nodes))
    in_lists = [[] for _ in range(V)]
    out_lists = [[] for _ in range(V)]
    for e in range(E):  # original edge order
        s, d = int(edges[0, e]), int(edges[1, e])
        in_lists[d].append(pos[s])
        out_lists[s].append(pos[d])
    in_ptr, in_src, out_ptr, out_dst = [0], [], [0], []
    for v in perm:
        in_src += in_lists[v]
        in_ptr.append(len(in_src))
        out_dst += out_lists[v]
        out_ptr.append(len(out_dst))
    seen = [0] * NUM_TYPES
    row_of = [0] * V
    for v in range(V):
        row_of[v] = seen[int(node_type[v])]
        seen[int(node_type[v])] += 1
    param_row = [row_of[v] for v in perm]
    i32 = lambda a: np.asarray(a, dtype=np.int32)  # noqa: E731
    return Schedule(i32([IN] + types + [OUT]), i32(step_ptr), i32(perm), i32(in_ptr),
                    i32(in_src), i32(out_ptr), i32(out_dst), i32(param_row))
