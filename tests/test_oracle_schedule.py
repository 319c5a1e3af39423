"""Pins of the oracle scheduler against what the paper fixes (Sec. 2 "Batched processing",
"Type scheduling"): partition, causality, homogeneity, V_0 = inputs, V_N = outputs, maximal
subsets; optimal = brute force; beam(1) = greedy; unbounded beam = optimal; the Fig. 1 example
length (|V| = 21, N = 9)."""
import numpy as np
import pytest

import synth
from oracle import schedule as osch

METHODS = [osch.ONE_BY_ONE, osch.GREEDY, osch.BEAM, osch.OPTIMAL]


def _preds(g):
    p = [set() for _ in range(g.num_nodes)]
    for s, d in g.edges.T:
        p[int(d)].add(int(s))
    return p


def _reachable(g):
    """reach[a] = set of nodes reachable from a by a non-empty path."""
    succ = [set() for _ in range(g.num_nodes)]
    for s, d in g.edges.T:
        succ[int(s)].add(int(d))
    reach = []
    for a in range(g.num_nodes):
        seen, stack = set(), list(succ[a])
        while stack:
            v = stack.pop()
            if v not in seen:
                seen.add(v)
                stack.extend(succ[v])
        reach.append(seen)
    return reach


def check_invariants(g, sch, maximal=True):
    V = g.num_nodes
    nt = g.node_type
    perm = sch.perm
    assert sorted(perm.tolist()) == list(range(V))  # partition
    step_of = np.empty(V, dtype=np.int64)
    N = sch.num_steps
    assert sch.step_ptr[0] == 0 and sch.step_ptr[-1] == V
    for n in range(N + 1):
        nodes = perm[sch.step_ptr[n]:sch.step_ptr[n + 1]]
        step_of[nodes] = n
        # homogeneous
        assert all(int(nt[v]) == int(sch.step_type[n]) for v in nodes)
        if 0 < n < N:
            assert len(nodes) > 0
        # nodes sorted by original id inside a step
        assert list(nodes) == sorted(nodes)
    # V_0 = all inputs, V_N = all outputs
    assert set(perm[sch.step_ptr[0]:sch.step_ptr[1]].tolist()) == set(np.flatnonzero(nt == 0))
    assert set(perm[sch.step_ptr[N]:sch.step_ptr[N + 1]].tolist()) == set(np.flatnonzero(nt == 1))
    # causal: no path from a node of step n to a node of step m <= n
    reach = _reachable(g)
    for a in range(V):
        for b in reach[a]:
            assert step_of[a] < step_of[b]
    # maximal (batched methods): no ready node of type t_n is left for later
    preds = _preds(g)
    done = set(perm[:sch.step_ptr[1]].tolist())
    for n in range(1, N):
        t = int(sch.step_type[n])
        nodes = set(perm[sch.step_ptr[n]:sch.step_ptr[n + 1]].tolist())
        ready_t = {v for v in range(V) if v not in done and int(nt[v]) == t and preds[v] <= done}
        if maximal:
            assert nodes == ready_t
        else:
            assert len(nodes) == 1 and nodes <= ready_t
        done |= nodes
    # index lists: in/out CSR and param rows
    pos = np.empty(V, dtype=np.int64)
    pos[perm] = np.arange(V)
    for i, v in enumerate(perm):
        ins = [int(pos[s]) for s, d in g.edges.T if d == v]
        outs = [int(pos[d]) for s, d in g.edges.T if s == v]
        assert sch.in_src[sch.in_ptr[i]:sch.in_ptr[i + 1]].tolist() == ins
        assert sch.out_dst[sch.out_ptr[i]:sch.out_ptr[i + 1]].tolist() == outs
        assert sch.param_row[i] == int(np.count_nonzero(nt[:v] == nt[v]))


def brute_force_optimal(g):
    """Every maximal-subset type string by exhaustive recursion (no pruning, no deduplication):
    the shortest, then the lexicographically smallest."""
    nt = [int(t) for t in g.node_type]
    preds = _preds(g)
    proc = [v for v in range(g.num_nodes) if nt[v] not in (0, 1)]
    best = [None]

    def rec(done, s):
        if best[0] is not None and len(s) > len(best[0]):
            return
        left = [v for v in proc if v not in done]
        if not left:
            if best[0] is None or (len(s), s) < (len(best[0]), best[0]):
                best[0] = s
            return
        ready = [v for v in left if preds[v] <= done]
        for t in sorted({nt[v] for v in ready}):
            rec(done | {v for v in ready if nt[v] == t}, s + (t,))

    rec({v for v in range(g.num_nodes) if nt[v] == 0}, ())
    return list(best[0])


@pytest.mark.parametrize("seed", range(40))
def test_invariants_random(seed):
    rng = synth.rng_for(100 + seed, 0)
    g = synth.random_dag(rng, int(rng.integers(3, 14)), types=(2, 3, 4, 5), edge_p=0.35,
                         n_out=int(rng.integers(1, 3)))
    for m in METHODS:
        sch = osch.schedule(g.node_type, g.edges, m, beam_width=4)
        check_invariants(g, sch, maximal=m != osch.ONE_BY_ONE)


@pytest.mark.parametrize("seed", range(60))
def test_optimal_is_brute_force(seed):
    rng = synth.rng_for(200 + seed, 0)
    g = synth.random_dag(rng, int(rng.integers(4, 13)), types=(2, 3, 4, 5), edge_p=0.3)
    opt = osch.type_string(g.node_type, g.edges, osch.OPTIMAL)
    assert opt == brute_force_optimal(g)


@pytest.mark.parametrize("seed", range(40))
def test_beam_limits_and_order(seed):
    rng = synth.rng_for(300 + seed, 0)
    g = synth.random_dag(rng, int(rng.integers(6, 30)), types=(2, 3, 4, 5, 6), edge_p=0.2)
    greedy = osch.type_string(g.node_type, g.edges, osch.GREEDY)
    beam1 = osch.type_string(g.node_type, g.edges, osch.BEAM, beam_width=1)
    assert beam1 == greedy
    opt = osch.type_string(g.node_type, g.edges, osch.OPTIMAL)
    wide = osch.type_string(g.node_type, g.edges, osch.BEAM, beam_width=10 ** 6)
    assert wide == opt
    b4 = osch.type_string(g.node_type, g.edges, osch.BEAM, beam_width=4)
    obo = osch.type_string(g.node_type, g.edges, osch.ONE_BY_ONE)
    n_proc = int(np.count_nonzero(g.node_type >= 2))
    assert len(opt) <= len(b4) <= n_proc
    assert len(opt) <= len(greedy) <= len(obo) == n_proc


def fig1_like_graph():
    """21 nodes: four tracks (e-c-g-d, e-c-g, e-g-d, c-d) into a mix, then e-g-d and the output.
    The paper's Fig. 1 graph is an image that is not available; this graph is built to have the
    same size and the same optimal string shape (i e c g r m e g r o, with the delay standing
    in for the reverb), i.e. N = 9 processing calls for |V| = 21."""
    b = synth.GraphBuilder()
    E, C, G, D, M = synth.EQ, synth.COMP, synth.GAIN_PAN, synth.DELAY, synth.MIX
    ends = []
    for chain in ([E, C, G, D], [E, C, G], [E, G, D], [C, D]):
        i = b.add(synth.IN)
        a, z = b.chain(chain)
        b.connect(i, a)
        ends.append(z)
    m, _ = b.chain([M, E, G, D, synth.OUT])
    for z in ends:
        b.connect(z, m)
    return b.build()


def test_fig1_example_length():
    g = fig1_like_graph()
    assert g.num_nodes == 21
    sch = osch.schedule(g.node_type, g.edges, osch.OPTIMAL)
    assert sch.num_steps == 9
    E, C, G, D, M = synth.EQ, synth.COMP, synth.GAIN_PAN, synth.DELAY, synth.MIX
    assert sch.type_string() == (0, E, C, G, D, M, E, G, D, 1)
    check_invariants(g, sch)
    obo = osch.schedule(g.node_type, g.edges, osch.ONE_BY_ONE)
    assert obo.num_steps == 21 - 4 - 1 + 1


def test_consoles_schedule():
    for w in (synth.tiny_console(T=8), synth.mixing_console(T=8)):
        for m in (osch.GREEDY, osch.BEAM, osch.ONE_BY_ONE):
            check_invariants(w.graph, osch.schedule(w.graph.node_type, w.graph.edges, m),
                             maximal=m != osch.ONE_BY_ONE)
    w = synth.tiny_console(T=8)
    s = osch.schedule(w.graph.node_type, w.graph.edges, osch.OPTIMAL)
    assert s.type_string() == (0, 3, 4, 5, 2, 3, 1)


def test_errors():
    ok_t = np.array([0, 3, 1], dtype=np.int32)
    ok_e = np.array([[0, 1], [1, 2]], dtype=np.int32)
    osch.schedule(ok_t, ok_e)
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(np.array([0, 3, 1, 3]), np.array([[0, 1, 3, 1], [1, 3, 1, 2]]))
    assert e.value.kind == "cycle"
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(ok_t, np.array([[0, 1, 1], [1, 2, 0]]))
    assert e.value.kind == "graph"  # edge into an input
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(np.array([0, 3, 1, 3]), np.array([[0, 1, 2], [1, 2, 3]]))
    assert e.value.kind == "graph"  # edge out of an output
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(np.array([0, 3]), np.array([[0], [1]]))
    assert e.value.kind == "graph"  # no output
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(np.array([0, 13, 1]), ok_e)
    assert e.value.kind == "type"
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(ok_t, ok_e, edge_type=np.ones((2, 2)))
    assert e.value.kind == "type"
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(ok_t, np.array([[0, 1], [1, 7]]))
    assert e.value.kind == "graph"
    rng = synth.rng_for(7, 0)
    g = synth.random_dag(rng, 40, types=(2, 3, 4, 5, 6, 7, 8), edge_p=0.05)
    with pytest.raises(osch.ScheduleError) as e:
        osch.schedule(g.node_type, g.edges, osch.OPTIMAL, state_limit=3)
    assert e.value.kind == "limit"
