"""The host C++ scheduler behind the C ABI against the oracle scheduler: every schedule array is
bit-equal for all four methods (paper Sec. 2 "Type scheduling"; Algorithm 1 preprocessing), the
error codes match, and the library exports every symbol its header declares. CPU only: these
calls never touch a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import schedule as osch
from paper_2408_03204_amd import (EXPORTS, GrafxError, Schedule, load, merge_graphs,
                                  schedule_many, set_schedule_threads)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
METHODS = [(osch.ONE_BY_ONE, "one_by_one"), (osch.GREEDY, "greedy"), (osch.BEAM, "beam"),
           (osch.OPTIMAL, "optimal")]


def assert_same(g, method_code, name, beam=32, limit=1 << 20):
    ref = osch.schedule(g.node_type, g.edges, method_code, beam_width=beam, state_limit=limit)
    got = Schedule(g.node_type, g.edges, name, beam_width=beam, state_limit=limit)
    for field in ("step_type", "step_ptr", "perm", "in_ptr", "in_src", "out_ptr", "out_dst",
                  "param_row"):
        a, b = getattr(ref, field), getattr(got, field)
        assert np.array_equal(a, b[:a.shape[0]]) and a.shape[0] == b.shape[0] or \
            (a.shape[0] == 0 and b.shape[0] == 0), (field, a, b)
    assert got.num_steps == ref.num_steps


def test_header_symbols_exported():
    header = open(os.path.join(ROOT, "include", "grafx.h")).read()
    declared = set(re.findall(r"^(?:grafx_status|void|int32_t|const char\*)\s+(grafx_\w+)\(", header,
                              re.M))
    assert declared == set(EXPORTS)
    lib = load()
    for name in declared:
        assert hasattr(lib, name)


@pytest.mark.parametrize("seed", range(60))
def test_bit_exact_random_dags(seed):
    rng = synth.rng_for(1000 + seed, 0)
    g = synth.random_dag(rng, int(rng.integers(3, 16)), types=(2, 3, 4, 5, 6), edge_p=0.3,
                         n_out=int(rng.integers(1, 3)))
    for code, name in METHODS:
        assert_same(g, code, name, beam=int(rng.integers(1, 6)))


@pytest.mark.parametrize("seed", range(10))
def test_bit_exact_larger_dags(seed):
    rng = synth.rng_for(2000 + seed, 0)
    g = synth.random_dag(rng, int(rng.integers(30, 80)), types=(2, 3, 4, 5, 6, 7, 8),
                         edge_p=0.08)
    for code, name in METHODS[:3]:
        assert_same(g, code, name, beam=32)


@pytest.mark.parametrize("seed", range(10))
def test_bit_exact_dags_with_noisegates(seed):
    rng = synth.rng_for(3000 + seed, 0)
    g = synth.random_dag(rng, int(rng.integers(8, 40)), types=(2, 3, 5, 9, 9), edge_p=0.15)
    assert (g.node_type == synth.GATE).any()
    for code, name in METHODS[:3]:
        assert_same(g, code, name, beam=8)


def test_noisegates_share_the_compressor_workspace():
    """Compressors and noisegates run one envelope scan and share its chunk state: relabelling
    every noisegate as a compressor leaves the workspace size unchanged."""
    rng = synth.rng_for(3100, 0)
    g = synth.random_dag(rng, 30, types=(2, 5, 9), edge_p=0.2)
    assert (g.node_type == synth.GATE).any() and (g.node_type == synth.COMP).any()
    relabelled = np.where(g.node_type == synth.GATE, synth.COMP, g.node_type).astype(np.int32)
    a, b = Schedule(g.node_type, g.edges), Schedule(relabelled, g.edges)
    for T in (1, 3072, 3073, 2 ** 17 + 5):
        for bwd in (False, True):
            assert a.workspace_bytes(T, bwd) == b.workspace_bytes(T, bwd)
    assert a.type_count[synth.GATE] == int((g.node_type == synth.GATE).sum())


def test_bit_exact_consoles():
    for w in (synth.tiny_console(T=8), synth.mixing_console(T=8), synth.large_console(T=8)):
        for code, name in METHODS[:3]:
            assert_same(w.graph, code, name)
    assert_same(synth.tiny_console(T=8).graph, osch.OPTIMAL, "optimal")


def _err(node_type, edges, **kw):
    with pytest.raises(GrafxError) as e:
        Schedule(np.asarray(node_type), np.asarray(edges), **kw)
    return e.value.status


def test_error_codes_match_oracle():
    assert _err([0, 3, 1, 3], [[0, 1, 3, 1], [1, 3, 1, 2]]) == "GRAFX_E_CYCLE"
    assert _err([0, 3, 1], [[0, 1, 1], [1, 2, 0]]) == "GRAFX_E_GRAPH"
    assert _err([0, 3, 1, 3], [[0, 1, 2], [1, 2, 3]]) == "GRAFX_E_GRAPH"
    assert _err([0, 3], [[0], [1]]) == "GRAFX_E_GRAPH"
    assert _err([0, 13, 1], [[0, 1], [1, 2]]) == "GRAFX_E_TYPE"
    assert _err([0, 3, 1], [[0, 1], [1, 2]], edge_type=np.ones((2, 2))) == "GRAFX_E_TYPE"
    assert _err([0, 3, 1], [[0, 1], [1, 7]]) == "GRAFX_E_GRAPH"
    assert _err([0, 3, 1], [[0, 1], [1, 2]], method="beam", beam_width=0) == "GRAFX_E_ARG"
    rng = synth.rng_for(7, 0)
    g = synth.random_dag(rng, 40, types=(2, 3, 4, 5, 6, 7, 8), edge_p=0.05)
    assert _err(g.node_type, g.edges, method="optimal", state_limit=3) == "GRAFX_E_LIMIT"
    with pytest.raises(osch.ScheduleError):
        osch.schedule(g.node_type, g.edges, osch.OPTIMAL, state_limit=3)


def test_no_processing_nodes_and_orphans():
    # inputs straight to outputs; a processing node without inputs; an unused input
    nt = np.array([0, 1, 3, 1, 0], dtype=np.int32)
    e = np.array([[0, 2], [1, 3]], dtype=np.int32)
    for code, name in METHODS:
        assert_same(synth.Graph(nt, e), code, name)
    s = Schedule(nt, e)
    assert s.type_string() == (0, 3, 1)
    s = Schedule(np.array([0, 1], dtype=np.int32), np.array([[0], [1]], dtype=np.int32))
    assert s.type_string() == (0, 1) and s.num_steps == 1


def test_workspace_bytes_grow_with_T():
    w = synth.mixing_console(T=8)
    s = Schedule(w.graph.node_type, w.graph.edges)
    a, b = s.workspace_bytes(2 ** 10, False), s.workspace_bytes(2 ** 18, False)
    assert 0 < a < b < s.workspace_bytes(2 ** 18, True)
    assert s.plan_bytes >= 4 * (2 * (w.graph.num_nodes + 1) + 2 * w.graph.num_edges)
    lib = load()
    n = ctypes.c_size_t()
    assert lib.grafx_workspace_bytes(s._h, 0, 0, ctypes.byref(n)) == 5  # T < 1: E_SHAPE


def test_tuning_settings():
    w = synth.tiny_console(T=8)
    s = Schedule(w.graph.node_type, w.graph.edges)
    assert s.get_tuning(Schedule.TUNE_POINTWISE_UNROLL) == 1
    assert s.get_tuning(Schedule.TUNE_AR_MAX_PASSES) == 16
    assert s.get_tuning(Schedule.TUNE_WAIT_POLLS) == 1 << 24
    before = s.workspace_bytes(3 * 2048 + 5, True)
    for v in (2, 4, 1):
        s.set_tuning(Schedule.TUNE_POINTWISE_UNROLL, v)
        assert s.get_tuning(Schedule.TUNE_POINTWISE_UNROLL) == v
        assert s.workspace_bytes(3 * 2048 + 5, True) == before  # sized for every setting
    for v in (1, 7, 16):
        s.set_tuning(Schedule.TUNE_AR_MAX_PASSES, v)
        assert s.get_tuning(Schedule.TUNE_AR_MAX_PASSES) == v
    for v in (0, 1, 1 << 30):
        s.set_tuning(Schedule.TUNE_WAIT_POLLS, v)
        assert s.get_tuning(Schedule.TUNE_WAIT_POLLS) == v
    assert s.get_tuning(Schedule.TUNE_EQ_ORDER) == 0
    assert s.get_tuning(Schedule.TUNE_DYN_ORDER) == 2
    assert s.get_tuning(Schedule.TUNE_TAP_TILES) == 16
    for knob, vals in ((Schedule.TUNE_EQ_ORDER, (1, 0)), (Schedule.TUNE_DYN_ORDER, (0, 1, 2)),
                       (Schedule.TUNE_TAP_TILES, (4, 8, 16))):
        for v in vals:
            s.set_tuning(knob, v)
            assert s.get_tuning(knob) == v
    assert s.workspace_bytes(3 * 2048 + 5, True) == before
    for knob, v in ((0, 3), (0, 0), (7, 1), (1, 0), (1, 17), (2, -1), (2, (1 << 30) + 1),
                    (3, 2), (3, -1), (4, 3), (4, -1), (5, 0), (5, 2), (5, 32), (6, 0)):
        with pytest.raises(GrafxError) as e:
            s.set_tuning(knob, v)
        assert e.value.status == "GRAFX_E_ARG"
    # a refused setting leaves the previous one in force
    assert s.get_tuning(Schedule.TUNE_AR_MAX_PASSES) == 16
    assert s.get_tuning(Schedule.TUNE_WAIT_POLLS) == 1 << 30


FIELDS = ("step_type", "step_ptr", "perm", "in_ptr", "in_src", "out_ptr", "out_dst", "param_row")


def _arrays(s):
    return [np.array(getattr(s, f)) for f in FIELDS]


def test_threaded_search_gives_the_serial_schedule():
    """A merged batch large enough for the beam search to split its depths over host threads
    (3,000+ processing nodes, 32 states): 1, 2, 3 and 8 threads give the same schedule bit for
    bit, at two beam widths (the children are merged in the serial order)."""
    ws = [synth.batched_graph(3, i, T_choices=(64,)) for i in range(24)]
    m = merge_graphs([(w.graph.node_type, w.graph.edges, w.T) for w in ws])
    assert sum(int(t) not in (synth.IN, synth.OUT) for t in m["node_type"]) >= 3000
    prev = set_schedule_threads(1)
    try:
        for width in (32, 5):
            set_schedule_threads(1)
            ref = _arrays(Schedule(m["node_type"], m["edges"], "beam", beam_width=width))
            for n in (2, 3, 8):
                set_schedule_threads(n)
                got = _arrays(Schedule(m["node_type"], m["edges"], "beam", beam_width=width))
                for f, a, b in zip(FIELDS, ref, got):
                    assert np.array_equal(a, b), (width, n, f)
    finally:
        set_schedule_threads(prev)


def test_schedule_threads_setting():
    prev = set_schedule_threads(3)
    try:
        assert set_schedule_threads(5) == 3
        assert load().grafx_set_schedule_threads(-1) == 5  # a query leaves it unchanged
        assert set_schedule_threads(0) == 5
        assert load().grafx_set_schedule_threads(-1) == 0
        with pytest.raises(ValueError):
            set_schedule_threads(-2)
    finally:
        set_schedule_threads(prev)


def test_schedule_many_matches_one_by_one():
    """Schedules computed concurrently on host threads equal the ones computed alone, in order,
    for graphs with and without per-node lengths."""
    graphs = []
    for i in range(6):
        w = synth.batched_graph(11, i, T_choices=(64,))
        graphs.append((w.graph.node_type, w.graph.edges))
    m = merge_graphs([(g[0], g[1], 32 + 8 * i) for i, g in enumerate(graphs[:3])])
    graphs.append((m["node_type"], m["edges"], m["lengths"]))
    many = schedule_many(graphs, "beam", workers=4)
    assert len(many) == len(graphs)
    for g, s in zip(graphs, many):
        alone = Schedule(g[0], g[1], "beam", lengths=g[2] if len(g) > 2 else None)
        for f, a, b in zip(FIELDS, _arrays(alone), _arrays(s)):
            assert np.array_equal(a, b), f


def test_concurrent_threaded_searches():
    """Several large searches at once, each splitting its depths over its own thread pool (four
    threads each, three searches on three host threads): every schedule equals the one computed
    alone on one thread."""
    merged = []
    for seed in (5, 6, 7):
        ws = [synth.batched_graph(seed, i, T_choices=(64,)) for i in range(20)]
        merged.append(merge_graphs([(w.graph.node_type, w.graph.edges, w.T) for w in ws]))
    prev = set_schedule_threads(1)
    try:
        alone = [_arrays(Schedule(m["node_type"], m["edges"], "beam")) for m in merged]
        set_schedule_threads(4)
        many = schedule_many([(m["node_type"], m["edges"]) for m in merged], "beam", workers=3)
        for ref, s in zip(alone, many):
            for f, a, b in zip(FIELDS, ref, _arrays(s)):
                assert np.array_equal(a, b), f
    finally:
        set_schedule_threads(prev)


def test_reverb_and_long_delay_schedule_like_the_oracle():
    """Graphs with the reverb (type 11) and the 2 s delay (type 12) get the oracle's schedule,
    read/write lists and parameter rows under every method."""
    for seed in range(4):
        w = synth.random_workload(1200 + seed, 12, 64, types=(synth.MIX, synth.REVERB,
                                                              synth.DELAY_LONG, synth.EQ,
                                                              synth.DELAY))
        for code, name in METHODS:
            assert_same(w.graph, code, name, beam=8)
