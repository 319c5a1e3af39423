"""Seeded synthetic workloads for the audio-graph renderer: graphs, sources, parameters.

This module only draws random numbers and lays out graph structure. It holds none of the
rendering method's arithmetic, so that both the FP64 oracle and the HIP path can consume the
same arrays. Every array is produced once, in float32, and handed to both sides unchanged.

Node type codes (shared interface, also fixed in the C header):
    0 in, 1 out, 2 mix, 3 gain_pan, 4 eq, 5 compressor, 6 imager, 7 delay, 8 tanh

Graph tensors follow the paper's representation (Sec. 2, "Graph representations"): a node type
vector, a 2 x |E| edge index (row 0 source, row 1 destination), one parameter matrix per type
whose l-th row belongs to the l-th node of that type in node order, and a source tensor
[K, C, L] whose k-th entry feeds the k-th `in` node.

The workloads are stand-ins for the paper's mixing consoles (Sec. 4, Fig. 2b); the paper's own
graphs and audio are not available, so every input here is synthetic and seeded.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FS = 44100

IN, OUT, MIX, GAIN_PAN, EQ, COMP, IMAGER, DELAY, TANH, GATE, COMP_AR, REVERB, DELAY_LONG = \
    range(13)
TYPE_NAMES = ("in", "out", "mix", "gain_pan", "eq", "compressor", "imager", "delay", "tanh",
              "noisegate", "compressor_ar", "reverb", "delay_long")
NUM_TYPES = len(TYPE_NAMES)
TYPE_CODES = {n: i for i, n in enumerate(TYPE_NAMES)}
# parameters per node of each type (0 for in/out/mix)
N_PARAMS = (0, 0, 0, 2, 1024, 4, 1, 220, 1, 4, 5, 768, 880)
# reverb: noise realisation of 2 s (mid, side); parameters [mid, side][H0, HD][192 bins]
REVERB_LEN = 2 * FS
REVERB_BINS = 192
REVERB_HOP = 192

# delay layout: [channel 2][slot M][re z, im z, 20 log-magnitudes]; M = 5 (delay, 500 ms) or
# M = 20 (delay_long, 2 s)
DELAY_TAPS = 5
DELAY_TAPS_LONG = 20
DELAY_SLOT = 4410  # 100 ms at 44.1 kHz
DELAY_BINS = 20

# random streams
S_STRUCT, S_SOURCE, S_PARAM, S_TARGET, S_ADJOINT, S_NOISE = 0, 1, 2, 3, 4, 5


def rng_for(seed: int, stream: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, index])))


@dataclasses.dataclass
class Graph:
    node_type: np.ndarray  # int32 [V]
    edges: np.ndarray  # int32 [2, E]

    @property
    def num_nodes(self) -> int:
        return int(self.node_type.shape[0])

    @property
    def num_edges(self) -> int:
        return int(self.edges.shape[1])

    def count(self, t: int) -> int:
        return int(np.count_nonzero(self.node_type == t))


class GraphBuilder:
    """Append-only node/edge lists; node ids are assigned in insertion order."""

    def __init__(self):
        self.types: list[int] = []
        self.src: list[int] = []
        self.dst: list[int] = []

    def add(self, t: int) -> int:
        self.types.append(int(t))
        return len(self.types) - 1

    def chain(self, types) -> tuple[int, int]:
        ids = [self.add(t) for t in types]
        for a, b in zip(ids[:-1], ids[1:]):
            self.connect(a, b)
        return ids[0], ids[-1]

    def connect(self, a: int, b: int) -> None:
        self.src.append(int(a))
        self.dst.append(int(b))

    def build(self) -> Graph:
        return Graph(np.asarray(self.types, dtype=np.int32),
                     np.asarray([self.src, self.dst], dtype=np.int32).reshape(2, -1))


# ---------------------------------------------------------------------------------------------
# sources

def make_sources(rng: np.random.Generator, K: int, T: int) -> np.ndarray:
    """White noise U[-1,1) per channel times a decaying envelope that restarts at Poisson onsets
    (4 per second plus one at t=0): amplitude U[0.05, 0.5], decay constant U[30, 500] ms.
    |s| <= 0.5 everywhere."""
    out = np.empty((K, 2, T), dtype=np.float32)
    t = np.arange(T, dtype=np.float64)
    for k in range(K):
        noise = rng.uniform(-1.0, 1.0, size=(2, T))
        n_on = rng.poisson(4.0 * T / FS)
        onsets = np.sort(np.concatenate([[0], rng.integers(0, max(T, 1), size=n_on)]))
        amp = rng.uniform(0.05, 0.5, size=onsets.shape[0])
        tau = rng.uniform(0.030, 0.500, size=onsets.shape[0]) * FS
        idx = np.searchsorted(onsets, t, side="right") - 1
        env = amp[idx] * np.exp(-(t - onsets[idx]) / tau[idx])
        out[k] = (noise * env[None, :]).astype(np.float32)
    return out


# ---------------------------------------------------------------------------------------------
# parameters (physical units as the renderer takes them)

LN10_20 = math.log(10.0) / 20.0  # dB (amplitude) -> natural log
LN10_10 = math.log(10.0) / 10.0  # dB (energy) -> natural log


def gain_pan_params(rng, n):
    return (rng.uniform(-12.0, 6.0, size=(n, 2)) * LN10_20).astype(np.float32)


def imager_params(rng, n):
    return (rng.uniform(-12.0, 6.0, size=(n, 1)) * LN10_20).astype(np.float32)


def tanh_params(rng, n):
    return (rng.uniform(0.0, 24.0, size=(n, 1)) * LN10_20).astype(np.float32)


def eq_params(rng, n, bands=6):
    """Six band gains U[-12,12] dB at log-spaced centres 20*1000^((b+0.5)/6) Hz, spread over the
    1024 log-magnitude bins (bin k at k*fs/2047 Hz) by linear interpolation in log-frequency,
    constant beyond the outer centres."""
    centres = 20.0 * 1000.0 ** ((np.arange(bands) + 0.5) / bands)
    f = np.arange(1024) * FS / 2047.0
    lf = np.log(np.maximum(f, 1e-3))
    out = np.empty((n, 1024), dtype=np.float32)
    for i in range(n):
        gains = rng.uniform(-12.0, 12.0, size=bands)
        out[i] = (np.interp(lf, np.log(centres), gains) * LN10_20).astype(np.float32)
    return out


def comp_params(rng, n, knee_db=3.0):
    """(alpha, T, W, R): one shared attack/release constant U[1,100] ms, threshold U[-30,-10] dB,
    knee half-width 3 dB, ratio U[2,8]. T and W are in natural-log energy units."""
    tau = rng.uniform(1e-3, 100e-3, size=n)
    alpha = np.exp(-1.0 / (tau * FS))
    thr = rng.uniform(-30.0, -10.0, size=n) * LN10_10
    knee = np.full(n, knee_db * LN10_10)
    ratio = rng.uniform(2.0, 8.0, size=n)
    return np.stack([alpha, thr, knee, ratio], axis=1).astype(np.float32)


def comp_ar_params(rng, n, knee_db=3.0):
    """(alpha_a, alpha_r, T, W, R): attack and release time constants U[1,100] ms each,
    threshold U[-30,-10] dB, knee half-width 3 dB, ratio U[2,8]."""
    tau = rng.uniform(1e-3, 100e-3, size=(n, 2))
    alpha = np.exp(-1.0 / (tau * FS))
    thr = rng.uniform(-30.0, -10.0, size=n) * LN10_10
    knee = np.full(n, knee_db * LN10_10)
    ratio = rng.uniform(2.0, 8.0, size=n)
    return np.stack([alpha[:, 0], alpha[:, 1], thr, knee, ratio], axis=1).astype(np.float32)


def gate_params(rng, n, knee_db=3.0):
    """Noisegate (alpha, T, W, R): time constant U[1,100] ms, threshold U[-50,-30] dB, knee
    half-width 3 dB, expansion ratio U[2,8]. T and W are in natural-log energy units."""
    tau = rng.uniform(1e-3, 100e-3, size=n)
    alpha = np.exp(-1.0 / (tau * FS))
    thr = rng.uniform(-50.0, -30.0, size=n) * LN10_10
    knee = np.full(n, knee_db * LN10_10)
    ratio = rng.uniform(2.0, 8.0, size=n)
    return np.stack([alpha, thr, knee, ratio], axis=1).astype(np.float32)


def delay_params(rng, n, max_ms=500.0, slots=None):
    """Per channel and 100 ms slot: an integer delay inside the slot encoded as a unit phasor
    z = exp(-2 pi i d / 4410), and 20 log-magnitudes for the slot's 39-tap filter: a flat level
    U[-24,-6] dB plus +-3 dB ripple per bin. `slots`: 5 (the 500 ms delay, default) or 20 (the
    2 s delay); slots past `max_ms` are silenced (-120 dB)."""
    M = slots or DELAY_TAPS
    taps = min(M, int(round(max_ms / 100.0)))
    out = np.zeros((n, 2, M, 2 + DELAY_BINS), dtype=np.float64)
    for i in range(n):
        for c in range(2):
            for m in range(M):
                d = int(rng.integers(0, DELAY_SLOT))
                ph = -2.0 * math.pi * d / DELAY_SLOT
                out[i, c, m, 0] = math.cos(ph)
                out[i, c, m, 1] = math.sin(ph)
                level = rng.uniform(-24.0, -6.0) if m < taps else -120.0
                out[i, c, m, 2:] = (level + rng.uniform(-3.0, 3.0, size=DELAY_BINS)) * LN10_20
    return out.reshape(n, 2 * M * (2 + DELAY_BINS)).astype(np.float32)


def delay_long_params(rng, n, max_ms=2000.0):
    """The 2 s delay (20 slots per channel), drawn like `delay_params`."""
    return delay_params(rng, n, max_ms, slots=DELAY_TAPS_LONG)


def reverb_params(rng, n):
    """Mid and side masks of the filtered-noise reverb, per one-sided bin k (k fs / 384 Hz) of
    the 384-point STFT: initial colouration H0 = a level U[-40, -30] dB (mid; side 3 to 9 dB
    lower) plus +-3 dB per six log-spaced bands, interpolated like the EQ; decay per 192-sample
    frame HD = -ln(1000) 192 / (fs RT60(f)) with RT60(f) = RT60_0 / (1 + f / 8 kHz) and
    RT60_0 U[0.3, 1.5] s (60 dB of decay over RT60). Natural-log units."""
    f = np.arange(REVERB_BINS) * FS / 384.0
    centres = 20.0 * 1000.0 ** ((np.arange(6) + 0.5) / 6)
    lf = np.log(np.maximum(f, 1e-3))
    out = np.empty((n, 2, 2, REVERB_BINS), dtype=np.float64)
    for i in range(n):
        level = rng.uniform(-40.0, -30.0)
        rt0 = rng.uniform(0.3, 1.5)
        for x in range(2):
            lv = level - (rng.uniform(3.0, 9.0) if x == 1 else 0.0)
            ripple = np.interp(lf, np.log(centres), rng.uniform(-3.0, 3.0, size=6))
            out[i, x, 0] = (lv + ripple) * LN10_20
            rt = rt0 * rng.uniform(0.9, 1.1) / (1.0 + f / 8000.0)
            out[i, x, 1] = -math.log(1000.0) * REVERB_HOP / (FS * rt)
    return out.reshape(n, 4 * REVERB_BINS).astype(np.float32)


def reverb_noise(seed: int, length: int = REVERB_LEN) -> np.ndarray:
    """The reverb's noise realisation [2, length] (mid, side): uniform in [-1, 1)."""
    return rng_for(seed, S_NOISE).uniform(-1.0, 1.0, size=(2, length)).astype(np.float32)


PARAM_DRAW = {GAIN_PAN: gain_pan_params, EQ: eq_params, COMP: comp_params,
              IMAGER: imager_params, DELAY: delay_params, TANH: tanh_params, GATE: gate_params,
              COMP_AR: comp_ar_params, REVERB: reverb_params, DELAY_LONG: delay_long_params}


def draw_params(rng: np.random.Generator, graph: Graph) -> dict[int, np.ndarray]:
    """One parameter matrix per processor type present, rows in node order."""
    out = {}
    for t in range(NUM_TYPES):
        if N_PARAMS[t] == 0:
            continue
        out[t] = PARAM_DRAW[t](rng, graph.count(t)).reshape(graph.count(t), N_PARAMS[t])
    return out


def default_params(graph: Graph) -> dict[int, np.ndarray]:
    """Neutral settings: unit gains, flat EQ, ratio-1 compressor, zero drive."""
    out = {}
    for t in range(NUM_TYPES):
        if N_PARAMS[t] == 0:
            continue
        n = graph.count(t)
        p = np.zeros((n, N_PARAMS[t]), dtype=np.float32)
        if t in (COMP, GATE):
            p[:, 0] = math.exp(-1.0 / (0.010 * FS))
            p[:, 1] = (-20.0 if t == COMP else -40.0) * LN10_10
            p[:, 2] = 3.0 * LN10_10
            p[:, 3] = 1.0
        elif t == COMP_AR:
            p[:, 0:2] = math.exp(-1.0 / (0.010 * FS))
            p[:, 2] = -20.0 * LN10_10
            p[:, 3] = 3.0 * LN10_10
            p[:, 4] = 1.0
        elif t == REVERB:  # -40 dB, about 1 s of decay (60 dB)
            p.reshape(n, 2, 2, REVERB_BINS)[:, :, 0] = -40.0 * LN10_20
            p.reshape(n, 2, 2, REVERB_BINS)[:, :, 1] = -math.log(1000.0) * REVERB_HOP / FS
        out[t] = p
    return out


# ---------------------------------------------------------------------------------------------
# graphs

CHAIN_POOL_C2 = (EQ, COMP, GAIN_PAN, IMAGER)
CHAIN_POOL_C3 = (EQ, COMP, GAIN_PAN, IMAGER, DELAY, TANH)


def _track_chains(rng, n_tracks, pool, kmin, kmax):
    chains = []
    for _ in range(n_tracks):
        k = int(rng.integers(kmin, kmax + 1))
        perm = rng.permutation(len(pool))
        chains.append([pool[i] for i in perm[:k]])
    return chains


def console_graph(rng, n_tracks: int, bus_levels: list[int], pool=CHAIN_POOL_C2, kmin=1,
                  kmax=3, master_chain=(EQ, COMP, GAIN_PAN), track_tail=()) -> Graph:
    """Mixing console: per track in -> random processor chain (+ `track_tail`) -> level-1 bus;
    each bus is mix -> eq -> compressor; buses feed the next level; the master is
    mix -> master_chain -> out. `bus_levels` lists the bus count per level (top level last)."""
    g = GraphBuilder()
    ends = []
    for chain in _track_chains(rng, n_tracks, pool, kmin, kmax):
        chain = chain + list(track_tail)
        i = g.add(IN)
        if chain:
            a, b = g.chain(chain)
            g.connect(i, a)
            ends.append(b)
        else:
            ends.append(i)
    for n_bus in bus_levels:
        order = rng.permutation(len(ends))
        groups = np.array_split(order, n_bus)
        new_ends = []
        for grp in groups:
            m, e = g.chain([MIX, EQ, COMP])
            for j in sorted(int(x) for x in grp):
                g.connect(ends[j], m)
            new_ends.append(e)
        ends = new_ends
    m, e = g.chain([MIX, *master_chain, OUT])
    for j in ends:
        g.connect(j, m)
    return g.build()


@dataclasses.dataclass
class Workload:
    name: str
    graph: Graph
    sources: np.ndarray  # float32 [K, 2, T]
    params: dict  # type -> float32 [n_t, N_t]
    target_params: dict | None
    T: int
    seed: int
    reverb_noise: np.ndarray | None = None  # [2, L] float32 when the graph has reverb nodes

    @property
    def processed_nodes(self) -> int:
        return self.graph.num_nodes - self.graph.count(IN)


def tiny_console(seed=1, T=2 ** 15, attack_release=False) -> Workload:
    """4 sources, each in -> gain_pan -> eq -> compressor, into one mix -> gain_pan -> out.
    With `attack_release` the compressors have distinct attack and release times."""
    g = GraphBuilder()
    ends = []
    for _ in range(4):
        i = g.add(IN)
        a, b = g.chain([GAIN_PAN, EQ, COMP_AR if attack_release else COMP])
        g.connect(i, a)
        ends.append(b)
    m, _ = g.chain([MIX, GAIN_PAN, OUT])
    for e in ends:
        g.connect(e, m)
    graph = g.build()
    return Workload("tiny_console_4src" + ("_ar" if attack_release else ""), graph, make_sources(rng_for(seed, S_SOURCE), 4, T),
                    draw_params(rng_for(seed, S_PARAM), graph),
                    draw_params(rng_for(seed, S_TARGET), graph), T, seed)


# ---------------------------------------------------------------------------------------------
# labelled tiny consoles (training and evaluation data of the learned initialiser)

LABEL_RANGES = [(-12.0, 6.0), (-12.0, 6.0)] + [(-12.0, 12.0)] * 6 + [(1.0, 100.0),
                                                                   (-30.0, -10.0), (2.0, 8.0)]
N_LABELS = len(LABEL_RANGES)


def eq_from_bands(band_db: np.ndarray) -> np.ndarray:
    """Six band gains (dB) -> 1024 log-magnitudes, the rule of `eq_params`."""
    centres = 20.0 * 1000.0 ** ((np.arange(6) + 0.5) / 6)
    f = np.arange(1024) * FS / 2047.0
    lf = np.log(np.maximum(f, 1e-3))
    return np.interp(lf, np.log(centres), band_db) * LN10_20


def track_params_from_labels(u: np.ndarray) -> tuple:
    """Labels in [0, 1]^11 -> (gain_pan [2], eq [1024], compressor [4]) rows: gain/pan dB per
    channel [-12, 6], six EQ band gains [-12, 12] dB, compressor time constant [1, 100] ms,
    threshold [-30, -10] dB, ratio [2, 8], knee 3 dB."""
    v = [lo + (hi - lo) * float(x) for x, (lo, hi) in zip(u, LABEL_RANGES)]
    gp = np.array(v[0:2]) * LN10_20
    eq = eq_from_bands(np.array(v[2:8]))
    comp = np.array([math.exp(-1.0 / (v[8] * 1e-3 * FS)), v[9] * LN10_10, 3.0 * LN10_10, v[10]])
    return gp, eq, comp


def labelled_tiny_consoles(seed: int, count: int, T: int = 2 ** 15, first: int = 0):
    """`count` tiny consoles (4 tracks of gain_pan -> eq -> compressor, mix, master gain_pan,
    out), console i drawn from its own streams: sources as `make_sources`, per-track labels
    U[0, 1]^11 mapped by `track_params_from_labels`, master gain U[-12, 6] dB per channel.
    Consoles `first` .. `first + count - 1` of the seed. Returns (workloads, labels
    [count, 4, 11]); each workload's `params` are the drawn ones, its `target_params` None."""
    g = tiny_console(T=8).graph
    out, labels = [], np.empty((count, 4, N_LABELS))
    for n in range(count):
        i = first + n
        rng = rng_for(seed, S_PARAM, i)
        u = rng.uniform(0.0, 1.0, size=(4, N_LABELS))
        labels[n] = u
        rows = [track_params_from_labels(x) for x in u]
        params = default_params(g)
        params[GAIN_PAN] = np.concatenate(
            [np.stack([r[0] for r in rows]),
             rng.uniform(-12.0, 6.0, size=(1, 2)) * LN10_20]).astype(np.float32)
        params[EQ] = np.stack([r[1] for r in rows]).astype(np.float32)
        params[COMP] = np.stack([r[2] for r in rows]).astype(np.float32)
        out.append(Workload(f"labelled_tiny_{i}", g, make_sources(rng_for(seed, S_SOURCE, i), 4,
                                                                    T), params, None, T, seed))
    return out, labels


def encoder_weights(seed: int = 0) -> np.ndarray:
    """Initial weights of the learned initialiser's encoder as one flat float32 vector, layout
    [W1 (64 x 256 x 5), b1 (64), W2 (64 x 64 x 5), b2, ..., W6, b6, Wh (11 x 64), bh (11)]:
    He-uniform weights (bound sqrt(6 / fan_in)), Glorot-uniform head, zero biases."""
    rng = rng_for(seed, S_PARAM, 99)
    parts, c_in = [], 256
    for _ in range(6):
        bound = math.sqrt(6.0 / (c_in * 5))
        parts += [rng.uniform(-bound, bound, 64 * c_in * 5), np.zeros(64)]
        c_in = 64
    bound = math.sqrt(6.0 / (64 + 11))
    parts += [rng.uniform(-bound, bound, 11 * 64), np.zeros(11)]
    return np.concatenate(parts).astype(np.float32)


def mixing_console(seed=2, T=2 ** 18, n_tracks=64, n_bus=8, attack_release=False) -> Workload:
    """64 tracks with chains of 1-3 from {eq, compressor, gain_pan, imager}, 8 buses of
    mix -> eq -> compressor, master mix -> eq -> compressor -> gain_pan -> out. With
    `attack_release` every compressor has distinct attack and release times (same graph)."""
    graph = console_graph(rng_for(seed, S_STRUCT), n_tracks, [n_bus])
    if attack_release:
        graph = Graph(np.where(graph.node_type == COMP, COMP_AR, graph.node_type).astype(np.int32),
                      graph.edges)
    K = graph.count(IN)
    return Workload(f"mixing_console_{n_tracks}trk" + ("_ar" if attack_release else ""), graph,
                    make_sources(rng_for(seed, S_SOURCE), K, T),
                    draw_params(rng_for(seed, S_PARAM), graph),
                    draw_params(rng_for(seed, S_TARGET), graph), T, seed)


def large_console(seed=5, T=2 ** 20, n_tracks=256) -> Workload:
    """256 tracks (chains as in the 64-track console), bus tree 32 -> 8 -> 2 -> master."""
    graph = console_graph(rng_for(seed, S_STRUCT), n_tracks, [32, 8, 2])
    K = graph.count(IN)
    return Workload(f"large_console_{n_tracks}trk", graph,
                    make_sources(rng_for(seed, S_SOURCE), K, T),
                    draw_params(rng_for(seed, S_PARAM), graph),
                    draw_params(rng_for(seed, S_TARGET), graph), T, seed)


def reverb_console(seed=3, T=2 ** 18, n_tracks=64, n_bus=8) -> Workload:
    """The 64-track console with a reverb closing every track chain (64 reverbs, 2 s noise)."""
    graph = console_graph(rng_for(seed, S_STRUCT), n_tracks, [n_bus], track_tail=(REVERB,))
    K = graph.count(IN)
    return Workload(f"reverb_console_{n_tracks}trk", graph,
                    make_sources(rng_for(seed, S_SOURCE), K, T),
                    draw_params(rng_for(seed, S_PARAM), graph),
                    draw_params(rng_for(seed, S_TARGET), graph), T, seed,
                    reverb_noise(seed))


def output_adjoint(seed: int, n_out: int, T: int) -> np.ndarray:
    """Seeded output adjoint dY [n_out, 2, T] (standard normal, float32) for parity of the
    render's adjoint: the gradient of sum(dY * Y)."""
    return rng_for(seed, S_ADJOINT).standard_normal((n_out, 2, T), dtype=np.float32)


def batched_graph(seed: int, index: int, T_choices=(2 ** 16, 2 ** 17, 2 ** 18),
                  src_range=(8, 96)) -> Workload:
    """One graph of the batched uneven-graph workload: K ~ U{8..96} sources, per-track chains of
    0-4 distinct processors from {eq, compressor, gain_pan, imager, delay, tanh}, a bus tree of
    depth 1-3 (ceil(K/8) level-1 buses, then ceil(n/4) per further level, each bus
    mix -> eq -> compressor), master mix -> eq -> compressor -> gain_pan -> out, and its own
    T drawn from `T_choices`. Graph `index` of seed `seed` uses its own generator streams."""
    rng = rng_for(seed, S_STRUCT, index)
    K = int(rng.integers(src_range[0], src_range[1] + 1))
    depth = int(rng.integers(1, 4))
    levels = [-(-K // 8)]
    for _ in range(depth - 1):
        levels.append(-(-levels[-1] // 4))
    graph = console_graph(rng, K, levels, pool=CHAIN_POOL_C3, kmin=0, kmax=4)
    T = int(T_choices[int(rng.integers(0, len(T_choices)))])
    return Workload(f"batched_{seed}_{index}", graph,
                    make_sources(rng_for(seed, S_SOURCE, index), K, T),
                    draw_params(rng_for(seed, S_PARAM, index), graph), None, T, seed)


def batched_graphs(count: int = 128, seed: int = 7, **kw) -> list[Workload]:
    """`count` graphs of the batched uneven-graph workload (see `batched_graph`)."""
    return [batched_graph(seed, i, **kw) for i in range(count)]


def random_dag(rng, n_nodes: int, types=(MIX, GAIN_PAN, EQ, COMP), edge_p: float = 0.3,
               n_in: int | None = None, n_out: int = 1, multi: bool = True,
               allow_orphans: bool = True) -> Graph:
    """A random DAG: `n_in` inputs, `n_out` outputs and processing nodes whose types are drawn
    from `types`. Edges only go forward in a hidden topological order (inputs first, outputs
    last); about 10 % of edges are doubled (parallel edges) when `multi`. Every output gets at
    least one predecessor; processing nodes may have none unless `allow_orphans` is False.
    Node ids and edge order are then shuffled so that neither reveals the hidden order."""
    if n_in is None:
        n_in = int(rng.integers(1, 4))
    n_proc = max(n_nodes - n_in - n_out, 0)
    kinds = [IN] * n_in + [int(types[rng.integers(0, len(types))]) for _ in range(n_proc)] \
        + [OUT] * n_out
    src, dst = [], []
    for b in range(n_in, len(kinds)):
        has_pred = False
        for a in range(0, min(b, n_in + n_proc)):
            if rng.random() < edge_p:
                src.append(a)
                dst.append(b)
                has_pred = True
                if multi and rng.random() < 0.1:
                    src.append(a)
                    dst.append(b)
        if not has_pred and (kinds[b] == OUT or not allow_orphans) and min(b, n_in + n_proc) > 0:
            src.append(int(rng.integers(0, min(b, n_in + n_proc))))
            dst.append(b)
    relabel = rng.permutation(len(kinds))
    node_type = np.empty(len(kinds), dtype=np.int32)
    for old, new in enumerate(relabel):
        node_type[new] = kinds[old]
    e = np.array([[relabel[s] for s in src], [relabel[d] for d in dst]], dtype=np.int64)
    e = e.reshape(2, -1)
    if e.shape[1]:
        e = e[:, rng.permutation(e.shape[1])]
    return Graph(node_type, e.astype(np.int32))


def random_workload(seed: int, n_nodes: int, T: int, types=(MIX, GAIN_PAN, EQ, COMP, IMAGER,
                    DELAY, TANH), edge_p=0.3, n_in=None, n_out=1, multi=True,
                    allow_orphans=False) -> Workload:
    """Random DAG (see `random_dag`) with seeded sources and parameters."""
    graph = random_dag(rng_for(seed, S_STRUCT), n_nodes, types, edge_p, n_in, n_out, multi,
                       allow_orphans)
    K = graph.count(IN)
    return Workload(f"random_{n_nodes}", graph, make_sources(rng_for(seed, S_SOURCE), K, T),
                    draw_params(rng_for(seed, S_PARAM), graph),
                    draw_params(rng_for(seed, S_TARGET), graph), T, seed)
