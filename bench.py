"""Benchmark: node-samples/s of one gradient step of a mixing-console graph on one MI355X.

A step is the whole hot path on one batch: the batched forward render of the graph, the
3-resolution STFT loss against a target mix rendered with hidden parameters, the loss adjoint
and the render adjoint down to every processor parameter. The default workload is the largest
single-GPU one, the 256-track console (bus tree 32 -> 8 -> 2 -> master, 904 nodes, T = 2^20);
`--workload console` is the 64-track console at T = 2^18. Throughput = processed (non-input)
nodes x T / step time, with every input already resident in HBM. All inputs are seeded
synthetic stand-ins for the paper's consoles.

Prints one JSON line with, besides the metric, the HBM roofline of the dominant step kernel
(its algorithmic bytes per launch / its event-timed launch duration, measured here, against
8 TB/s; for the FFT- and FIR-bound kernels also their flop rate against the FP32 vector issue
rate as a second view) and the FP64 CPU oracle timed on a bounded sample of the same workload
with one thread and with every host thread.

The timed step is issued as one HIP-graph replay of the whole step (default: `--mode graph`,
captured once from the same C-ABI calls); `--mode eager` issues those calls one by one and
`--mode autograd` goes through torch.autograd. All three are timed and listed in
`ms_per_step_by_issue`; the reported value is the selected one.

    python bench.py [--steps K] [--warmup W] [--workload console|tiny|large] [--method beam]
                    [--mode graph|eager|autograd]
"""
from __future__ import annotations

import argparse
import functools
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X published FP32 vector peak. This build emits no packed-FP32 instructions, but gfx950
# issues plain FP32 VALU instructions with register operands at up to two per SIMD every four
# cycles, so the unpacked rate is bounded by the same figure (a timing kernel of independent
# register adds reached 0.36 wave instructions per cycle per SIMD, 72 % of it); instructions with
# a scalar-register operand issue at half that rate.
FP32_VALU_TFLOPS = 157.3
EQ_FFT = 4096
WORKLOADS = {"console": "mixing_console", "tiny": "tiny_console", "large": "large_console",
             "batch": "batched_graphs", "console_ar": "mixing_console",
             "learned_init": "labelled_tiny_consoles", "reverb": "reverb_console"}
TYPE_NAMES = ("in", "out", "mix", "gain_pan", "eq", "compressor", "imager", "delay", "tanh",
              "noisegate", "compressor_ar", "reverb", "delay_long")
# kernel source of each step type (to tie a stored PMC traffic figure to the code it came from)
# (the kernel file, then the local headers whose code it compiles in, hashed in this order)
KERNEL_SRC = {"mix": ("k_pointwise.hip", "device_common.h"),
              "out": ("k_pointwise.hip", "device_common.h"),
              "gain_pan": ("k_pointwise.hip", "device_common.h"),
              "imager": ("k_pointwise.hip", "device_common.h"),
              "tanh": ("k_pointwise.hip", "device_common.h"),
              "eq": ("k_eq.hip", "fft4096.h", "device_common.h"),
              "compressor": ("k_comp.hip", "dynamics.h", "device_common.h"),
              "noisegate": ("k_comp.hip", "dynamics.h", "device_common.h"),
              "compressor_ar": ("k_comp_ar.hip", "dynamics.h", "device_common.h"),
              "delay": ("k_delay.hip", "device_common.h"),
              "reverb": ("k_reverb.hip", "fft4096.h", "device_common.h"),
              "delay_long": ("k_delay.hip", "device_common.h")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--method", default="beam")
    ap.add_argument("--graphs", type=int, default=128, help="graphs in the batch workload")
    ap.add_argument("--mode", default="graph", choices=("graph", "eager", "autograd"),
                    help="how the timed step is issued: one HIP-graph replay of the whole step "
                         "(default), the same C-ABI calls issued eagerly, or through autograd")
    ap.add_argument("--single-mode", action="store_true",
                    help="time only --mode (no graph capture unless it is the graph mode); for "
                         "profiler runs, where every kernel launch should belong to the timed mode")
    ap.add_argument("--T", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-forward-only", action="store_true",
                    help="skip timing the forward render alone (a trace then ends with the "
                         "timed step issues)")
    ap.add_argument("--breakdown-json", default=None, help="write the per-step timing table here")
    ap.add_argument("--train-consoles", type=int, default=25000,
                    help="learned_init: labelled tiny consoles rendered for training (4 examples each)")
    ap.add_argument("--epochs", type=int, default=6, help="learned_init: training epochs")
    ap.add_argument("--eval-consoles", type=int, default=8, help="learned_init: held-out consoles")
    ap.add_argument("--gd-steps", type=int, default=200, help="learned_init: plain GD steps")
    ap.add_argument("--workers", type=int, default=16,
                    help="learned_init: processes drawing the training consoles (0: this one)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the schedule's tuning settings by timing them first")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB first (scales PMC counters)")
    return ap.parse_args()


def step_bytes(sched, n: int, T: int, backward: bool) -> int:
    """Algorithmic HBM bytes of one step (stereo float32 = 8 B per node-sample): forward reads
    every input edge and writes the output, 8 (d_in + 1) T per node; the adjoint reads every
    output-edge adjoint, writes the input adjoint, and reads either the node output (gain_pan,
    imager: 1 row) or its inputs (eq, compressor, delay, tanh: d_in rows); mix reads neither."""
    t = int(sched.step_type[n])
    total = 0
    for i in range(int(sched.step_ptr[n]), int(sched.step_ptr[n + 1])):
        d_in = int(sched.in_ptr[i + 1] - sched.in_ptr[i])
        d_out = int(sched.out_ptr[i + 1] - sched.out_ptr[i])
        if not backward:
            rows = d_in + 1
        elif t == 2:
            rows = d_out + 1
        elif t in (3, 6):
            rows = d_out + 2
        else:
            rows = d_out + d_in + 1
        total += 8 * rows * _len(sched, i, T)
    return total


def _len(sched, i: int, T: int) -> int:
    """Signal length of the node at reordered position i (per-node lengths, else T)."""
    return T if sched.len_sigma is None else int(sched.len_sigma[i])


DELAY_FMA = 2 * 5 * 39  # per stereo sample: 2 channels x 5 taps x 39-tap FIR
RV_BLOCK, RV_HALF = 2048, 2049  # reverb output block, one-sided bins of its 4096-point transforms


def step_flops(sched, n: int, T: int, backward: bool) -> float:
    """Algorithmic FP32 flops of an FFT- or FIR-bound step. EQ: 5 N log2 N per complex N-point FFT
    (N = 4096), two transforms per 2048-sample tile forward (window FFT, inverse FFT) plus the
    real spectral product, three backward (adjoint window FFT, inverse FFT, input-tile FFT) plus
    the spectral product and the complex cross-spectrum accumulation. Delay: 2 flops per FMA of
    the 5 x 39-tap filters per channel, once forward, twice backward (input adjoint and tap
    gradients)."""
    if int(sched.step_type[n]) == 11:
        return reverb_flops(sched, n, T, backward)
    if int(sched.step_type[n]) in (7, 12):  # delay (5 slots), delay_long (20 slots)
        samples = sum(_len(sched, i, T) for i in range(int(sched.step_ptr[n]),
                                                         int(sched.step_ptr[n + 1])))
        slots = 20 if int(sched.step_type[n]) == 12 else 5
        return samples * 2.0 * DELAY_FMA * slots / 5 * (2 if backward else 1)
    tiles = sum(-(-_len(sched, i, T) // (EQ_FFT // 2))
                for i in range(int(sched.step_ptr[n]), int(sched.step_ptr[n + 1])))
    fft = 5.0 * EQ_FFT * np.log2(EQ_FFT)
    per_tile = 3 * fft + 2 * EQ_FFT + 8 * EQ_FFT if backward else 2 * fft + 2 * EQ_FFT
    return tiles * per_tile


def reverb_flops(sched, n: int, T: int, backward: bool) -> float:
    """Reverb step (partitioned overlap-save with 2048-tap partitions): per output block one
    4096-point FFT and one inverse (5 N log2 N each) and, for each partition in reach, the
    per-channel complex multiply-add of 2049 one-sided bins (2 x 8 flops); the adjoint does the
    same (its FIR-gradient cross-spectra run once after the last step and are not counted)."""
    L = sched.reverb_len
    parts = -(-L // RV_BLOCK)
    fft = 5.0 * EQ_FFT * np.log2(EQ_FFT)
    total = 0.0
    for i in range(int(sched.step_ptr[n]), int(sched.step_ptr[n + 1])):
        nb = -(-_len(sched, i, T) // RV_BLOCK)
        pairs = sum(min(parts, b + 1) for b in range(nb))  # same count forward and adjoint
        total += nb * 2 * fft + pairs * RV_HALF * 16
    return total


def stored_traffic(kernel_type: str, direction: str, workload: str):
    """HBM traffic of the dominant kernel from committed rocprofv3 PMC summaries, only if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        src = b"".join(open(os.path.join(ROOT, "paper_2408_03204_amd", "csrc", f), "rb").read()
                       for f in KERNEL_SRC[kernel_type])
        key = f"{direction}:{kernel_type}:{workload}"
        ent = rec.get(key)
        if ent and ent.get("src_sha256") == hashlib.sha256(src).hexdigest():
            return ent.get("bytes_per_launch")
    except Exception:  # noqa: BLE001
        return None
    return None


CPU_SAMPLE_T = 2 ** 15  # oracle sample length: a few seconds of CPU work per step on any graph


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed_reps(fn, min_seconds: float, max_reps: int):
    reps, t0 = 0, time.perf_counter()
    while reps < max_reps and (reps == 0 or time.perf_counter() - t0 < min_seconds):
        fn()
        reps += 1
    return reps, time.perf_counter() - t0


def cpu_baseline(maker, T_full: int, seed_T: int, min_seconds: float = 8.0, max_reps: int = 6):
    """The FP64 oracle (forward render, MRSTFT loss, autograd backward) on the same graph, as it
    stands, on a bounded sample of the workload (the graph at length `seed_T`), repeated until
    about `min_seconds` of CPU work, once with one thread and once with every host thread."""
    import torch

    from oracle import mrstft as OM
    from oracle import render as OR
    threads = len(os.sched_getaffinity(0))
    # one untimed pass on a short signal first (thread pool and FFT plan set-up)
    wu = maker(T=4096)
    Pu = OR.as_params64(wu.params, requires_grad=True)
    Lu = OM.mrstft(OR.render(wu.graph.node_type, wu.graph.edges, wu.sources, Pu,
                             reverb_noise=wu.reverb_noise),
                   torch.as_tensor(wu.sources[:1], dtype=torch.float64))
    torch.autograd.grad(Lu, [Pu[t] for t in Pu if Pu[t].shape[0] > 0])
    w = maker(T=seed_T)
    g = w.graph
    P = OR.as_params64(w.params, requires_grad=True)
    with torch.no_grad():
        tgt = OR.render(g.node_type, g.edges, w.sources, OR.as_params64(w.target_params),
                        reverb_noise=w.reverb_noise)
    keys = [t for t in P if P[t].shape[0] > 0]

    def step():
        Y = OR.render(g.node_type, g.edges, w.sources, P, reverb_noise=w.reverb_noise)
        L = OM.mrstft(Y, tgt)
        torch.autograd.grad(L, [P[t] for t in keys])

    before = torch.get_num_threads()
    rates = {}
    for n in (1, threads):
        torch.set_num_threads(n)
        reps, dt = _timed_reps(step, min_seconds, max_reps)
        rates[n] = (w.processed_nodes * seed_T * reps / dt, reps, dt)
    torch.set_num_threads(before)
    frac = "" if seed_T == T_full else f" (1/{T_full // seed_T} of the benchmark length)"
    v, reps, dt = rates[threads]
    v1, reps1, dt1 = rates[1]
    return {"value": round(v, 1), "unit": "node-samples/s", "cores": threads, "kind": "oracle",
            "single_thread": round(v1, 1), "cpu_model": _cpu_model(),
            "sample": f"{w.name} graph at T={seed_T}{frac}: forward+MRSTFT+backward in float64 "
                      f"(torch autograd), {reps} step(s) in {dt:.1f} s on {threads} threads, "
                      f"{reps1} in {dt1:.1f} s on 1 thread"}


def cpu_baseline_graph(w, min_seconds: float = 8.0, max_reps: int = 6):
    """The FP64 oracle (forward render and the adjoint of a seeded output adjoint, by autograd) on
    one graph of the batch at its own T, repeated until about `min_seconds` of CPU work, with one
    thread and with every host thread."""
    import torch

    from oracle import render as OR
    g = w.graph
    threads = len(os.sched_getaffinity(0))
    P = OR.as_params64(w.params, requires_grad=True)
    keys = [t for t in P if P[t].shape[0] > 0]
    dY = torch.as_tensor(np.random.default_rng(1).standard_normal(
        (g.count(1), 2, w.T)), dtype=torch.float64)

    def step():
        Y = OR.render(g.node_type, g.edges, w.sources, P)
        torch.autograd.grad((Y * dY).sum(), [P[t] for t in keys])

    before = torch.get_num_threads()
    rates = {}
    for n in (1, threads):
        torch.set_num_threads(n)
        reps, dt = _timed_reps(step, min_seconds, max_reps)
        rates[n] = (w.processed_nodes * w.T * reps / dt, reps, dt)
    torch.set_num_threads(before)
    v, reps, dt = rates[threads]
    return {"value": round(v, 1), "unit": "node-samples/s", "cores": threads, "kind": "oracle",
            "single_thread": round(rates[1][0], 1), "cpu_model": _cpu_model(),
            "sample": f"graph 0 of the batch ({g.num_nodes} nodes, T={w.T}), forward+backward in "
                      f"float64, {reps} step(s) in {dt:.1f} s on {threads} threads"}


def _tune(args, sched, S, P) -> dict:
    """Optionally autotune the schedule; returns the settings in force for the config record."""
    from paper_2408_03204_amd import autotune
    times = None
    if args.autotune:
        times = autotune.tune_all(sched, S, P)
        print(f"autotune (setting -> candidate -> ms): {times}", file=sys.stderr)
    out = {**autotune.settings(sched), "autotuned": bool(args.autotune)}
    if times:
        out["autotune_ms"] = {k: {str(c): round(v, 4) for c, v in r.items()}
                              for k, r in times.items()}
    return out


def setup_console(args, dev):
    """The mixing-console gradient step: render, MRSTFT loss against a target rendered with
    hidden parameters, loss adjoint, render adjoint (GradStep; also issued through autograd)."""
    import torch

    import synth
    from paper_2408_03204_amd import GradStep, Schedule, mrstft_loss, render

    maker = getattr(synth, WORKLOADS[args.workload])
    if args.workload == "console_ar":  # the same console, attack/release compressors
        maker = functools.partial(maker, attack_release=True)
    w = maker(T=args.T) if args.T else maker()
    g = w.graph
    t_s = time.perf_counter()
    sched = Schedule(g.node_type, g.edges, args.method)
    schedule_ms = (time.perf_counter() - t_s) * 1e3
    if w.reverb_noise is not None:
        sched.set_reverb_noise(torch.as_tensor(w.reverb_noise, device=dev))
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev).requires_grad_(True)
         for t, p in w.params.items() if p.shape[0] > 0}
    with torch.no_grad():
        Ptgt = {t: torch.as_tensor(p, device=dev) for t, p in w.target_params.items()
                if p.shape[0] > 0}
        target = render(sched, S, Ptgt).clone()
    plist = list(P.values())

    def autograd_step():
        Y = render(sched, S, P)
        L = mrstft_loss(Y, target)
        return torch.autograd.grad(L, plist)

    tuning = _tune(args, sched, S, {t: p.detach() for t, p in P.items()})
    gs = GradStep(sched, S, {t: p.detach() for t, p in P.items()}, target)
    wanted = {args.mode} if args.single_mode else {"graph", "eager", "autograd"}
    if "graph" in wanted:
        gs.capture()
    steps = {m: fn for m, fn in (("graph", gs.replay), ("eager", gs.run),
                                 ("autograd", autograd_step)) if m in wanted}
    config = {"workload": w.name, "nodes": g.num_nodes, "processed_nodes": w.processed_nodes,
              "edges": g.num_edges, "T": w.T, "schedule": args.method,
              "steps_in_schedule": sched.num_steps, "loss": "mrstft 512/1024/2048",
              "step": "render+loss+adjoint", "host_schedule_ms": round(schedule_ms, 2),
              **tuning}
    return {"sched": sched, "S": S, "P": {t: p.detach() for t, p in P.items()}, "T": w.T,
            "rb": None, "node_samples": w.processed_nodes * w.T, "steps": steps,
            "config": config, "key": args.workload,
            "cpu": (lambda: cpu_baseline(maker, w.T, min(w.T, CPU_SAMPLE_T)))}


def setup_batch(args, dev):
    """Uneven graphs merged into one schedule (per-node lengths): forward render and render
    adjoint of all graphs with a seeded output adjoint (no loss: the MRSTFT loss takes one
    length), issued eagerly or as one captured HIP graph."""
    import concurrent.futures
    import functools

    import torch

    import synth
    from paper_2408_03204_amd import RenderBuffers, Schedule, merge_graphs, merge_inputs

    count, seed = args.graphs, 7
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        ws = list(ex.map(functools.partial(synth.batched_graph, seed), range(count)))
    m = merge_graphs([(w.graph.node_type, w.graph.edges, w.T) for w in ws])
    S_h, P_h = merge_inputs(m, [w.sources for w in ws], [w.params for w in ws])
    sample = ws[0]
    node_samples = sum(w.processed_nodes * w.T for w in ws)
    n_out = [(m["output_offset"][i], w.graph.count(synth.OUT), w.T) for i, w in enumerate(ws)]
    del ws
    t_s = time.perf_counter()
    sched = Schedule(m["node_type"], m["edges"], args.method, lengths=m["lengths"])
    schedule_ms = (time.perf_counter() - t_s) * 1e3
    T = m["T"]
    S = torch.as_tensor(S_h, device=dev)
    del S_h
    P = {t: torch.as_tensor(p, device=dev) for t, p in P_h.items()}
    rng = np.random.default_rng(seed)
    dY_h = np.zeros((sched.num_outputs, 2, T), dtype=np.float32)
    for o0, n, Tg in n_out:
        dY_h[o0:o0 + n, :, :Tg] = rng.standard_normal((n, 2, Tg), dtype=np.float32)
    dY = torch.as_tensor(dY_h, device=dev)
    rb = RenderBuffers(sched, T, dev, with_backward=True)
    dP = {t: torch.empty_like(p) for t, p in P.items()}
    tuning = _tune(args, sched, S, P)

    def eager():
        rb.forward(S, P)
        rb.backward(S, P, dY, dP)

    wanted = {args.mode} if args.single_mode else {"graph", "eager"}
    steps = {}
    if "graph" in wanted:
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            eager()
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            eager()
        steps["graph"] = graph.replay
    if "eager" in wanted:
        steps["eager"] = eager
    counts = np.bincount(m["node_type"], minlength=len(TYPE_NAMES))
    config = {"workload": f"batched_uneven_{count}graphs", "graphs": count,
              "nodes": int(counts.sum()), "processed_nodes": int(counts.sum() - counts[0]),
              "edges": int(m["edges"].shape[1]), "T": "per graph U{2^16, 2^17, 2^18}",
              "row_stride": T, "schedule": args.method, "steps_in_schedule": sched.num_steps,
              "step": "render+adjoint (seeded output adjoint)",
              "host_schedule_ms": round(schedule_ms, 2), **tuning}
    return {"sched": sched, "S": S, "P": P, "T": T, "rb": rb, "dY": dY,
            "node_samples": node_samples, "steps": steps, "config": config, "key": "batch",
            "cpu": (lambda: cpu_baseline_graph(sample))}


def run_learned_init(args, pool):
    """Time to the plain run's final MRSTFT loss: gradient descent from the encoder's prediction
    against gradient descent from the default parameters, on held-out tiny consoles. The encoder
    is first trained on consoles rendered by the library (not timed)."""
    import torch

    from paper_2408_03204_amd import learned_init as LI

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    t0 = time.perf_counter()
    dry, mixf, lab = LI.render_dataset(11, args.train_consoles, pool, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"rendered {dry.shape[0]} training examples in {t1 - t0:.1f} s")
    net, hist = LI.train(dry, mixf, lab, epochs=args.epochs, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del dry, mixf
    # encoder inference at the training batch: bf16 MFMA convolutions against float32
    from paper_2408_03204_amd import encoder as ENC
    Fr = ENC.n_frames(2 ** 15)
    xb = torch.randn((256, 2 * ENC.N_MELS, Fr), device=dev)
    inf = ENC.Encoder(net.w, 256, Fr)
    conv_flops, f_in, c_in = 0, Fr, 2 * ENC.N_MELS
    for _ in range(6):
        f_out = (f_in + 1) // 2
        conv_flops += 2 * 256 * 64 * f_out * c_in * 5
        f_in, c_in = f_out, 64
    inf_ms = {}
    for bf in (True, False):
        for _ in range(3):
            inf.forward(xb, bf16=bf)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            inf.forward(xb, bf16=bf)
        e1.record()
        torch.cuda.synchronize()
        inf_ms["bf16" if bf else "f32"] = e0.elapsed_time(e1) / 20
    tf = conv_flops / (inf_ms["bf16"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                "frac": round(tf / 2500.0, 5), "traffic": None,
                "kernel": "conv_fwd_mfma (bf16, whole encoder forward, batch 256)",
                "flops_per_launch": conv_flops, "ms": round(inf_ms["bf16"], 4),
                "f32_forward_ms": round(inf_ms["f32"], 4)}
    rows = LI.gd_compare(net.w, n_consoles=args.eval_consoles, steps=args.gd_steps, log=log)
    hit = [r for r in rows if r["learned_ms"] is not None]
    ratios = [r["plain_ms"] / r["learned_ms"] for r in hit]
    out = {"metric": "time to the plain GD final MRSTFT loss: plain / learned init",
           "value": round(float(np.median(ratios)), 3) if ratios else None, "unit": "x",
           "n_gpus": 1, "steps": args.gd_steps, "warmup": 0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 (encoder inference bf16)",
           "data": "synthetic",
           "config": {"workload": "learned_init_tiny_console_4trk", "T": 2 ** 15,
                      "train_consoles": args.train_consoles,
                      "train_examples": 4 * args.train_consoles, "epochs": args.epochs,
                      "eval_consoles": args.eval_consoles, "gd_steps": args.gd_steps,
                      "optimizer": "adam lr 0.01"},
           "reached": f"{len(hit)}/{len(rows)}",
           "plain_ms_median": round(float(np.median([r["plain_ms"] for r in rows])), 3),
           "learned_ms_median": round(float(np.median([r["learned_ms"] for r in hit])), 3)
           if hit else None,
           "learned_steps_median": float(np.median([r["learned_steps_to_target"] for r in hit]))
           if hit else None,
           "roofline": roofline,
           "training_loss_by_epoch": [round(h, 5) for h in hist],
           "train_seconds": round(t2 - t1, 1), "render_dataset_seconds": round(t1 - t0, 1),
           "per_console": rows}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "learned_init":
        from paper_2408_03204_amd import learned_init as LI
        if args.workers <= 0:
            run_learned_init(args, LI.InlinePool())
            return
        pool = LI.make_pool(args.workers)  # forked before this process first touches the GPU
        try:
            run_learned_init(args, pool)
        finally:
            pool.shutdown()
        return
    import torch

    from paper_2408_03204_amd import RenderBuffers

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:  # a plain copy of known size, for PMC counter scaling
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = setup_batch(args, dev) if args.workload == "batch" else setup_console(args, dev)
    sched, S, T = ctx["sched"], ctx["S"], ctx["T"]
    steps = ctx["steps"]
    if args.mode not in steps:
        raise SystemExit(f"--mode {args.mode} is not available for this workload")

    def timed(fn) -> float:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    modes = {m: timed(fn) for m, fn in steps.items() if m != args.mode}
    ms = timed(steps[args.mode])  # the reported mode is timed last
    modes[args.mode] = ms
    value = ctx["node_samples"] / (ms * 1e-3)
    # the same step timed one by one: spread of the step time
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record()
        steps[args.mode]()
        b.record()
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in evs)
    spread = {q: round(float(np.percentile(per, q)), 4) for q in (10, 50, 90)}
    # the forward render alone (the paper's render call), eager issue
    forward = None
    if not args.no_forward_only:
        rbf = ctx["rb"] or RenderBuffers(sched, T, dev, with_backward=False)
        fwd_ms = timed(lambda: rbf.forward(S, ctx["P"]))
        fwd_bytes = sum(step_bytes(sched, n, T, False) for n in range(1, sched.num_steps + 1))
        forward = {"ms": round(fwd_ms, 4),
                   "node_samples_per_s": round(ctx["node_samples"] / (fwd_ms * 1e-3), 1),
                   "algorithmic_GBps": round(fwd_bytes / (fwd_ms * 1e6), 1),
                   "hbm_frac": round(fwd_bytes / (fwd_ms * 1e6) / HBM_PEAK_GBS, 4)}

    # ---- per-step breakdown: every render / adjoint step timed with events on its stream ------
    roofline, table, steps_hbm = None, [], None
    if not args.no_breakdown:
        rb = ctx["rb"] or RenderBuffers(sched, T, dev, with_backward=True)
        Pd = ctx["P"]
        dY = ctx.get("dY")
        if dY is None:
            dY = torch.randn((sched.num_outputs, 2, T), device=dev)
        dPd = {t: torch.empty_like(p) for t, p in Pd.items()}
        rb.forward(S, Pd)
        rb.backward(S, Pd, dY, dPd)
        reps = 5
        evs = []
        for direction in ("fwd", "bwd"):
            steps = range(1, sched.num_steps + 1) if direction == "fwd" else \
                range(sched.num_steps - 1, 0, -1)
            for n in steps:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    if direction == "fwd":
                        rb.step(S, Pd, n)
                    else:
                        rb.backward_step(S, Pd, dY, n)
                b.record()
                evs.append((direction, n, a, b))
        torch.cuda.synchronize()
        agg: dict = {}
        for direction, n, a, b in evs:
            t_ms = a.elapsed_time(b) / reps
            tname = TYPE_NAMES[int(sched.step_type[n])]
            nbytes = step_bytes(sched, n, T, direction == "bwd")
            nodes = int(sched.step_ptr[n + 1] - sched.step_ptr[n])
            table.append({"dir": direction, "step": n, "type": tname, "nodes": nodes,
                          "ms": round(t_ms, 5), "GB/s": round(nbytes / (t_ms * 1e6), 1)})
            k = (direction, tname)
            tb = agg.setdefault(k, [0.0, 0, 0])
            tb[0] += t_ms
            tb[1] += nbytes
            tb[2] += 1
        (d, tname), (t_tot, b_tot, cnt) = max(agg.items(), key=lambda kv: kv[1][0])
        # the dominant step kernel: algorithmic bytes per launch over its average launch time
        achieved = b_tot / (t_tot * 1e6)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": stored_traffic(tname, d, ctx["key"]),
                    "kernel": f"{tname} {d}", "launches": cnt,
                    "algorithmic_bytes_per_launch": round(b_tot / cnt),
                    "ms_per_launch": round(t_tot / cnt, 5)}
        if tname in ("eq", "delay", "reverb", "delay_long"):  # FFT / FIR arithmetic: flop rate
            flops = sum(step_flops(sched, r["step"], T, d == "bwd") for r in table
                        if r["dir"] == d and r["type"] == tname)
            tf = flops / (t_tot * 1e-3) / 1e12
            roofline["alu_view"] = {
                "achieved": round(tf, 2), "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP32_VALU_TFLOPS, 4),
                "count": {"eq": "5 N log2 N flops per 4096-point complex FFT plus the spectral "
                                "products",
                          "delay": "2 flops per FIR multiply-add",
                          "delay_long": "2 flops per FIR multiply-add",
                          "reverb": "5 N log2 N flops per 4096-point complex FFT plus 16 flops "
                                    "per one-sided bin, partition and block"}[tname],
                "peak_basis": "published FP32 vector peak (unpacked instructions with register "
                              "operands dual-issue on gfx950)"}
        all_t = sum(v[0] for v in agg.values())
        all_b = sum(v[1] for v in agg.values())
        steps_hbm = {"ms": round(all_t, 4), "GB/s": round(all_b / (all_t * 1e6), 1),
                     "frac": round(all_b / (all_t * 1e6) / HBM_PEAK_GBS, 4)}
        if args.breakdown_json:
            with open(args.breakdown_json, "w") as f:
                json.dump({"step_ms": ms, "table": table,
                           "by_type": {f"{k[0]}:{k[1]}": v for k, v in agg.items()}}, f,
                          indent=1)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = ctx["cpu"]()

    out = {"metric": "node-samples/s fwd+bwd", "value": round(value, 1),
           "unit": "node-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": dict(ctx["config"], issue=args.mode),
           "ms_per_step_by_issue": {m: round(v, 4) for m, v in modes.items()},
           "ms_per_step_p10_p50_p90": [spread[10], spread[50], spread[90]],
           "forward_only": forward,
           "roofline": roofline, "render_adjoint_steps": steps_hbm, "cpu_baseline": cpu}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
