"""Autotuner of the schedule's launch-shape settings (include/grafx.h, grafx_schedule_set_tuning).

For one schedule and signal length it times, under every candidate value of a setting, the render
and adjoint steps of the node types that setting shapes, with HIP events on the current stream,
and keeps the fastest:

* pointwise unroll (mix, out, gain_pan, imager, tanh): 1024-sample parts per block, 1 / 2 / 4;
* EQ block order: tiles of a node on one XCD, or the hardware order;
* dynamics block order (compressor, noisegate, compressor_ar): a node's chunks contiguous, or
  the step's nodes interleaved;
* delay tap-gradient tiles per block: 4 / 8 / 16.

Settings only move launches (the two orders leave every bit unchanged; unroll and tap tiles
regroup parameter-gradient partial sums). The choice is the caller's to keep (e.g. in a cache
keyed by the graph and T)."""
from __future__ import annotations

import torch

from .api import RenderBuffers, Schedule

POINTWISE_TYPES = (1, 2, 3, 6, 8)  # out, mix, gain_pan, imager, tanh
CANDIDATES = (1, 2, 4)
# setting -> (node types whose steps it shapes, candidate values; the first is the default)
KNOBS = {
    Schedule.TUNE_POINTWISE_UNROLL: (POINTWISE_TYPES, CANDIDATES),
    Schedule.TUNE_EQ_ORDER: ((4,), (0, 1)),
    Schedule.TUNE_DYN_ORDER: ((5, 9, 10), (2, 1, 0)),
    Schedule.TUNE_TAP_TILES: ((7, 12), (16, 8, 4)),
}
KNOB_NAMES = {Schedule.TUNE_POINTWISE_UNROLL: "pointwise_unroll",
              Schedule.TUNE_EQ_ORDER: "eq_order", Schedule.TUNE_DYN_ORDER: "dyn_order",
              Schedule.TUNE_TAP_TILES: "tap_tiles"}


def tune_knob(sched: Schedule, knob: int, S: torch.Tensor, P: dict, reps: int = 5,
              rb: RenderBuffers | None = None) -> dict:
    """Times the steps of the types `knob` shapes under each candidate, sets the fastest on
    `sched` and returns {candidate: milliseconds per render+adjoint of those steps} ({} when the
    schedule has no such step, leaving the setting as it was)."""
    types, cands = KNOBS[knob]
    steps = [n for n in range(1, sched.num_steps + 1) if int(sched.step_type[n]) in types]
    if not steps:
        return {}
    dev = S.device
    T = int(S.shape[-1])
    rb = rb or RenderBuffers(sched, T, dev, with_backward=True)
    dY = torch.randn((sched.num_outputs, 2, T), device=dev)
    result = {}
    for v in cands:
        sched.set_tuning(knob, v)
        rb.forward(S, P)
        rb.backward(S, P, dY)  # every step's inputs current, designs and carries in place
        for n in steps:  # warm-up of this setting's kernels
            rb.step(S, P, n)
            if n < sched.num_steps:
                rb.backward_step(S, P, dY, n)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            for n in steps:
                rb.step(S, P, n)
                if n < sched.num_steps:
                    rb.backward_step(S, P, dY, n)
        e1.record()
        torch.cuda.synchronize(dev)
        result[v] = e0.elapsed_time(e1) / reps
    sched.set_tuning(knob, min(result, key=result.get))
    return result


def tune_pointwise(sched: Schedule, S: torch.Tensor, P: dict, reps: int = 5,
                   rb: RenderBuffers | None = None) -> dict:
    """tune_knob for the pointwise unroll."""
    return tune_knob(sched, Schedule.TUNE_POINTWISE_UNROLL, S, P, reps, rb)


def tune_all(sched: Schedule, S: torch.Tensor, P: dict, reps: int = 5) -> dict:
    """Every setting in turn (each with the others at their current values); returns
    {setting name: {candidate: ms}} for the settings the schedule has steps for."""
    rb = RenderBuffers(sched, int(S.shape[-1]), S.device, with_backward=True)
    out = {}
    for knob in KNOBS:
        r = tune_knob(sched, knob, S, P, reps, rb)
        if r:
            out[KNOB_NAMES[knob]] = r
    return out


def settings(sched: Schedule) -> dict:
    """The launch-shape settings in force, by name."""
    return {name: sched.get_tuning(k) for k, name in KNOB_NAMES.items()}
