"""Autotuner of the schedule's tuning settings (include/grafx.h, grafx_schedule_set_tuning).

For one schedule and signal length it times the pointwise steps of a render and of its adjoint
(mix, out, gain_pan, imager and tanh, the HBM-bound kernels whose best work per thread depends on
how many nodes and samples a step carries) under every candidate setting, with HIP events on the
current stream, and keeps the fastest. Only launches move; the choice is the caller's to keep
(e.g. in a cache keyed by the graph and T)."""
from __future__ import annotations

import torch

from .api import RenderBuffers, Schedule

POINTWISE_TYPES = (1, 2, 3, 6, 8)  # out, mix, gain_pan, imager, tanh
CANDIDATES = (1, 2, 4)


def tune_pointwise(sched: Schedule, S: torch.Tensor, P: dict, reps: int = 5,
                   rb: RenderBuffers | None = None) -> dict:
    """Times the pointwise steps under each unroll candidate, sets the fastest on `sched` and
    returns {candidate: milliseconds per render+adjoint of those steps}."""
    dev = S.device
    T = int(S.shape[-1])
    rb = rb or RenderBuffers(sched, T, dev, with_backward=True)
    dY = torch.randn((sched.num_outputs, 2, T), device=dev)
    steps = [n for n in range(1, sched.num_steps + 1) if int(sched.step_type[n]) in POINTWISE_TYPES]
    result = {}
    for un in CANDIDATES:
        sched.set_tuning(Schedule.TUNE_POINTWISE_UNROLL, un)
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
        result[un] = e0.elapsed_time(e1) / reps
    best = min(result, key=result.get)
    sched.set_tuning(Schedule.TUNE_POINTWISE_UNROLL, best)
    return result
