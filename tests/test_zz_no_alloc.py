"""grafx_render_noalloc, the allocation-free variant of grafx_render (its workspace is a static
scratch array in the library), against grafx_render through the C ABI on one GPU: three calls in
a row, each on a smaller input than the one before, with every node type that keeps state in the
workspace (EQ and delay designs, compressor, noisegate and attack/release chunk states). The
scratch keeps each call's contents, so a later call that read stale state would differ. Each
call's U must be bit-identical with grafx_render's on a fresh workspace; the last one is also
checked against the FP64 oracle at the render tolerance."""
import pytest
import torch

import synth
from gpu_common import check_render, device_inputs, say
from paper_2408_03204_amd import RenderBuffers, Schedule, render_noalloc

pytestmark = pytest.mark.gpu


def _pair(w):
    sched = Schedule(w.graph.node_type, w.graph.edges, "beam")
    need = sched.workspace_bytes(w.T, False)
    assert need <= (32 << 20), need  # the scratch's size (GRAFX_NOALLOC_SCRATCH_BYTES)
    S, P = device_inputs(w)
    ref = RenderBuffers(sched, w.T, "cuda", with_backward=False)
    ref.forward(S, P)
    U = torch.full((sched.num_nodes, 2, w.T), float("nan"), dtype=torch.float32, device="cuda")
    Y = render_noalloc(sched, ref.plan, S, P, U)
    torch.cuda.synchronize()
    K = sched.num_inputs
    same = torch.equal(U[K:].view(torch.int32), ref.U[K:].view(torch.int32))
    say(f"   nodes={sched.num_nodes} T={w.T} scratch {need} B: bit-identical={same}")
    assert same
    return sched, Y, U


def test_noalloc_render_matches_render_on_successive_smaller_inputs():
    dyn = (synth.MIX, synth.GAIN_PAN, synth.EQ, synth.COMP, synth.IMAGER, synth.DELAY,
           synth.TANH, synth.GATE, synth.COMP_AR)
    cases = [synth.mixing_console(T=2 ** 18),
             synth.random_workload(77, 16, 3 * 2 ** 15 + 1234, types=dyn, edge_p=0.3),
             synth.tiny_console(T=6001, attack_release=True)]
    for i, w in enumerate(cases):
        say(f"[noalloc] call {i + 1}: {w.name}")
        sched, Y, U = _pair(w)
    check_render(w, sched, Y, U)

