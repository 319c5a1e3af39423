"""GPU: the bounded chunk waits of the dynamics kernels (the chunked scan of the envelope
recursion, paper Eq. 8) and the workspace's error word, forced from the host. With the
schedule's GRAFX_TUNE_WAIT_POLLS set to 0 every wait gives up at once: the kernels still run to
their end, the affected outputs are NaN and grafx_workspace_error reports bit 0. With the default
setting the word is clear again after the next render, and the render matches the FP64 oracle
and the first render bit for bit. No kernel faults or spins: each wait is a bounded loop."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import check_render, say
from paper_2408_03204_amd import RenderBuffers, Schedule

pytestmark = pytest.mark.gpu
CHUNK = 3072


def dynamics_graph(T, seed=71):
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    c = b.add(synth.COMP)
    gte = b.add(synth.GATE)
    ar = b.add(synth.COMP_AR)
    m = b.add(synth.MIX)
    o = b.add(synth.OUT)
    b.connect(i0, c)
    b.connect(i1, c)
    b.connect(c, gte)
    b.connect(i1, ar)
    b.connect(gte, m)
    b.connect(ar, m)
    b.connect(m, o)
    g = b.build()
    return synth.Workload("dynamics_wait", g, synth.make_sources(synth.rng_for(seed, 1), 2, T),
                          synth.draw_params(synth.rng_for(seed, 2), g), None, T, seed)


def test_wait_give_up_is_reported_and_cleared():
    T = 6 * CHUNK + 1000
    w = dynamics_graph(T)
    dev = torch.device("cuda")
    sched = Schedule(w.graph.node_type, w.graph.edges)
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    dY = torch.as_tensor(np.random.default_rng(3).standard_normal(
        (sched.num_outputs, 2, T)).astype(np.float32), device=dev)
    rb = RenderBuffers(sched, T, dev, with_backward=True)
    dP = {t: torch.empty_like(p) for t, p in P.items()}

    say(f"[wait] default polls, T={T}")
    rb.forward(S, P)
    rb.backward(S, P, dY, dP)
    assert rb.error_word() == 0
    Y0 = rb.Y.clone()
    check_render(w, sched, rb.Y, rb.U)

    say("[wait] polls = 0: every chunk wait gives up")
    sched.set_tuning(Schedule.TUNE_WAIT_POLLS, 0)
    rb.forward(S, P)
    word = rb.error_word()
    assert word & 1, word
    pos = {int(v): i for i, v in enumerate(sched.perm)}
    comp = rb.U[pos[2]].cpu().numpy()
    assert np.isfinite(comp[:, :CHUNK]).all()  # the first chunk waits for nothing
    assert np.isnan(comp[:, CHUNK:]).any()

    say("[wait] default polls again: forward clears the word; a give-up in the adjoint alone")
    sched.set_tuning(Schedule.TUNE_WAIT_POLLS, 1 << 24)
    rb.forward(S, P)
    assert rb.error_word() == 0
    assert torch.equal(rb.Y, Y0)
    sched.set_tuning(Schedule.TUNE_WAIT_POLLS, 0)
    rb.backward(S, P, dY, dP)
    assert rb.error_word() & 1
    sched.set_tuning(Schedule.TUNE_WAIT_POLLS, 1 << 24)
    rb.forward(S, P)
    rb.backward(S, P, dY, dP)
    torch.cuda.synchronize()
    assert rb.error_word() == 0
    for t, d in dP.items():
        assert torch.isfinite(d).all(), t


def test_graph_without_dynamics_reports_zero():
    w = synth.random_workload(5, 8, 4096, types=(synth.MIX, synth.GAIN_PAN, synth.EQ))
    dev = torch.device("cuda")
    sched = Schedule(w.graph.node_type, w.graph.edges)
    rb = RenderBuffers(sched, w.T, dev, with_backward=False)
    rb.ws.fill_(0xFF)  # garbage in the workspace: the word of a graph without dynamics is 0
    assert rb.error_word() == 0
