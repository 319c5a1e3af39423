"""GPU: the whole gradient step (render, MRSTFT loss, loss adjoint, render adjoint) captured in a
HIP graph and replayed.

Every replay is checked bit for bit against the same step issued eagerly through the C ABI, with
eager work and host synchronisations between replays; an in-place parameter update between
replays must be seen by the next replay. The eager step itself is checked bit for bit against
the autograd path, which the other GPU tests pin to the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_common import say
from paper_2408_03204_amd import GradStep, Schedule, mrstft_loss, render

pytestmark = pytest.mark.gpu


def _setup(T):
    w = synth.mixing_console(T=T)
    g = w.graph
    dev = torch.device("cuda")
    sched = Schedule(g.node_type, g.edges, "beam")
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    with torch.no_grad():
        tgt = render(sched, S, {t: torch.as_tensor(p, device=dev)
                                for t, p in w.target_params.items() if p.shape[0] > 0}).clone()
    return w, sched, S, P, tgt


def _snapshot(gs):
    torch.cuda.synchronize()
    return float(gs.loss), {t: g.clone() for t, g in gs.grads.items()}


def _same(a, b):
    la, ga = a
    lb, gb = b
    assert np.float32(la).tobytes() == np.float32(lb).tobytes(), (la, lb)
    for t in ga:
        assert torch.equal(ga[t], gb[t]), t


@pytest.mark.parametrize("T", [2 ** 15 + 1234, 2 ** 17])
def test_graph_replay_matches_eager(T):
    w, sched, S, P, tgt = _setup(T)
    say(f"[graph] {w.name} T={T}")
    gs = GradStep(sched, S, P, tgt)
    gs.run()
    eager = _snapshot(gs)
    # the eager step equals the autograd path
    Pg = {t: p.clone().requires_grad_(True) for t, p in P.items()}
    L = mrstft_loss(render(sched, S, Pg), tgt)
    keys = list(Pg)
    gr = torch.autograd.grad(L, [Pg[t] for t in keys])
    torch.cuda.synchronize()
    _same(eager, (float(L.detach()), {t: g for t, g in zip(keys, gr)}))
    gs.capture()
    for rep in range(3):
        gs.replay()
        _same(_snapshot(gs), eager)
        gs.run()  # eager work between replays, on the same buffers
        _same(_snapshot(gs), eager)
    # in-place update of the parameters between replays
    with torch.no_grad():
        for p in P.values():
            p.mul_(0.99)
    gs.run()
    eager2 = _snapshot(gs)
    assert abs(eager2[0] - eager[0]) > 0
    for rep in range(2):
        gs.replay()
        _same(_snapshot(gs), eager2)
    say(f"   loss {eager[0]:.6f} -> {eager2[0]:.6f}; replays bitwise equal to eager")


def test_graph_replay_with_dynamics_variants():
    """A console whose compressors have attack/release ballistics, plus noisegates on the tracks:
    their chunk state is reset by kernels, not memsets, so a captured step replays bit for bit
    (the attack/release forward's branch-pattern passes included)."""
    T = 2 ** 15 + 1234
    w = synth.mixing_console(T=T, attack_release=True)
    g = w.graph
    # every imager becomes a noisegate (same position in the graph, gate parameters drawn)
    nt = np.where(g.node_type == synth.IMAGER, synth.GATE, g.node_type).astype(np.int32)
    g2 = synth.Graph(nt, g.edges)
    params = synth.draw_params(synth.rng_for(77, 2), g2)
    dev = torch.device("cuda")
    sched = Schedule(g2.node_type, g2.edges, "beam")
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in params.items() if p.shape[0] > 0}
    assert synth.GATE in P and synth.COMP_AR in P
    with torch.no_grad():
        tgt = (0.5 * render(sched, S, P)).contiguous()
    say(f"[graph dynamics] {g2.num_nodes} nodes, gates {int((nt == synth.GATE).sum())}, "
        f"attack/release {int((nt == synth.COMP_AR).sum())}")
    gs = GradStep(sched, S, P, tgt)
    gs.run()
    eager = _snapshot(gs)
    gs.capture()
    for rep in range(3):
        gs.replay()
        _same(_snapshot(gs), eager)
        gs.run()
        _same(_snapshot(gs), eager)


def test_graph_replay_with_reverbs_and_2s_delays():
    """The reverb console with 2 s delays and the delay surrogate on: IR synthesis, partitioned
    products, cross-spectra and phasor gradients replay bit for bit (no memset, no allocation in
    the captured step), with eager steps between replays and after a parameter update."""
    T = 2 ** 15 + 1234
    w = synth.reverb_console(T=T)
    g = w.graph
    # every imager becomes a 2 s delay (same position in the graph, parameters drawn)
    nt = np.where(g.node_type == synth.IMAGER, synth.DELAY_LONG, g.node_type).astype(np.int32)
    g2 = synth.Graph(nt, g.edges)
    params = synth.draw_params(synth.rng_for(78, 2), g2)
    dev = torch.device("cuda")
    sched = Schedule(g2.node_type, g2.edges, "beam")
    sched.set_reverb_noise(torch.as_tensor(w.reverb_noise, device=dev))
    sched.set_delay_surrogate(True)
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in params.items() if p.shape[0] > 0}
    assert synth.REVERB in P and synth.DELAY_LONG in P
    with torch.no_grad():
        tgt = (0.5 * render(sched, S, P)).contiguous()
    say(f"[graph reverb] {g2.num_nodes} nodes, reverbs {int((nt == synth.REVERB).sum())}, "
        f"2 s delays {int((nt == synth.DELAY_LONG).sum())}")
    gs = GradStep(sched, S, P, tgt)
    gs.run()
    eager = _snapshot(gs)
    assert float(gs.grads[synth.DELAY_LONG].reshape(-1, 2, 20, 22)[..., :2].abs().max()) > 0
    gs.capture()
    for rep in range(3):
        gs.replay()
        _same(_snapshot(gs), eager)
        gs.run()
        _same(_snapshot(gs), eager)
    with torch.no_grad():
        for p in P.values():
            p.mul_(0.999)
    gs.run()
    eager2 = _snapshot(gs)
    gs.replay()
    _same(_snapshot(gs), eager2)
