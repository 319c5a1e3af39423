"""GPU: graphs of different lengths merged into one schedule (per-node lengths; the paper's
graph-level batching, Sec. 2 "Batched processing"). From one merged render and adjoint, each
graph's output rows, source adjoint and parameter-gradient rows must equal, bit for bit, those
of the same graph rendered alone at its own T (tiles and chunks start at sample 0 either way
and every reduction adds the extra tiles' zeros at the end of a fixed order); outputs are also
checked against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import RENDER_TOL, rel_err, say
from oracle import render as OR
from paper_2408_03204_amd import RenderBuffers, Schedule, merge_graphs, merge_inputs

pytestmark = pytest.mark.gpu


def _alone(w, dY, dev, noise=None, surrogate=False):
    g = w.graph
    sched = Schedule(g.node_type, g.edges, "beam")
    sched.set_delay_surrogate(surrogate)
    if noise is not None:
        sched.set_reverb_noise(torch.as_tensor(noise, device=dev))
    S = torch.as_tensor(w.sources, device=dev)
    P = {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}
    rb = RenderBuffers(sched, w.T, dev, with_backward=True)
    rb.forward(S, P)
    dP = {t: torch.empty_like(p) for t, p in P.items()}
    dS = torch.zeros_like(S)
    rb.backward(S, P, torch.as_tensor(dY, device=dev), dP, dS=dS)
    torch.cuda.synchronize()
    return (rb.Y.cpu().numpy(), {t: d.cpu().numpy() for t, d in dP.items()}, dS.cpu().numpy())


def _check_merged(ws, tag, noise=None, surrogate=False):
    dev = torch.device("cuda")
    m = merge_graphs([(w.graph.node_type, w.graph.edges, w.T) for w in ws])
    say(f"[batch {tag}] {len(ws)} graphs, lengths {[w.T for w in ws]}, {len(m['node_type'])} "
        f"nodes, stride {m['T']}")
    S, P = merge_inputs(m, [w.sources for w in ws], [w.params for w in ws])
    sched = Schedule(m["node_type"], m["edges"], "beam", lengths=m["lengths"])
    sched.set_delay_surrogate(surrogate)
    if noise is not None:
        sched.set_reverb_noise(torch.as_tensor(noise, device=dev))
    Sd = torch.as_tensor(S, device=dev)
    Pd = {t: torch.as_tensor(p, device=dev) for t, p in P.items()}
    rng = np.random.default_rng(5)
    dY = np.zeros((sched.num_outputs, 2, m["T"]), dtype=np.float32)
    dY_each = []
    for i, w in enumerate(ws):
        n_out, o0 = w.graph.count(synth.OUT), m["output_offset"][i]
        d = rng.standard_normal((n_out, 2, w.T)).astype(np.float32)
        dY[o0:o0 + n_out, :, :w.T] = d
        dY_each.append(d)
    rb = RenderBuffers(sched, m["T"], dev, with_backward=True)
    rb.forward(Sd, Pd)
    dPd = {t: torch.empty_like(p) for t, p in Pd.items()}
    dSd = torch.zeros_like(Sd)
    rb.backward(Sd, Pd, torch.as_tensor(dY, device=dev), dPd, dS=dSd)
    torch.cuda.synchronize()
    Y, dS = rb.Y.cpu().numpy(), dSd.cpu().numpy()
    dP = {t: d.cpu().numpy() for t, d in dPd.items()}
    for i, w in enumerate(ws):
        g = w.graph
        Ya, dPa, dSa = _alone(w, dY_each[i], dev, noise, surrogate)
        n_out, o0, k0 = g.count(synth.OUT), m["output_offset"][i], m["input_offset"][i]
        K = g.count(synth.IN)
        assert np.array_equal(Y[o0:o0 + n_out, :, :w.T], Ya), (tag, i, "Y")
        assert np.array_equal(dS[k0:k0 + K, :, :w.T], dSa), (tag, i, "dS")
        for t, d in dPa.items():
            r0 = int(m["param_offset"][i][t])
            assert np.array_equal(dP[t][r0:r0 + d.shape[0]], d), (tag, i, "dP", t)
        Y64 = OR.render(g.node_type, g.edges, w.sources, OR.as_params64(w.params),
                        reverb_noise=noise).numpy()
        e = rel_err(Ya.astype(np.float64), Y64)
        assert e <= RENDER_TOL, (tag, i, e)
    say("   merged == alone bit for bit (Y, dS, dP); alone vs oracle within tolerance")


@pytest.mark.parametrize("lengths", [(6699, 9220, 3001, 4101), (8192, 4096, 6144, 2048)])
def test_merged_random_graphs(lengths):
    ws = [synth.random_workload(300 + i, 12 + 2 * i, T) for i, T in enumerate(lengths)]
    _check_merged(ws, f"random {lengths}")


def test_merged_batched_consoles():
    ws = synth.batched_graphs(6, 21, T_choices=(2 ** 12, 2 ** 13, 2 ** 14), src_range=(4, 12))
    _check_merged(ws, "consoles")


def test_merged_graphs_with_reverbs_and_2s_delays():
    """Reverbs (one noise for the whole batch) and 2 s delays with the delay-time surrogate in
    graphs of different lengths: merged == alone bit for bit (phasor gradients included), alone
    within the render tolerance of the oracle."""
    types = (synth.MIX, synth.GAIN_PAN, synth.REVERB, synth.DELAY_LONG, synth.EQ)
    ws = [synth.random_workload(seed, 9, T, types=types, edge_p=0.35)
          for seed, T in ((1402, 5 * 2048 + 300), (1411, 2048), (1413, 9001))]
    assert all(w.graph.count(synth.REVERB) >= 1 and w.graph.count(synth.DELAY_LONG) >= 1
               for w in ws)
    _check_merged(ws, "reverb + 2 s delay", noise=synth.reverb_noise(14, 7000), surrogate=True)
