"""Learned initialisation of gradient-descent mixing (the application of paper Sec. 4, "Example
usage", started from an encoder's prediction instead of default parameters).

* `render_dataset`: labelled tiny consoles (4 tracks of gain_pan -> eq -> compressor into a mix,
  a master gain, an output) rendered by this library in merged batches; the log-mel features of
  every dry track and of every rendered mix, and the normalised labels of every track.
* `train`: the encoder trained on them with the library's float32 training kernels and Adam.
* `gd_compare`: on held-out consoles, gradient descent on the MRSTFT loss (render, loss and
  adjoint through the library, Adam through the library) from the default parameters and from
  the encoder's bfloat16 prediction; the wall time each needs to reach the loss the plain run
  ends at.

Every step of the method runs in the HIP library; this module only moves data and loops."""
from __future__ import annotations

import concurrent.futures
import multiprocessing
import os
import time

import numpy as np
import torch

import synth

from . import encoder as enc
from .api import GradStep, RenderBuffers, Schedule, merge_graphs, merge_inputs

N_TRACKS = 4
GP, EQ, COMP = synth.GAIN_PAN, synth.EQ, synth.COMP
# Adam step scale per compressor parameter (alpha, T, W, R): alpha lies within 0.03 of 1 and
# moves at most 1e-6 per step at lr 0.01 (so a 100 ms constant stays below 1 over 200 steps),
# the knee stays fixed, the ratio moves slower than the threshold
COMP_LR_SCALE = (1e-4, 1.0, 0.0, 0.3)


def _draw(args):
    seed, first, count, T = args
    ws, labels = synth.labelled_tiny_consoles(seed, count, T, first=first)
    return [w.sources for w in ws], [w.params for w in ws], labels


def _idle(seconds):
    time.sleep(seconds)
    return os.getpid()


class InlinePool:
    """Draws the consoles in this process (no workers)."""

    @staticmethod
    def map(fn, jobs):
        return map(fn, jobs)


def make_pool(workers: int = 16):
    """Worker processes for drawing the consoles' sources and parameters (numpy only). Create it
    before the process first uses the GPU: the workers are forked copies of this process, and
    overlapping idle tasks make every worker start here rather than at the first real task."""
    ctx = multiprocessing.get_context("fork")
    pool = concurrent.futures.ProcessPoolExecutor(max_workers=max(1, workers), mp_context=ctx)
    list(pool.map(_idle, [0.3] * max(1, workers)))
    return pool


def render_dataset(seed: int, n_consoles: int, pool, T: int = 2 ** 15, chunk: int = 128,
                   device="cuda"):
    """Returns (dry features [4n, 128, F], mix features [n, 128, F], labels [4n, 11]) on the
    device; track j of console i is row 4 i + j. `pool` draws the consoles (see make_pool)."""
    dev = torch.device(device)
    one = synth.tiny_console(T=8).graph
    F = enc.n_frames(T)
    dry = torch.empty((N_TRACKS * n_consoles, enc.N_MELS, F), dtype=torch.float32, device=dev)
    mixf = torch.empty((n_consoles, enc.N_MELS, F), dtype=torch.float32, device=dev)
    labels = np.empty((n_consoles, N_TRACKS, synth.N_LABELS))
    m = merge_graphs([(one.node_type, one.edges, T)] * chunk)
    sched = Schedule(m["node_type"], m["edges"], "beam")
    rb = RenderBuffers(sched, T, dev, with_backward=False)
    jobs = [(seed, c0, min(chunk, n_consoles - c0), T) for c0 in range(0, n_consoles, chunk)]
    for (_, c0, cnt, _), (srcs, params, lab) in zip(jobs, pool.map(_draw, jobs)):
        if cnt < chunk:  # pad the last chunk with copies of its first console
            srcs = srcs + [srcs[0]] * (chunk - cnt)
            params = params + [params[0]] * (chunk - cnt)
        S, P = merge_inputs(m, srcs, params)
        Sd = torch.as_tensor(S, device=dev)
        Pd = {t: torch.as_tensor(p, device=dev) for t, p in P.items()}
        rb.forward(Sd, Pd)
        dry[N_TRACKS * c0:N_TRACKS * (c0 + cnt)] = enc.logmel(Sd[:N_TRACKS * cnt])
        mixf[c0:c0 + cnt] = enc.logmel(rb.Y[:cnt])
        labels[c0:c0 + cnt] = lab
    lab = torch.as_tensor(labels.reshape(-1, synth.N_LABELS), dtype=torch.float32, device=dev)
    return dry, mixf, lab


def train(dry, mixf, labels, epochs: int = 4, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Encoder trained on the rendered examples (shuffled each epoch); returns the Encoder with
    the trained weights and the per-epoch mean training loss."""
    dev = dry.device
    n, F = dry.shape[0], dry.shape[-1]
    net = enc.Encoder(torch.as_tensor(synth.encoder_weights(seed), device=dev), batch, F)
    x = torch.empty((batch, 2 * enc.N_MELS, F), dtype=torch.float32, device=dev)
    lab = torch.empty((batch, enc.N_OUT), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        steps = n // batch
        d_all = torch.as_tensor(perm[:steps * batch].astype(np.int32), device=dev)
        m_all = torch.as_tensor((perm[:steps * batch] // N_TRACKS).astype(np.int32), device=dev)
        losses = torch.empty(steps, dtype=torch.float32, device=dev)
        for s in range(steps):
            d, mi = d_all[s * batch:(s + 1) * batch], m_all[s * batch:(s + 1) * batch]
            net.gather(dry, d, mixf, mi, x, labels, lab)
            net.train_step(x, lab, lr)
            losses[s:s + 1].copy_(net.loss.reshape(1))
        history.append(float(losses.mean()))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean training loss {history[-1]:.5f}")
    return net, history


class _GD:
    """Adam on a tiny console's parameters through GradStep (render, MRSTFT loss, adjoint)."""

    def __init__(self, sched, S, P, target, lr):
        self.P = P
        self.gs = GradStep(sched, S, P, target)
        self.lr = lr
        self.m = {t: torch.zeros_like(p) for t, p in P.items()}
        self.v = {t: torch.zeros_like(p) for t, p in P.items()}
        scale = torch.tensor(COMP_LR_SCALE, dtype=torch.float32, device=S.device)
        self.scale = {COMP: scale.repeat(P[COMP].shape[0], 1).contiguous()}
        self.step = 0

    def run(self, n, losses=None):
        for i in range(n):
            loss = self.gs.run()
            if losses is not None:
                losses[self.step:self.step + 1].copy_(loss.reshape(1))
            self.step += 1
            for t, p in self.P.items():
                enc.adam(p, self.gs.grads[t], self.m[t], self.v[t], self.step, self.lr,
                         lr_scale=self.scale.get(t))


def _console_inputs(w, dev):
    S = torch.as_tensor(w.sources, device=dev)
    return S, {t: torch.as_tensor(p, device=dev) for t, p in w.params.items() if p.shape[0] > 0}


def _defaults(w, dev):
    return {t: torch.as_tensor(p, device=dev)
            for t, p in synth.default_params(w.graph).items() if p.shape[0] > 0}


def _predict(net1, w, S, target, P):
    """Features, bfloat16 encoder forward and the parameter map, written into P (in place)."""
    feats = enc.logmel(S)
    mixf = enc.logmel(target)
    dev = S.device
    x = torch.empty((N_TRACKS, 2 * enc.N_MELS, feats.shape[-1]), dtype=torch.float32, device=dev)
    net1.gather(feats, net1.idx_dry, mixf, net1.idx_mix, x)
    out = net1.forward(x, bf16=True)
    gp, eq, comp = enc.chain_params(out)
    P[GP][:N_TRACKS].copy_(gp)
    P[EQ].copy_(eq)
    P[COMP].copy_(comp)


def gd_compare(weights, n_consoles: int = 8, seed: int = 1000, T: int = 2 ** 15,
               steps: int = 200, lr: float = 0.01, log=None):
    """Per held-out console: the loss curve and time of `steps` plain GD steps from the default
    parameters, and the step and time at which GD from the encoder's prediction first reaches
    the plain run's final loss (prediction included in the time)."""
    dev = weights.device
    ws, _ = synth.labelled_tiny_consoles(seed, n_consoles, T)
    sched = Schedule(ws[0].graph.node_type, ws[0].graph.edges, "beam")
    F = enc.n_frames(T)
    net1 = enc.Encoder(weights, N_TRACKS, F)
    net1.idx_dry = torch.arange(N_TRACKS, dtype=torch.int32, device=dev)
    net1.idx_mix = torch.zeros(N_TRACKS, dtype=torch.int32, device=dev)
    rows = []
    for i, w in enumerate(ws):
        S, Ptrue = _console_inputs(w, dev)
        target = torch.empty((1, 2, T), dtype=torch.float32, device=dev)
        rb = RenderBuffers(sched, T, dev, with_backward=False)
        rb.forward(S, Ptrue)
        target.copy_(rb.Y)
        # plain run (recorded), then the learned run (recorded)
        plain_l = torch.empty(steps, dtype=torch.float32, device=dev)
        P0 = _defaults(w, dev)
        _GD(sched, S, P0, target, lr).run(steps, plain_l)
        init_l = torch.empty(steps, dtype=torch.float32, device=dev)
        P1 = _defaults(w, dev)
        _predict(net1, w, S, target, P1)
        _GD(sched, S, P1, target, lr).run(steps, init_l)
        torch.cuda.synchronize(dev)
        pl, il = plain_l.cpu().numpy(), init_l.cpu().numpy()
        goal = float(pl[-1])
        hit = np.nonzero(il <= goal)[0]
        k = int(hit[0]) + 1 if hit.size else None
        # timed runs: plain `steps` steps; learned prediction + k steps
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        P0 = _defaults(w, dev)
        g0 = _GD(sched, S, P0, target, lr)
        P1 = _defaults(w, dev)
        g1 = _GD(sched, S, P1, target, lr)
        torch.cuda.synchronize(dev)
        e0.record()
        g0.run(steps)
        e1.record()
        if k is not None:
            _predict(net1, w, S, target, P1)
            g1.run(k)
        e2.record()
        torch.cuda.synchronize(dev)
        t_plain, t_learn = e0.elapsed_time(e1), e1.elapsed_time(e2)
        row = {"console": i, "plain_final_loss": goal, "plain_first_loss": float(pl[0]),
               "learned_first_loss": float(il[0]), "learned_final_loss": float(il[-1]),
               "learned_steps_to_target": k, "plain_ms": round(t_plain, 3),
               "learned_ms": round(t_learn, 3) if k is not None else None}
        rows.append(row)
        if log:
            log(str(row))
    return rows
