"""Binding of the learned parameter initialiser (include/grafx.h: grafx_logmel,
grafx_encoder_*, grafx_adam): argument marshalling only, every step runs in the HIP library.

The encoder maps the log-mel features of a dry track and of the target mix ([256, F]) to the 11
normalised parameters of the track's gain_pan -> eq -> compressor chain; `chain_params` turns
them into parameter rows the renderer takes (the gradient-descent application of paper Sec. 4
then starts from them)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, load

N_MELS, N_OUT = 128, 11


def _st(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _need(t: torch.Tensor, name: str, dtype=torch.float32) -> torch.Tensor:
    """The library reads raw device pointers: tensors must be contiguous, on the GPU, of the
    expected dtype."""
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t


def n_frames(T: int) -> int:
    return (T - 1024) // 256 + 1 if T >= 1024 else 0


def logmel(signals: torch.Tensor) -> torch.Tensor:
    """[n, 2, T] float32 device signals -> [n, 128, F] features."""
    n, _, T = _need(signals, "signals").shape
    out = torch.empty((n, N_MELS, n_frames(T)), dtype=torch.float32, device=signals.device)
    check(load().grafx_logmel(n, T, signals.data_ptr(), out.data_ptr(), _st(signals.device)))
    return out


def sizes(batch: int, frames: int) -> tuple[int, int, int]:
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check(load().grafx_encoder_sizes(batch, frames, ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def adam(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
         lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
         lr_scale: torch.Tensor | None = None) -> None:
    """One Adam step in place; `lr_scale` (same size as p) multiplies lr per value."""
    tensors = [(p, "p"), (g, "g"), (m, "m"), (v, "v")]
    if lr_scale is not None:
        tensors.append((lr_scale, "lr_scale"))
    for t, name in tensors:
        _need(t, name)
        if t.numel() != p.numel():
            raise ValueError("p, g, m, v and lr_scale must have the same size")
    check(load().grafx_adam(p.numel(), p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                            None if lr_scale is None else lr_scale.data_ptr(), step, lr, beta1,
                            beta2, eps, _st(p.device)))


class Encoder:
    """Flat float32 weights on the device plus the buffers of one batch shape."""

    def __init__(self, weights: torch.Tensor, batch: int, frames: int):
        n_w, n_act, n_grad = sizes(batch, frames)
        if _need(weights, "weights").numel() != n_w:
            raise ValueError(f"weights must have {n_w} entries")
        dev = weights.device
        self.w, self.batch, self.frames = weights, batch, frames
        self.acts = torch.empty(n_act, dtype=torch.float32, device=dev)
        self.grads = torch.empty(n_grad, dtype=torch.float32, device=dev)
        self.out = torch.empty((batch, N_OUT), dtype=torch.float32, device=dev)
        self.dw = torch.empty_like(weights)
        self.m = torch.zeros_like(weights)
        self.v = torch.zeros_like(weights)
        self.loss = torch.zeros((), dtype=torch.float32, device=dev)
        self.step = 0

    def gather(self, dry_feats: torch.Tensor, dry: torch.Tensor, mix_feats: torch.Tensor,
               mix: torch.Tensor, x: torch.Tensor, label_table: torch.Tensor | None = None,
               labels: torch.Tensor | None = None) -> torch.Tensor:
        """x[b] = [dry_feats[dry[b]]; mix_feats[mix[b]]]; labels[b] = label_table[dry[b]]."""
        _need(dry_feats, "dry_feats"), _need(mix_feats, "mix_feats"), _need(x, "x")
        _need(dry, "dry", torch.int32), _need(mix, "mix", torch.int32)
        if label_table is not None:
            _need(label_table, "label_table"), _need(labels, "labels")
        check(load().grafx_encoder_gather(
            self.batch, self.frames, dry_feats.data_ptr(), dry.data_ptr(), mix_feats.data_ptr(),
            mix.data_ptr(), None if label_table is None else label_table.data_ptr(),
            None if labels is None else labels.data_ptr(), x.data_ptr(), _st(x.device)))
        return x

    def forward(self, x: torch.Tensor, bf16: bool = False) -> torch.Tensor:
        if tuple(_need(x, "x").shape) != (self.batch, 2 * N_MELS, self.frames):
            raise ValueError(f"x must have shape {(self.batch, 2 * N_MELS, self.frames)}")
        check(load().grafx_encoder_forward(self.batch, self.frames, x.data_ptr(), self.w.data_ptr(),
                                           int(bf16), self.acts.data_ptr(), self.out.data_ptr(),
                                           _st(x.device)))
        return self.out

    def backward(self, x: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
        """After a float32 forward on x: loss into self.loss, weight gradients into self.dw."""
        if tuple(_need(labels, "labels").shape) != (self.batch, N_OUT):
            raise ValueError(f"labels must have shape {(self.batch, N_OUT)}")
        check(load().grafx_encoder_backward(self.batch, self.frames, x.data_ptr(),
                                            self.w.data_ptr(), self.acts.data_ptr(),
                                            self.out.data_ptr(), labels.data_ptr(),
                                            self.loss.data_ptr(), self.dw.data_ptr(),
                                            self.grads.data_ptr(), _st(x.device)))
        return self.loss

    def train_step(self, x: torch.Tensor, labels: torch.Tensor, lr: float) -> torch.Tensor:
        self.forward(x)
        self.backward(x, labels)
        self.step += 1
        adam(self.w, self.dw, self.m, self.v, self.step, lr)
        return self.loss


def chain_params(out: torch.Tensor) -> tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Normalised outputs [B, 11] -> (gain_pan [B, 2], eq [B, 1024], compressor [B, 4])."""
    B, dev = _need(out, "out").shape[0], out.device
    gp = torch.empty((B, 2), dtype=torch.float32, device=dev)
    eq = torch.empty((B, 1024), dtype=torch.float32, device=dev)
    comp = torch.empty((B, 4), dtype=torch.float32, device=dev)
    check(load().grafx_encoder_params(B, out.data_ptr(), gp.data_ptr(), eq.data_ptr(),
                                      comp.data_ptr(), _st(dev)))
    return gp, eq, comp
