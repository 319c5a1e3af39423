"""GPU parity of the learned initialiser against its FP64 oracle (oracle/encoder.py): log-mel
features, the float32 encoder forward and its hand-written backward, Adam, the bfloat16
matrix-core forward (each layer against the oracle convolution of the same bfloat16-rounded
operands, which pins the MFMA lane layout), the map onto parameter rows, and the batch gather.
Tolerances: features 2e-4 absolute (they are ln-energies / 5), outputs 1e-5, gradients 1e-3 of
each tensor's largest entry, bfloat16 layers 1e-4 of the layer's largest output (float32 sums
of exact bfloat16 products)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import grad_err, say
from oracle import encoder as E
from paper_2408_03204_amd import encoder as enc

pytestmark = pytest.mark.gpu
F64 = torch.float64


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def example_inputs(B, T, seed):
    """Encoder inputs from real features: dry sources and mixes of pairs of them."""
    src = synth.make_sources(synth.rng_for(seed, 1), B + 1, T)
    mix = src[:-1] + src[1:]
    return np.ascontiguousarray(
        np.stack([E.encoder_input(src[b], mix[b]) for b in range(B)]), dtype=np.float32)


@pytest.mark.parametrize("T", [2 ** 15, 5000])
def test_logmel_matches_oracle(T):
    say(f"[logmel] T={T}")
    sig = synth.make_sources(synth.rng_for(3, 1), 3, T)
    sig[1] *= 1e-3  # a quiet signal: features near the floor of the logarithm
    feats = enc.logmel(torch.as_tensor(sig).cuda()).cpu().numpy()
    for i in range(3):
        ref = E.log_mel(sig[i])
        assert feats[i].shape == ref.shape
        err = float(np.max(np.abs(feats[i] - ref)))
        say(f"   signal {i}: max |err| {err:.2e}")
        assert err <= 2e-4


def _weights(seed=0):
    w = synth.encoder_weights(seed)
    ws = E.unflatten(w)
    return w, ws


def test_forward_backward_match_oracle():
    B, T = 6, 2 ** 15
    say(f"[encoder fp32] B={B} T={T}")
    x = example_inputs(B, T, 5)
    F = x.shape[-1]
    w, ws = _weights(0)
    lab = np.random.default_rng(6).uniform(size=(B, 11)).astype(np.float32)
    net = enc.Encoder(torch.as_tensor(w).cuda(), B, F)
    xd, ld = torch.as_tensor(x).cuda(), torch.as_tensor(lab).cuda()
    out = net.forward(xd).cpu().numpy()
    net.backward(xd, ld)
    torch.cuda.synchronize()
    loss, dw = float(net.loss), net.dw.cpu().numpy()
    # each layer against the oracle convolution of the GPU's own previous layer
    acts = net.acts.cpu().numpy()
    frames, off, prev = F, 0, x.astype(np.float64)
    for layer in range(6):
        Fo = (frames + 1) // 2
        y = acts[off:off + B * 64 * Fo].reshape(B, 64, Fo)
        ref = E.conv_layer(torch.as_tensor(prev), ws[2 * layer], ws[2 * layer + 1]).numpy()
        e = float(np.max(np.abs(y - ref))) / max(float(np.max(np.abs(ref))), 1e-30)
        say(f"   layer {layer + 1}: rel err {e:.2e}")
        assert e <= 1e-5, (layer, e)
        off += B * 64 * Fo
        frames, prev = Fo, y.astype(np.float64)
    # oracle in float64 from the same float32 inputs and weights
    ws64 = [t.clone().requires_grad_(True) for t in ws]
    x64, l64 = torch.as_tensor(x, dtype=F64), torch.as_tensor(lab, dtype=F64)
    ref_out = E.forward(x64, ws64)
    ref_loss = ((ref_out - l64) ** 2).mean()
    grads = torch.autograd.grad(ref_loss, ws64)
    e_out = float(np.max(np.abs(out - ref_out.detach().numpy())))
    say(f"   out max |err| {e_out:.2e}, loss {loss:.7f} vs {float(ref_loss.detach()):.7f}")
    assert e_out <= 1e-5
    assert abs(loss - float(ref_loss.detach())) <= 1e-5 * float(ref_loss.detach())
    ref_flat = torch.cat([g.reshape(-1) for g in grads]).numpy()
    o = 0
    for i, g in enumerate(grads):
        n = g.numel()
        e = grad_err(dw[o:o + n], ref_flat[o:o + n])
        assert e <= 1e-3, (i, e)
        o += n
    # fixed summation orders: a second backward gives the same bits
    net.backward(xd, ld)
    torch.cuda.synchronize()
    assert np.array_equal(net.dw.cpu().numpy(), dw)


def test_bf16_forward_layers_and_output():
    B, T = 5, 2 ** 15
    say(f"[encoder bf16] B={B}")
    x = example_inputs(B, T, 7)
    F = x.shape[-1]
    w, ws = _weights(1)
    net = enc.Encoder(torch.as_tensor(w).cuda(), B, F)
    xd = torch.as_tensor(x).cuda()
    out32 = net.forward(xd).cpu().numpy()
    out16 = net.forward(xd, bf16=True).cpu().numpy()
    acts = net.acts.cpu().numpy()
    torch.cuda.synchronize()
    # each layer: the GPU's bfloat16 output against the float64 convolution of the same
    # bfloat16-rounded operands (its own input: the previous GPU layer)
    frames, off, prev = F, 0, x
    for layer in range(6):
        Fo = (frames + 1) // 2
        y = acts[off:off + B * 64 * Fo].reshape(B, 64, Fo)
        Wl = bf16_round(ws[2 * layer].numpy().astype(np.float32))
        ref = E.conv_layer(torch.as_tensor(bf16_round(prev)), torch.as_tensor(Wl),
                           ws[2 * layer + 1]).numpy()
        e = float(np.max(np.abs(y - ref))) / max(float(np.max(np.abs(ref))), 1e-30)
        say(f"   layer {layer + 1}: rel err {e:.2e}")
        assert e <= 1e-4, (layer, e)
        off += B * 64 * Fo
        frames, prev = Fo, y
    e_out = float(np.max(np.abs(out16 - out32)))
    say(f"   bf16 vs fp32 outputs max |diff| {e_out:.2e}")
    assert e_out <= 3e-2


def test_adam_matches_oracle():
    rng = np.random.default_rng(8)
    p0 = rng.normal(size=1000).astype(np.float32)
    gs = [rng.normal(size=1000).astype(np.float32) for _ in range(3)]
    p = torch.as_tensor(p0).cuda()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    ref = [torch.as_tensor(p0, dtype=F64)]
    st = {}
    for t, g in enumerate(gs, start=1):
        enc.adam(p, torch.as_tensor(g).cuda(), m, v, t, 1e-2)
        E.adam(ref, [torch.as_tensor(g, dtype=F64)], st, 1e-2)
    torch.cuda.synchronize()
    assert float(np.max(np.abs(p.cpu().numpy() - ref[0].numpy()))) <= 1e-6


def test_chain_params_match_oracle():
    s = np.random.default_rng(9).uniform(0.02, 0.98, size=(7, 11)).astype(np.float32)
    gp, eq, comp = enc.chain_params(torch.as_tensor(s).cuda())
    torch.cuda.synchronize()
    for b in range(7):
        r = E.to_params(s[b].astype(np.float64))
        assert np.max(np.abs(gp[b].cpu().numpy() - r["gain_pan"])) <= 1e-5
        assert np.max(np.abs(eq[b].cpu().numpy() - r["eq"])) <= 1e-5
        assert np.max(np.abs(comp[b].cpu().numpy() - r["compressor"]) /
                      np.maximum(np.abs(r["compressor"]), 1.0)) <= 1e-5


def test_gather_is_a_copy():
    feats = torch.randn((5, 128, 9), device="cuda")
    mixf = torch.randn((4, 128, 9), device="cuda")
    table = torch.randn((5, 11), device="cuda")
    dry = torch.tensor([4, 0, 2], dtype=torch.int32, device="cuda")
    mix = torch.tensor([1, 1, 3], dtype=torch.int32, device="cuda")
    net = enc.Encoder(torch.as_tensor(synth.encoder_weights(0)).cuda(), 3, 9)
    x = torch.empty((3, 256, 9), device="cuda")
    lab = torch.empty((3, 11), device="cuda")
    net.gather(feats, dry, mixf, mix, x, table, lab)
    torch.cuda.synchronize()
    assert torch.equal(x, torch.cat([feats[dry.long()], mixf[mix.long()]], dim=1))
    assert torch.equal(lab, table[dry.long()])
