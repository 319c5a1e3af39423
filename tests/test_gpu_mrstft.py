"""GPU parity of the multi-resolution STFT loss and its gradient against the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_common import GRAD_TOL, grad_err, say
from oracle import mrstft as OM

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,T", [(1, 9000), (2, 2 ** 14 + 3), (1, 700), (1, 300)])
def test_mrstft_loss_and_grad(rows, T):
    from paper_2408_03204_amd import mrstft_loss
    say(f"[mrstft] rows={rows} T={T}")
    rng = np.random.default_rng(T)
    tgt = (rng.normal(size=(rows, 2, T)) * 0.3).astype(np.float32)
    y = (tgt + 0.2 * rng.normal(size=(rows, 2, T))).astype(np.float32)
    Y = torch.as_tensor(y).cuda().requires_grad_(True)
    L = mrstft_loss(Y, torch.as_tensor(tgt).cuda())
    L.backward()
    torch.cuda.synchronize()
    y64 = torch.as_tensor(y, dtype=torch.float64).requires_grad_(True)
    L64 = OM.mrstft(y64, torch.as_tensor(tgt, dtype=torch.float64))
    (g64,) = torch.autograd.grad(L64, [y64]) if L64.requires_grad else (torch.zeros_like(y64),)
    loss, loss64 = float(L.detach()), float(L64.detach())
    say("   loss", loss, loss64)
    assert abs(loss - loss64) <= 1e-5 * max(1.0, abs(loss64))
    e = grad_err(Y.grad.cpu().numpy(), g64.numpy())
    say("   grad err", e)
    assert e <= GRAD_TOL
