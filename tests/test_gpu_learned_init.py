"""GPU: the learned-initialiser pipeline end to end at a small size. Labelled tiny consoles are
rendered by the library and turned into features; the encoder trains on them with the library's
training kernels (its training loss must fall); gradient descent from the default parameters
lowers the MRSTFT loss; the comparison with the encoder's prediction runs and reports
consistent numbers. The consoles are drawn in this process (no worker pool)."""
import numpy as np
import pytest
import torch

from gpu_common import say
from paper_2408_03204_amd import learned_init as LI

pytestmark = pytest.mark.gpu


def test_pipeline_small():
    dev = torch.device("cuda")
    dry, mixf, lab = LI.render_dataset(21, 96, LI.InlinePool(), chunk=32, device=dev)
    torch.cuda.synchronize()
    assert dry.shape[0] == 4 * 96 and mixf.shape[0] == 96 and lab.shape == (4 * 96, 11)
    assert torch.isfinite(dry).all() and torch.isfinite(mixf).all()
    assert float(lab.min()) >= 0.0 and float(lab.max()) <= 1.0
    net, hist = LI.train(dry, mixf, lab, epochs=8, batch=32, lr=1e-3, log=say)
    assert hist[-1] < hist[0], hist
    rows = LI.gd_compare(net.w, n_consoles=1, seed=2000, steps=30, log=say)
    r = rows[0]
    assert r["plain_final_loss"] < r["plain_first_loss"]
    assert np.isfinite(r["learned_first_loss"]) and r["plain_ms"] > 0
