"""CPU pins of the gradient-judging helper shared by the GPU parity tests (tests/gpu_common.py):
per-column scales, the structural-zero floor, and the column groups (EQ bins, reverb masks,
delay phasor pairs)."""
import numpy as np

from gpu_common import ZERO_COLUMN_FLOOR, column_scales, grad_err


def test_plain_columns_are_judged_on_their_own():
    ref = np.array([[1.0, 1e-3, 0.0], [-2.0, 5e-4, 0.0]])
    got = ref.copy()
    got[0, 1] += 1e-6  # 1e-3 of column 1's largest entry: at the tolerance
    assert abs(grad_err(got, ref) - 1e-3) < 1e-9
    sc = column_scales(ref)
    assert sc[0] == 2.0 and sc[1] == 1e-3 and sc[2] == ZERO_COLUMN_FLOOR * 2.0


def test_eq_bins_share_one_group():
    ref = np.ones((1, 1024))
    ref[0, 7] = 1e-7  # a bin crossing zero is judged against 1e-3 of the group's peak
    assert column_scales(ref)[7] == 1e-3


def test_reverb_masks_form_four_groups():
    ref = np.concatenate([np.full(192, 10.0), np.full(192, 1.0), np.full(192, 0.1),
                          np.full(192, 1e-9)])[None, :]
    ref[0, 5] = 0.0
    sc = column_scales(ref)
    assert sc[5] == 1e-2 and sc[200] == 1.0 and sc[400] == 0.1
    assert sc[600] == max(1e-12, ZERO_COLUMN_FLOOR * 10.0)


def test_delay_phasor_pairs_are_groups_and_magnitudes_are_not():
    ref = np.zeros((1, 220))
    ref[0, 0], ref[0, 1] = 1e-6, 50.0  # a phasor gradient along the imaginary axis
    ref[0, 2:22] = 1.0
    ref[0, 5] = 1e-6  # a log-magnitude entry stays its own column
    sc = column_scales(ref)
    assert sc[0] == 50.0 * 1e-3 and sc[1] == 50.0
    assert sc[5] == max(1e-6, ZERO_COLUMN_FLOOR * 50.0)
