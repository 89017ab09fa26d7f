"""12-real link compression (rows 0 and 1 stored, row 2 rebuilt as
conj(row0 x row1)) is exact for SU(3) links and fails for a link with a
boundary sign folded in, which is why the library applies boundary phases in
the kernel and never into the links."""
import numpy as np

from paper_2303_08609_amd import inputs
from tests._helpers import reconstruct_row2, round_f32


def test_reconstruction_exact_for_su3():
    u = inputs.gen_su3_near_unit(inputs.rng(3), 5000, 0.7)
    assert np.abs(reconstruct_row2(u) - u).max() < 1e-14
    u32 = round_f32(u)
    assert np.abs(reconstruct_row2(u32) - u32).max() < 1e-6


def test_folding_the_antiperiodic_sign_breaks_reconstruction():
    u = inputs.gen_su3_near_unit(inputs.rng(4), 1000, 0.7)
    folded = -u                          # det(-U) = -1: no longer SU(3)
    rebuilt = reconstruct_row2(folded)
    # rows 0 and 1 survive, row 2 comes back with the wrong sign
    assert np.abs(rebuilt[:, :2] - folded[:, :2]).max() == 0
    assert np.allclose(rebuilt[:, 2], -folded[:, 2], atol=1e-13)
    assert np.abs(rebuilt[:, 2] - folded[:, 2]).max() > 0.5
