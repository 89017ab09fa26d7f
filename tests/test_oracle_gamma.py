"""Pins of the oracle's gamma matrices against the properties paper Sec. 2
states (one +-1/+-i per row, square to one) and the Clifford algebra."""
import itertools

import numpy as np

from oracle.gamma import GAMMA, GAMMA5, ID4, proj_minus, proj_plus


def test_clifford_algebra():
    for mu, nu in itertools.product(range(4), repeat=2):
        anti = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
        assert np.allclose(anti, 2 * ID4 * (mu == nu), atol=0)


def test_hermitian_and_one_unit_entry_per_row():
    allowed = {1, -1, 1j, -1j}
    for g in GAMMA:
        assert np.array_equal(g, np.conj(g.T))
        for row in g:
            nz = row[row != 0]
            assert len(nz) == 1 and complex(nz[0]) in allowed


def test_projectors_are_twice_rank_two_projectors():
    for mu in range(4):
        for p in (proj_minus(mu), proj_plus(mu)):
            assert np.allclose(p @ p, 2 * p)
            assert np.linalg.matrix_rank(p) == 2
        assert np.allclose(proj_minus(mu) @ proj_plus(mu), 0)


def test_gamma5_explicit():
    want = np.array([[0, 0, -1, 0], [0, 0, 0, -1], [-1, 0, 0, 0], [0, -1, 0, 0]])
    assert np.array_equal(GAMMA5, want)
    for g in GAMMA:
        assert np.allclose(GAMMA5 @ g + g @ GAMMA5, 0)


def test_dirac_representation_entries():
    # gamma_4 is diagonal in the Dirac representation; gamma_1 as written out
    assert np.array_equal(GAMMA[3], np.diag([1, 1, -1, -1]))
    g1 = np.array([[0, 0, 0, -1j], [0, 0, -1j, 0], [0, 1j, 0, 0], [1j, 0, 0, 0]])
    assert np.array_equal(GAMMA[0], g1)
