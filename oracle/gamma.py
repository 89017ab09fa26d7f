"""Euclidean gamma matrices used by the oracle.

Paper Sec. 2 (text after Eq. (1)) fixes only the properties that matter: each
gamma_mu has exactly one non-zero entry per row, equal to +-1 or +-i, and
gamma_mu^2 = 1, so (1 -+ gamma_mu) is twice a rank-2 projector.  The flop-count
footnote in Sec. 2 says the representation is the implementation's choice.
The oracle uses the Dirac representation

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   (k = 1, 2, 3: x, y, z)
    gamma_4 = diag(1, 1, -1, -1)                   (t)

built here from the Pauli matrices.  Index 0..3 below is mu = x, y, z, t.
"""
import numpy as np

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)

_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)

GAMMA = np.stack([
    np.block([[_Z2, -1j * SIGMA[0]], [1j * SIGMA[0], _Z2]]),
    np.block([[_Z2, -1j * SIGMA[1]], [1j * SIGMA[1], _Z2]]),
    np.block([[_Z2, -1j * SIGMA[2]], [1j * SIGMA[2], _Z2]]),
    np.block([[_I2, _Z2], [_Z2, -_I2]]),
])

GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

ID4 = np.eye(4, dtype=np.complex128)


def proj_minus(mu: int) -> np.ndarray:
    """(1 - gamma_mu): multiplies the forward-neighbour term of Eq. (1)."""
    return ID4 - GAMMA[mu]


def proj_plus(mu: int) -> np.ndarray:
    """(1 + gamma_mu): multiplies the backward-neighbour term of Eq. (1)."""
    return ID4 + GAMMA[mu]
