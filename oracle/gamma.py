"""Dirac matrices in a chiral basis and the chiral projectors of eq.(coeff).

The paper does not fix a basis.  The oracle uses the chiral basis
    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = x, y, z),
    gamma_t = [[0, 1], [1, 0]],
with gamma_5 formed as the product gamma_x gamma_y gamma_z gamma_t, and
P+- = (1 +- gamma_5) / 2 as in eq.(coeff).
"""

import numpy as np

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)

GAMMA = tuple(
    [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in SIGMA]
    + [np.block([[_Z2, _I2], [_I2, _Z2]])]
)
ONE = np.eye(4, dtype=np.complex128)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
P_PLUS = 0.5 * (ONE + GAMMA5)
P_MINUS = 0.5 * (ONE - GAMMA5)


def spin_apply(mat: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a 4x4 spin matrix to a field whose last two axes are (spin, colour)."""
    return np.matmul(mat, psi)
