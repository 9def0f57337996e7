"""Dense and closed-form tools of Appendix A/B, used only as pins.

* ``dense_matrix``   -- the matrix of any linear field map, column by column.
* ``overlap_D4``     -- the 4D overlap operator through the transfer matrices,
                        D_OV(m) = 1/2 [ (1+m) + (1-m) gamma_5 (S - 1)(S + 1)^-1 ]
                        with S = S_1 ... S_Ls, S_i = -Q_{i-}^-1 Q_{i+},
                        Q_{i+-} = gamma_5 D_w (b_i P+- + c_i P-+) +- 1
                        (App. A, eq.(startprop) and the definitions below eq.(4d-5d)).
* ``free_dw``        -- D_w of a free field on a plane wave exp(i p.x):
                        (4 + M5) - sum_mu cos p_mu + i sum_mu gamma_mu sin p_mu.
* ``overlap_tanh_spin`` -- the polar form of eq.(polar) for constant b, c:
                        (S-1)/(S+1) = [(1+H)^Ls - (1-H)^Ls] [(1+H)^Ls + (1-H)^Ls]^-1
                        with the Moebius kernel H = (b+c) gamma_5 D_w [2 + (b-c) D_w]^-1
                        of eq.(argument) (the "D" there is D_w).
"""

import numpy as np

from .gamma import GAMMA, GAMMA5, ONE, P_MINUS, P_PLUS


def dense_matrix(apply_fn, in_shape, dtype=np.complex128):
    n = int(np.prod(in_shape))
    cols = []
    for k in range(n):
        e = np.zeros(n, dtype=dtype)
        e[k] = 1.0
        cols.append(np.asarray(apply_fn(e.reshape(in_shape))).reshape(-1))
    return np.stack(cols, axis=1)


def _spin_kron(vol, spin_mat):
    """spin_mat acting on a (V, 4, 3)-flattened vector."""
    return np.kron(np.kron(np.eye(vol), spin_mat), np.eye(3))


def overlap_D4(Dw, vol, m, b, c):
    """Dense D_OV(m) from a dense D_w (12 V x 12 V) via the transfer matrices."""
    n = Dw.shape[0]
    g5 = _spin_kron(vol, GAMMA5)
    pp, pm = _spin_kron(vol, P_PLUS), _spin_kron(vol, P_MINUS)
    one = np.eye(n)
    S = one.astype(np.complex128)
    for i in range(len(b)):
        q_plus = g5 @ Dw @ (b[i] * pp + c[i] * pm) + one
        q_minus = g5 @ Dw @ (b[i] * pm + c[i] * pp) - one
        S_i = -np.linalg.solve(q_minus, q_plus)
        S = S @ S_i
    eps = (S - one) @ np.linalg.inv(S + one)
    return 0.5 * ((1.0 + m) * one + (1.0 - m) * g5 @ eps)


def free_dw(p, M5):
    """4x4 spin matrix of D_w on exp(i p.x) for U = 1."""
    out = (4.0 + M5 - sum(np.cos(pm) for pm in p)) * ONE
    for mu in range(4):
        out = out + 1j * np.sin(p[mu]) * GAMMA[mu]
    return out


def overlap_tanh_spin(Dw4, m, b, c, Ls):
    """Polar form of D_OV(m) for a 4x4 momentum-space D_w (constant b, c)."""
    H = (b + c) * GAMMA5 @ Dw4 @ np.linalg.inv(2.0 * ONE + (b - c) * Dw4)
    up = np.linalg.matrix_power(ONE + H, Ls)
    dn = np.linalg.matrix_power(ONE - H, Ls)
    eps = (up - dn) @ np.linalg.inv(up + dn)
    return 0.5 * ((1.0 + m) * ONE + (1.0 - m) * GAMMA5 @ eps)
