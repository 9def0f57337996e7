"""The Wilson Dirac operator of eq.(wilson), written out literally.

    (D_w psi)(x) = (4 + M5) psi(x)
                   - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x)       psi(x + mu)
                                + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]

Fields are full-lattice complex128 arrays.  A 4D field has shape (V, 4, 3)
(site, spin, colour) and a 5D field (Ls, V, 4, 3); any leading axes are
carried along.  Links have shape (4, V, 3, 3) with U_mu(x) on the link
x -> x + mu acting on psi(x + mu).  Sites are lexicographic with x fastest,
site = x + Lx*(y + Ly*(z + Lz*t)).

The paper states no fermion boundary condition; the oracle uses periodic
x, y, z and, when ``antiperiodic_t`` is set, a factor -1 on every hop that
crosses the time boundary.  The sign is applied to the shifted field here,
never folded into the links.
"""

import numpy as np

from .gamma import GAMMA, ONE, spin_apply

# axis of mu in a grid shaped (..., Lt, Lz, Ly, Lx, 4 or 3, 3), counted from the end
_AXIS_FROM_END = {0: -3, 1: -4, 2: -5, 3: -6}


def to_grid(f: np.ndarray, dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    return f.reshape(f.shape[:-3] + (lt, lz, ly, lx) + f.shape[-2:])


def from_grid(g: np.ndarray) -> np.ndarray:
    return g.reshape(g.shape[:-6] + (-1,) + g.shape[-2:])


def shift(g: np.ndarray, mu: int, direction: int, antiperiodic_t: bool) -> np.ndarray:
    """Return the grid field evaluated at x + direction*mu (direction = +1 or -1),
    including the time boundary sign."""
    ax = _AXIS_FROM_END[mu]
    out = np.roll(g, -direction, axis=ax)
    if mu == 3 and antiperiodic_t:
        out = out.copy()
        lt = g.shape[ax]
        idx = [slice(None)] * g.ndim
        # psi(x+t) at t = Lt-1 wraps to t = 0; psi(x-t) at t = 0 wraps to t = Lt-1
        idx[ax] = lt - 1 if direction > 0 else 0
        out[tuple(idx)] *= -1.0
    return out


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _colour(u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Colour matrix times spinor: out[..., s, a] = sum_b u[..., a, b] g[..., s, b]."""
    return np.matmul(g, np.swapaxes(u, -1, -2))


def dw(U, psi, M5: float, dims, antiperiodic_t: bool = True) -> np.ndarray:
    """D_w psi following eq.(wilson).  U = None means all links are zero, which
    leaves only the diagonal (4 + M5) of eq.(wilson)."""
    f = to_grid(psi, dims)
    out = (4.0 + M5) * f
    if U is not None:
        ug = to_grid(U, dims)  # (4, Lt, Lz, Ly, Lx, 3, 3)
        for mu in range(4):
            u_fwd = ug[mu]                                             # U_mu(x)
            u_bwd = _dag(np.roll(ug[mu], 1, axis=_AXIS_FROM_END[mu]))  # U_mu(x-mu)^dag
            t_fwd = spin_apply(ONE - GAMMA[mu], _colour(u_fwd, shift(f, mu, +1, antiperiodic_t)))
            t_bwd = spin_apply(ONE + GAMMA[mu], _colour(u_bwd, shift(f, mu, -1, antiperiodic_t)))
            out = out - 0.5 * (t_fwd + t_bwd)
    return from_grid(out)


def dw_dag(U, psi, M5: float, dims, antiperiodic_t: bool = True) -> np.ndarray:
    """The adjoint of eq.(wilson) as a stencil: the transpose of each hop with its
    link daggered.  The term (1 - gamma_mu) U_mu(x) delta(x+mu, y) becomes
    (1 - gamma_mu) U_mu(y-mu)^dag acting on psi(y - mu), and likewise for the
    backward term (gamma_mu is Hermitian, boundary signs are real)."""
    f = to_grid(psi, dims)
    out = (4.0 + M5) * f
    if U is not None:
        ug = to_grid(U, dims)
        for mu in range(4):
            u_fwd = ug[mu]
            u_bwd = _dag(np.roll(ug[mu], 1, axis=_AXIS_FROM_END[mu]))
            t_a = spin_apply(ONE - GAMMA[mu], _colour(u_bwd, shift(f, mu, -1, antiperiodic_t)))
            t_b = spin_apply(ONE + GAMMA[mu], _colour(u_fwd, shift(f, mu, +1, antiperiodic_t)))
            out = out - 0.5 * (t_a + t_b)
    return from_grid(out)
