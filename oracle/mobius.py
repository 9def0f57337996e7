"""The alpha-Moebius domain-wall operator D_alpha(m) of eq.(mobius1), literally.

D_alpha(m) is an Ls x Ls block matrix over the fifth dimension whose blocks are
4D operators built from
    D_{i+} = b_i D_w + 1,   D_{i-} = c_i D_w - 1            (eq.(coeff))
and the chiral projectors P+-.  Slices are 0-based here: s = 0 .. Ls-1 stands
for the paper's i_5 = 1 .. Ls.  The per-slice b_i, c_i belong to the row, the
output slice, exactly as D_{i+-} appear in row i of eq.(mobius1).

The non-zero blocks, written as (row, column, scalar, D_{i+} or D_{i-}, right
spin factor), are:
    row 0      : (0, 0, 1, +, P- + alpha P+), (0, 1, alpha, -, P-), (0, Ls-1, -m, -, P+)
    row i      : (i, i-1, alpha, -, P+), (i, i, alpha, +, 1), (i, i+1, alpha, -, P-)
    row Ls-1   : (Ls-1, 0, -m, -, P-), (Ls-1, Ls-2, alpha, -, P+),
                 (Ls-1, Ls-1, 1, +, P+ + alpha P-)
Blocks that land on the same (row, column), as happens for Ls = 2, are summed.
"""

import numpy as np

from .gamma import ONE, P_MINUS, P_PLUS, spin_apply
from .wilson import dw, dw_dag


def block_terms(Ls: int, m: float, alpha: float):
    """The list of non-zero blocks of eq.(mobius1)."""
    if Ls < 2:
        raise ValueError("Ls must be at least 2")
    t = [(0, 0, 1.0, "+", P_MINUS + alpha * P_PLUS),
         (0, 1, alpha, "-", P_MINUS),
         (0, Ls - 1, -m, "-", P_PLUS)]
    for i in range(1, Ls - 1):
        t += [(i, i - 1, alpha, "-", P_PLUS),
              (i, i, alpha, "+", ONE),
              (i, i + 1, alpha, "-", P_MINUS)]
    t += [(Ls - 1, 0, -m, "-", P_MINUS),
          (Ls - 1, Ls - 2, alpha, "-", P_PLUS),
          (Ls - 1, Ls - 1, 1.0, "+", P_PLUS + alpha * P_MINUS)]
    return t


def apply_D(U, psi5, M5, m, alpha, b, c, dims, antiperiodic_t=True):
    """D_alpha(m) psi for a 5D field psi5 of shape (Ls, V, 4, 3): every block of
    eq.(mobius1) acts on its column slice and adds into its row slice.  The D_w
    of all blocks are evaluated in one call on the stacked inputs."""
    Ls = psi5.shape[0]
    terms = block_terms(Ls, m, alpha)
    inputs = np.stack([spin_apply(right, psi5[j]) for (_, j, _, _, right) in terms])
    dws = dw(U, inputs, M5, dims, antiperiodic_t)
    out = np.zeros_like(psi5)
    for k, (i, j, coef, kind, right) in enumerate(terms):
        if kind == "+":
            out[i] += coef * (b[i] * dws[k] + inputs[k])      # coef D_{i+} R psi_j
        else:
            out[i] += coef * (c[i] * dws[k] - inputs[k])      # coef D_{i-} R psi_j
    return out


def apply_D_dag(U, psi5, M5, m, alpha, b, c, dims, antiperiodic_t=True):
    """D_alpha(m)^dag psi: block (j, i) of the adjoint is the adjoint of block (i, j),
    (coef D_{i+-} R)^dag = coef* R^dag D_{i+-}^dag with D_{i+}^dag = b_i D_w^dag + 1 and
    D_{i-}^dag = c_i D_w^dag - 1 (b_i, c_i real)."""
    Ls = psi5.shape[0]
    terms = block_terms(Ls, m, alpha)
    rows = np.stack([psi5[i] for (i, _, _, _, _) in terms])
    dws = dw_dag(U, rows, M5, dims, antiperiodic_t)
    out = np.zeros_like(psi5)
    for k, (i, j, coef, kind, right) in enumerate(terms):
        if kind == "+":
            d = b[i] * dws[k] + rows[k]
        else:
            d = c[i] * dws[k] - rows[k]
        out[j] += np.conj(coef) * spin_apply(np.conj(right.T), d)
    return out


def apply_D_conventional(U, psi5, M5, m, b, c, dims, antiperiodic_t=True):
    """The conventional Moebius domain-wall operator, coded independently of
    eq.(mobius1):
        (D psi)_s = D_{s+} psi_s + D_{s-} (P- psi_{s+1} + P+ psi_{s-1})
    with the walls closed by psi_{Ls} -> -m psi_0 and psi_{-1} -> -m psi_{Ls-1}."""
    Ls = psi5.shape[0]
    dw_of = lambda f: dw(U, f, M5, dims, antiperiodic_t)
    out = np.zeros_like(psi5)
    for s in range(Ls):
        up = psi5[s + 1] if s + 1 < Ls else -m * psi5[0]
        dn = psi5[s - 1] if s - 1 >= 0 else -m * psi5[Ls - 1]
        hop5 = spin_apply(P_MINUS, up) + spin_apply(P_PLUS, dn)
        out[s] = (b[s] * dw_of(psi5[s]) + psi5[s]) + (c[s] * dw_of(hop5) - hop5)
    return out


def apply_P(psi5):
    """The matrix P of eq.(eqP): P- on the diagonal, P+ on the cyclic
    superdiagonal including the (Ls, 1) entry, (P psi)_i = P- psi_i + P+ psi_{i+1}."""
    Ls = psi5.shape[0]
    out = np.empty_like(psi5)
    for i in range(Ls):
        out[i] = spin_apply(P_MINUS, psi5[i]) + spin_apply(P_PLUS, psi5[(i + 1) % Ls])
    return out


def apply_P_inv(psi5):
    """Inverse of P: z_i = P- psi_i + P+ psi_{i-1} (cyclic)."""
    Ls = psi5.shape[0]
    out = np.empty_like(psi5)
    for i in range(Ls):
        out[i] = spin_apply(P_MINUS, psi5[i]) + spin_apply(P_PLUS, psi5[(i - 1) % Ls])
    return out


def apply_A(psi5, alpha):
    """A = diag(1, alpha, ..., alpha) of Sec. 2."""
    out = alpha * psi5
    out[0] = psi5[0]
    return out


def embed_source(eta, Ls):
    """b = (eta, 0, ..., 0): the 4D source in the first slice."""
    b = np.zeros((Ls,) + eta.shape, dtype=np.complex128)
    b[0] = eta
    return b
