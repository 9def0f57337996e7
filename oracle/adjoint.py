"""Gradients of a real scalar of the 4D propagator, by the adjoint-state method.

The scalar is L = Re <eta', y_1>, with y_1 the propagator of eq.(tosolve) for the
source eta (y_1 = extraction of psi, D_alpha(m) psi = rho = D_1(1) P (eta, 0, ...)).
Writing f = E^dag eta' for the 5D field whose extraction pairs with eta'
(Re <eta', E psi> = Re <f, psi>), and lambda for the solution of
    D_alpha(m)^dag lambda = f,
every first-order change of L is
    dL = Re <lambda, d rho - (d D_alpha) psi>.
This module evaluates that formula term by term from the literal block matrix of
eq.(mobius1) (``mobius.block_terms``) and the literal Wilson operator of
eq.(wilson); it shares nothing with the GPU path.

Gradient convention: for a complex parameter z the gradient g has
g = dL/dRe z + i dL/dIm z, so that dL = Re sum conj(g) dz; for the links the
perturbation of U_mu(x) enters the backward hop as its conjugate transpose (the
links are treated as unconstrained complex 3 x 3 matrices).  Real parameters
(alpha, b_i, c_i) get ordinary derivatives.
"""

import numpy as np

from . import mobius, redblack
from .gamma import GAMMA, ONE, P_MINUS, P_PLUS, spin_apply
from .wilson import dw, from_grid, shift, to_grid


def source5(eta, Ls):
    """P b with b = (eta, 0, ..., 0) (eq.(eqP), eq.(tosolve))."""
    return mobius.apply_P(mobius.embed_source(eta, Ls))


def extraction_adjoint(eta_p, Ls):
    """f = E^dag eta' for the extraction y_1 = P- psi_1 + P+ psi_Ls (eq.(tosolve1)):
    Re <eta', E psi> = Re <f, psi> with f_1 = P- eta', f_Ls = P+ eta'."""
    f = np.zeros((Ls,) + eta_p.shape, dtype=np.complex128)
    f[0] += spin_apply(P_MINUS, eta_p)
    f[Ls - 1] += spin_apply(P_PLUS, eta_p)
    return f


def loss(U, eta, eta_p, p: redblack.Params, tol=1e-13):
    """L = Re <eta', y_1>."""
    y1, _ = redblack.propagator(U, eta, p, tol=tol)
    return float(np.vdot(eta_p.reshape(-1), y1.reshape(-1)).real)


def dw_link_grad(a, b, dims, antiperiodic_t=True):
    """Gradient of Re <a, D_w(U) b> with respect to the links (shape (4, V, 3, 3)).

    From eq.(wilson), U_mu(x) appears in the forward hop at x, -1/2 (1 - g_mu) U_mu(x)
    b(x + mu), and (daggered) in the backward hop at x + mu, -1/2 (1 + g_mu)
    U_mu(x)^dag b(x).  With the boundary sign s of the hop across the time edge,
        g_mu(x)_{ij} = -1/2 s sum_spin [ ((1 - g_mu) a(x))_i conj(b(x + mu))_j
                                         + b(x)_i conj(((1 + g_mu) a(x + mu))_j) ].
    a and b may carry leading axes (slices), which are summed."""
    A = to_grid(a, dims)
    B = to_grid(b, dims)
    lead = "".join("klmn"[: A.ndim - 6])
    spec = f"{lead}tzyxsi,{lead}tzyxsj->tzyxij"
    out = []
    for mu in range(4):
        a_f = spin_apply(ONE - GAMMA[mu], A)
        b_up = shift(B, mu, +1, antiperiodic_t)            # s * b(x + mu)
        a_b = shift(spin_apply(ONE + GAMMA[mu], A), mu, +1, antiperiodic_t)  # s * (..)(x + mu)
        g = np.einsum(spec, a_f, np.conj(b_up)) + np.einsum(spec, B, np.conj(a_b))
        out.append(-0.5 * g.reshape(-1, 3, 3))
    return np.stack(out)


def _dw_part_terms(x5, m, alpha, p):
    """For D_alpha(m) (block terms of eq.(mobius1)) applied to the 5D field x5, the
    list of (row, coefficient of D_w, D_w input) of its D_w-dependent part: a block
    coef * D_{i+} R (resp. coef * D_{i-} R) contributes coef * b_i D_w (R x_j)
    (resp. coef * c_i D_w (R x_j))."""
    out = []
    for (i, j, coef, kind, right) in mobius.block_terms(p.Ls, m, alpha):
        bc = p.b[i] if kind == "+" else p.c[i]
        out.append((i, coef * bc, spin_apply(right, x5[j]), kind))
    return out


def adjoint_field(U, eta_p, p: redblack.Params, tol=1e-13, maxiter=200000, f5=None):
    """lambda with D_alpha(m)^dag lambda = E^dag eta' (or = f5, a general 5D cotangent,
    when given), by CGLS on the full 5D system (no red-black), so it is independent of
    the Schur algebra."""
    rb = redblack.RedBlack(U, p)
    f = extraction_adjoint(eta_p, p.Ls) if f5 is None else f5
    lam, info = redblack.cgls(rb.D_dag, rb.D, f, tol, maxiter)
    return lam, info


def gradients(U, eta, eta_p, p: redblack.Params, tol=1e-13, f5=None):
    """dL with respect to the links, eta, alpha, b_i and c_i, for L = Re <eta', y_1> (or,
    with f5 given, for L = Re <f5, psi> of the whole 5D solution, whose alpha derivative
    does not vanish).  Returns a dict with 'U' (4, V, 3, 3), 'eta' (V, 4, 3), 'alpha'
    (float), 'b' and 'c' (Ls,) and the forward psi and adjoint lambda."""
    Ls, dims = p.Ls, p.dims
    _, _, psi = redblack.propagator(U, eta, p, tol=tol, return_psi=True)
    lam, _ = adjoint_field(U, eta_p, p, tol=tol, f5=f5)
    pb = source5(eta, Ls)
    dwf = lambda x: dw(U, x, p.M5, dims, p.antiperiodic_t)

    # links: rho = D_1(1) P b (alpha = 1, m = 1) and D_alpha(m) psi depend on U only
    # through D_w in their block terms
    gU = np.zeros_like(U)
    for (i, w, x, _) in _dw_part_terms(pb, 1.0, 1.0, p):
        gU += w * dw_link_grad(lam[i], x, dims, p.antiperiodic_t)
    for (i, w, x, _) in _dw_part_terms(psi, p.m, p.alpha, p):
        gU -= w * dw_link_grad(lam[i], x, dims, p.antiperiodic_t)

    # b_i, c_i: the blocks are linear in them; d/db_i of coef * (b_i D_w + 1) R x_j is
    # coef * D_w R x_j in row i, and likewise for c_i with the D_{i-} blocks
    gb = np.zeros(Ls)
    gc = np.zeros(Ls)
    for sign, x5, m, alpha in ((+1.0, pb, 1.0, 1.0), (-1.0, psi, p.m, p.alpha)):
        for (i, j, coef, kind, right) in mobius.block_terms(Ls, m, alpha):
            val = sign * np.vdot(lam[i].reshape(-1), (coef * dwf(spin_apply(right, x5[j]))).reshape(-1)).real
            if kind == "+":
                gb[i] += val
            else:
                gc[i] += val

    # alpha: every block of eq.(mobius1) is affine in alpha, so
    # d D_alpha / d alpha = D_{alpha+1} - D_alpha exactly; rho does not depend on alpha
    dD = (mobius.apply_D(U, psi, p.M5, p.m, p.alpha + 1.0, p.b, p.c, dims, p.antiperiodic_t)
          - mobius.apply_D(U, psi, p.M5, p.m, p.alpha, p.b, p.c, dims, p.antiperiodic_t))
    galpha = -float(np.vdot(lam.reshape(-1), dD.reshape(-1)).real)

    # eta: rho is linear in eta, dL = Re <lambda, D_1(1) P (d eta, 0, ...)>, so the
    # gradient is the first slice of P^dag D_1(1)^dag lambda (P is unitary)
    t = mobius.apply_D_dag(U, lam, p.M5, 1.0, 1.0, p.b, p.c, dims, p.antiperiodic_t)
    geta = mobius.apply_P_inv(t)[0]
    return {"U": gU, "eta": geta, "alpha": galpha, "b": gb, "c": gc, "psi": psi, "lambda": lam}
