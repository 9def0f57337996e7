"""Pins of the oracle's adjoint-state gradients (oracle/adjoint.py).

The gradient of L = Re <eta', y_1> is pinned by
  * central finite differences of L itself (two propagator solves per direction,
    step 1e-6, solves at 1e-13) in random directions of the links, eta, b_i, c_i
    and alpha, with per-slice b_i, c_i that have no symmetry;
  * dL/dalpha = 0, since y_1 does not depend on alpha (Sec. 2, eq.(tosolve1));
  * the gamma_5 identity dL/deta = g5 y_1[g5 eta'], which holds when the 4D operator
    is g5-Hermitian: for constant b_i, c_i or ones symmetric under s -> Ls - 1 - s
    (the transfer-matrix product of App. A is then a symmetric product); with
    asymmetric coefficients it must fail.
"""

import numpy as np
import pytest

from oracle import adjoint, mobius, redblack
from oracle.gamma import GAMMA5, spin_apply
from paper_1501_04950_amd import synth

DIMS, LS = (2, 2, 2, 4), 4
EPS = 1e-6


def _setup(b, c, alpha=0.8, m=0.1):
    U = synth.su3_field(DIMS, 0.5, 77)
    p = redblack.Params.make(DIMS, LS, -1.8, m, alpha, b, c)
    eta = synth.gaussian_source(DIMS, 3)
    eta_p = synth.gaussian_source(DIMS, 4)
    return U, p, eta, eta_p


@pytest.fixture(scope="module")
def asym():
    rng = np.random.default_rng(11)
    b, c = rng.uniform(1.0, 2.0, LS), rng.uniform(0.1, 0.9, LS)
    U, p, eta, eta_p = _setup(b, c)
    g = adjoint.gradients(U, eta, eta_p, p)
    return U, p, eta, eta_p, g


def _fd(fun):
    return (fun(EPS) - fun(-EPS)) / (2 * EPS)


def _close(fd, adj, scale):
    assert abs(fd - adj) <= 1e-6 * max(abs(adj), scale), (fd, adj)


def test_link_gradient_matches_finite_differences(asym):
    U, p, eta, eta_p, g = asym
    rng = np.random.default_rng(12)
    L0 = adjoint.loss(U, eta, eta_p, p)
    for _ in range(2):
        d = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
        fd = _fd(lambda e: adjoint.loss(U + e * d, eta, eta_p, p))
        _close(fd, float(np.vdot(g["U"].ravel(), d.ravel()).real), abs(L0))


def test_source_gradient_matches_finite_differences(asym):
    U, p, eta, eta_p, g = asym
    rng = np.random.default_rng(13)
    d = rng.normal(size=eta.shape) + 1j * rng.normal(size=eta.shape)
    fd = _fd(lambda e: adjoint.loss(U, eta + e * d, eta_p, p))
    _close(fd, float(np.vdot(g["eta"].ravel(), d.ravel()).real), abs(adjoint.loss(U, eta, eta_p, p)))


@pytest.mark.parametrize("which", ["b", "c"])
def test_moebius_coefficient_gradients_match_finite_differences(asym, which):
    U, p, eta, eta_p, g = asym
    rng = np.random.default_rng(14 if which == "b" else 15)
    d = rng.normal(size=LS)
    base = getattr(p, which)
    fd = _fd(lambda e: adjoint.loss(U, eta, eta_p, p.with_(**{which: base + e * d})))
    _close(fd, float(g[which] @ d), abs(adjoint.loss(U, eta, eta_p, p)))


def test_alpha_gradient_vanishes(asym):
    U, p, eta, eta_p, g = asym
    L0 = adjoint.loss(U, eta, eta_p, p)
    fd = _fd(lambda e: adjoint.loss(U, eta, eta_p, p.with_(alpha=p.alpha + e)))
    assert abs(g["alpha"]) <= 1e-10 * abs(L0)
    assert abs(fd) <= 1e-6 * abs(L0)


@pytest.mark.parametrize("b,c,holds", [
    (1.5, 0.5, True),
    (np.array([1.2, 1.7, 1.7, 1.2]), np.array([0.3, 0.6, 0.6, 0.3]), True),
    (np.array([1.2, 1.7, 1.5, 1.1]), np.array([0.3, 0.6, 0.4, 0.2]), False),
])
def test_source_gradient_gamma5_identity(b, c, holds):
    U, p, eta, eta_p = _setup(b, c)
    g = adjoint.gradients(U, eta, eta_p, p)
    y5, _ = redblack.propagator(U, spin_apply(GAMMA5, eta_p), p, tol=1e-13)
    r = np.linalg.norm(g["eta"] - spin_apply(GAMMA5, y5)) / np.linalg.norm(g["eta"])
    assert (r < 1e-10) == holds, r


def test_P_is_unitary():
    rng = np.random.default_rng(16)
    a = rng.normal(size=(LS, 8, 4, 3)) + 1j * rng.normal(size=(LS, 8, 4, 3))
    b = rng.normal(size=(LS, 8, 4, 3)) + 1j * rng.normal(size=(LS, 8, 4, 3))
    lhs = np.vdot(mobius.apply_P(a).ravel(), mobius.apply_P(b).ravel())
    assert abs(lhs - np.vdot(a.ravel(), b.ravel())) < 1e-12 * abs(lhs)
    assert np.allclose(mobius.apply_P_inv(mobius.apply_P(a)), a, atol=1e-14)


def test_adjoint_field_solves_adjoint_system(asym):
    U, p, eta, eta_p, g = asym
    rb = redblack.RedBlack(U, p)
    f = adjoint.extraction_adjoint(eta_p, LS)
    lam = g["lambda"]
    assert np.linalg.norm(rb.D_dag(lam) - f) <= 1e-12 * np.linalg.norm(f)
    # and f pairs with psi as the extraction does: Re <f, psi> = Re <eta', y_1>
    y1 = redblack.extract_y1(g["psi"])
    assert abs(np.vdot(f.ravel(), g["psi"].ravel()) - np.vdot(eta_p.ravel(), y1.ravel())) < 1e-12


def test_alpha_gradient_formula_on_a_5d_loss(asym):
    """The alpha term of the adjoint gradient, on a loss whose alpha derivative does not
    vanish: L5 = Re <f5, psi> of the whole 5D solution of D_alpha psi = D_1(1) P b
    (rho does not depend on alpha, eq.(tosolve)).  The oracle's dL5/dalpha (lambda from
    D_alpha^dag lambda = f5) equals central finite differences of L5 in alpha, and is
    far from zero, so its sign is pinned (for y_1-losses it is zero, eq.(tosolve1))."""
    U, p, eta, eta_p, _ = asym
    f5 = synth.gaussian_field5(DIMS, LS, 9)
    g = adjoint.gradients(U, eta, eta_p, p, f5=f5)

    def L5(d):
        q = p.with_(alpha=p.alpha + d)
        _, _, psi = redblack.propagator(U, eta, q, tol=1e-13, return_psi=True)
        return float(np.vdot(f5.reshape(-1), psi.reshape(-1)).real)

    fd = _fd(L5)
    assert abs(fd) > 1e-2
    _close(fd, g["alpha"], abs(fd))
