"""Zolotarev coefficients of the alpha-Moebius operator (Sec. 3: the Zolotarev row of the
table and the paragraph on the ordering of the coefficients; App. A, eq.(polar) and
eq.(argument)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With per-slice coefficients b_i = c_i = omega_i the kernel of eq.(argument) is the Wilson
kernel a_i X_i = omega_i gamma_5 D_w, and eq.(polar) reads

    (S - 1)/(S + 1) = [prod (1 + omega_i H) - prod (1 - omega_i H)]
                      / [prod (1 + omega_i H) + prod (1 - omega_i H)],   H = gamma_5 D_w,

i.e. eps(H) = (1 - r(H)) / (1 + r(H)) with r(x) = prod_i (1 - omega_i x)/(1 + omega_i x).
eps approximates sign(H) where |r| is small on the spectrum [lambda_min, lambda_max] of |H|.
The omega_i that minimise max |r(x)| over that interval are Zolotarev's solution of his
third problem (the rational function of this product form with least deviation from zero
on an interval; it equioscillates at Ls + 1 points), in closed form through the Jacobi
elliptic function dn of modulus k' = sqrt(1 - (lambda_min/lambda_max)^2):

    1/omega_j = lambda_max dn((2j - 1) K(k') / (2 Ls), k'),   j = 1 .. Ls.

Reading (the paper takes its coefficients from code it does not print): "Zolotarev
coefficients" are these omega_j, placed on the diagonal as b_i = c_i = omega_i; the sign
approximation then has |1 - eps(x)| <= 2 delta / (1 - delta) with delta = max |r|.
The elliptic functions come from scipy.special (a library primitive).
"""

import numpy as np
from scipy import special


def omegas(lmin, lmax, Ls):
    """The Zolotarev coefficients omega_j, j = 1 .. Ls, in increasing order."""
    k = lmin / lmax
    kp2 = 1.0 - k * k                      # the parameter m = k'^2 of scipy's functions
    K = special.ellipkm1(k * k)            # K(m) for m = 1 - k^2, accurate near m = 1
    j = np.arange(1, Ls + 1)
    dn = special.ellipj((2 * j - 1) * K / (2 * Ls), kp2)[2]
    return np.sort(1.0 / (lmax * dn))


def ratio(x, om):
    """r(x) = prod_i (1 - omega_i x) / (1 + omega_i x)."""
    x = np.asarray(x, dtype=float)
    r = np.ones_like(x)
    for w in om:
        r = r * (1.0 - w * x) / (1.0 + w * x)
    return r


def eps(x, om):
    """The approximation to sign(x) of eq.(polar): (1 - r) / (1 + r)."""
    r = ratio(x, om)
    return (1.0 - r) / (1.0 + r)


def deviation(lmin, lmax, om, n=20001):
    """max |r| over [lmin, lmax] (log-spaced sampling plus the end points)."""
    x = np.geomspace(lmin, lmax, n)
    return float(np.max(np.abs(ratio(x, om))))


def concave(om):
    """The ordering of Sec. 3: the smallest coefficients at i_5 = 1 and i_5 = Ls, the
    largest in the centre (i_5 = Ls/2).  Sorted values are placed from both ends
    inwards, alternately at the front and at the back."""
    s = np.sort(np.asarray(om, dtype=float))
    out = np.empty_like(s)
    lo, hi = 0, len(s) - 1
    for k, v in enumerate(s):
        if k % 2 == 0:
            out[lo] = v
            lo += 1
        else:
            out[hi] = v
            hi -= 1
    return out


def wilson_kernel_spectrum(U, dims, M5, antiperiodic_t=True):
    """Eigenvalues of |gamma_5 D_w| on a small lattice, from the dense matrix of D_w
    (eq.(wilson)) built column by column with the oracle's own operator."""
    from . import overlap, wilson
    from .gamma import GAMMA5
    V = int(np.prod(dims))
    Dw = overlap.dense_matrix(lambda e: wilson.dw(U, e, M5, dims, antiperiodic_t), (V, 4, 3))
    g5 = np.kron(np.kron(np.eye(V), GAMMA5), np.eye(3))
    return np.sort(np.abs(np.linalg.eigvalsh(g5 @ Dw)))
