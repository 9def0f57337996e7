"""Red-black preconditioning of eq.(redblack), CG on the normal equations and
the 4D propagator of eq.(tosolve)/(tosolve1).

Readings of points the paper leaves open:
* parity p(x) = (x + y + z + t) mod 2; black = even sites, red = odd sites;
* I is the 4D-site-local part of D_alpha(m): D_alpha with every link set to
  zero, so D_w reduces to its diagonal (4 + M5).  It couples all slices and
  spins of one site and is the same matrix at every site; its inverse is taken
  as a dense (4 Ls) x (4 Ls) inverse;
* the hopping blocks D_rb, D_br are D_alpha(U) - D_alpha(U = 0), restricted
  between parities (they carry the -1/2 of eq.(wilson));
* "CG on the normal equation" (Sec. 3) is CGLS on D_bb^dag D_bb x = D_bb^dag phi;
  it stops on the recursive residual |phi - D_bb x| / |phi| <= tol.

Half-lattice fields are full-lattice arrays that vanish on the other parity.
"""

from dataclasses import dataclass, field

import numpy as np

from . import mobius
from .gamma import GAMMA5, P_MINUS, P_PLUS, spin_apply


def parity(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


@dataclass
class Params:
    """Physical parameters of D_alpha(m); b, c are per-slice (length Ls)."""
    dims: tuple
    Ls: int
    M5: float
    m: float
    alpha: float
    b: np.ndarray
    c: np.ndarray
    antiperiodic_t: bool = True

    @staticmethod
    def make(dims, Ls, M5, m, alpha, b, c, antiperiodic_t=True):
        bb = np.full(Ls, float(b)) if np.isscalar(b) else np.asarray(b, dtype=float)
        cc = np.full(Ls, float(c)) if np.isscalar(c) else np.asarray(c, dtype=float)
        return Params(tuple(dims), Ls, float(M5), float(m), float(alpha), bb, cc,
                      antiperiodic_t)

    def with_(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Params(**d)


def vdot(a, b) -> complex:
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def norm(a) -> float:
    return float(np.linalg.norm(a.reshape(-1)))


class RedBlack:
    """The pieces of eq.(redblack) for one gauge field and parameter set."""

    def __init__(self, U, p: Params):
        self.U, self.p = U, p
        par = parity(p.dims)
        self.black = (par == 0).astype(float)[None, :, None, None]
        self.red = (par == 1).astype(float)[None, :, None, None]
        self.I_mat = self._site_local_matrix()
        self.I_inv = np.linalg.inv(self.I_mat)

    # --- D_alpha and its parts -------------------------------------------
    def D(self, psi5, U="self"):
        p = self.p
        U = self.U if isinstance(U, str) else U
        return mobius.apply_D(U, psi5, p.M5, p.m, p.alpha, p.b, p.c, p.dims, p.antiperiodic_t)

    def D_dag(self, psi5, U="self"):
        p = self.p
        U = self.U if isinstance(U, str) else U
        return mobius.apply_D_dag(U, psi5, p.M5, p.m, p.alpha, p.b, p.c, p.dims,
                                  p.antiperiodic_t)

    def _site_local_matrix(self):
        """(4 Ls) x (4 Ls) matrix of D_alpha(U = 0) on one site, index s*4 + spin
        (colour is untouched)."""
        p = self.p
        n = 4 * p.Ls
        mat = np.zeros((n, n), dtype=np.complex128)
        for s in range(p.Ls):
            for spin in range(4):
                e = np.zeros((p.Ls, 1, 4, 3), dtype=np.complex128)
                e[s, 0, spin, 0] = 1.0
                col = mobius.apply_D(None, e, p.M5, p.m, p.alpha, p.b, p.c, (1, 1, 1, 1))
                mat[:, s * 4 + spin] = col[:, 0, :, 0].reshape(-1)
        return mat

    def bg_matrix(self):
        """(4 Ls) x (4 Ls) site matrix of the D_w parts of eq.(mobius1), index s*4 + spin:
        block (i, j, scalar, D_{i+-}, S) contributes scalar * (b_i for D_{i+}, c_i for
        D_{i-}) * S, so that D_alpha = D_w (this matrix) + (the parts without D_w)."""
        p = self.p
        mat = np.zeros((4 * p.Ls, 4 * p.Ls), dtype=np.complex128)
        for i, j, scal, sign, spin in mobius.block_terms(p.Ls, p.m, p.alpha):
            coef = p.b[i] if sign == "+" else p.c[i]
            mat[4 * i:4 * i + 4, 4 * j:4 * j + 4] += scal * coef * spin
        return mat

    def mix_matrix(self, kind):
        """The site matrix (index s*4 + spin) of a fifth-dimension mix of the red-black
        operators, from the zero-link block I = I_1 G and BG: N = B I_1^-1 = BG I^-1 and its
        transpose NT, G^-1 I_1^-1 = I^-1, G B^T g5 = (BG)^T g5 (all real), BG itself."""
        Ls = self.p.Ls
        I, BG = self.I_mat, self.bg_matrix()
        g5 = np.kron(np.eye(Ls), GAMMA5)
        Iinv = np.linalg.inv(I)
        return {"identity": np.eye(4 * Ls), "BG": BG, "N": BG @ Iinv, "NT": (BG @ Iinv).T,
                "Ginv_Iinv": Iinv, "G_BT_g5": BG.T @ g5, "I_alpha": I}[kind]

    def site_apply(self, mat, psi5):
        """A (4 Ls) x (4 Ls) site matrix (index s*4 + spin) applied at every site."""
        return self._site_apply(mat, psi5)

    def _site_apply(self, mat, psi5):
        Ls = self.p.Ls
        m4 = mat.reshape(Ls, 4, Ls, 4)
        return np.einsum("aibj,bxjc->axic", m4, psi5)

    def I(self, psi5):
        return self._site_apply(self.I_mat, psi5)

    def I_inv_apply(self, psi5):
        return self._site_apply(self.I_inv, psi5)

    def I_inv_dag_apply(self, psi5):
        return self._site_apply(np.conj(self.I_inv.T), psi5)

    def hop(self, psi5):
        """The hopping part D_alpha(U) - D_alpha(0)."""
        return self.D(psi5) - self.D(psi5, U=None)

    def hop_dag(self, psi5):
        return self.D_dag(psi5) - self.D_dag(psi5, U=None)

    def D_rb(self, xb):
        return self.red * self.hop(self.black * xb)

    def D_br(self, xr):
        return self.black * self.hop(self.red * xr)

    # --- eq.(redblack) ---------------------------------------------------
    def Dbb(self, xb):
        """D_bb x = x - I_bb^-1 D_br I_rr^-1 D_rb x."""
        t = self.I_inv_apply(self.D_rb(xb))
        return xb - self.I_inv_apply(self.D_br(t))

    def Dbb_dag(self, yb):
        """D_bb^dag y = y - D_rb^dag I_rr^-dag D_br^dag I_bb^-dag y."""
        t = self.I_inv_dag_apply(self.black * yb)
        t = self.red * self.hop_dag(t)
        t = self.I_inv_dag_apply(t)
        return self.black * (yb - self.hop_dag(t))

    # --- eq.(redblack1) and its row-scaled form (Sec. 3) --------------------
    def I_dag_apply(self, psi5):
        return self._site_apply(np.conj(self.I_mat.T), psi5)

    def Dbb1(self, xb):
        """D'_bb x = I_bb x - D_br I_rr^-1 D_rb x (eq.(redblack1))."""
        return self.black * self.I(self.black * xb) - self.D_br(self.I_inv_apply(self.D_rb(xb)))

    def Dbb1_dag(self, yb):
        """D'_bb^dag y = I_bb^dag y - D_rb^dag I_rr^-dag D_br^dag y."""
        t = self.red * self.hop_dag(self.black * yb)
        t = self.I_inv_dag_apply(t)
        return self.black * (self.I_dag_apply(self.black * yb) - self.hop_dag(t))

    def row_weights(self):
        """The row scaling described after eq.(redblack1): row s (the output slice, the row
        that holds the coefficients b_s, c_s) is divided by its coefficient when that
        exceeds one.  Reading: the coefficient of row s is max(b_s, c_s) (b_s = c_s =
        omega_s for Zolotarev coefficients)."""
        p = self.p
        return 1.0 / np.maximum(1.0, np.maximum(np.abs(p.b), np.abs(p.c)))

    def scale_rows(self, psi5):
        return self.row_weights()[:, None, None, None] * psi5

    def schur_form(self, form):
        """(apply A, apply A^dag, rhs map) of the Schur system of form 0 (eq.(redblack)),
        1 (eq.(redblack1)) or 2 (eq.(redblack1) with scaled rows); every form has the
        solution of D_bb x = phi'."""
        if form == 0:
            return self.Dbb, self.Dbb_dag, lambda phi: phi
        if form == 1:
            return self.Dbb1, self.Dbb1_dag, lambda phi: self.black * self.I(phi)
        w = self.scale_rows
        return (lambda x: w(self.Dbb1(x)), lambda y: self.Dbb1_dag(w(y)),
                lambda phi: w(self.black * self.I(phi)))

    def schur_rhs(self, rho):
        """phi' = I_bb^-1 (rho_b - D_br I_rr^-1 rho_r)."""
        t = self.I_inv_apply(self.red * rho)
        return self.I_inv_apply(self.black * rho - self.D_br(t))

    def reconstruct_red(self, psi_b, rho):
        """psi_r = I_rr^-1 (rho_r - D_rb psi_b)."""
        return self.I_inv_apply(self.red * rho - self.D_rb(psi_b))


@dataclass
class SolveInfo:
    iters: int = 0
    converged: bool = False
    rel_resid_recursive: float = float("nan")
    rel_resid_true: float = float("nan")
    history: list = field(default_factory=list)


def cgls(apply_A, apply_Adag, rhs, tol, maxiter, x0=None):
    """Conjugate gradient on the normal equations A^dag A x = A^dag rhs (CGLS).

    x_0 = 0 (or x0), r = rhs - A x, z = A^dag r, p = z, gamma = |z|^2; then
        q = A p, a = gamma / |q|^2, x += a p, r -= a q,
        z = A^dag r, gamma' = |z|^2, p = z + (gamma'/gamma) p
    until |r| / |rhs| <= tol (r is the recursive residual)."""
    info = SolveInfo()
    bnorm = norm(rhs)
    if bnorm == 0.0:
        info.converged = True
        return np.zeros_like(rhs), info
    x = np.zeros_like(rhs) if x0 is None else x0.copy()
    r = rhs - apply_A(x) if x0 is not None else rhs.copy()
    z = apply_Adag(r)
    p = z.copy()
    gamma = norm(z) ** 2
    rel = norm(r) / bnorm
    info.history.append(rel)
    k = 0
    while rel > tol and k < maxiter:
        q = apply_A(p)
        a = gamma / norm(q) ** 2
        x = x + a * p
        r = r - a * q
        z = apply_Adag(r)
        gamma_new = norm(z) ** 2
        p = z + (gamma_new / gamma) * p
        gamma = gamma_new
        k += 1
        rel = norm(r) / bnorm
        info.history.append(rel)
    info.iters = k
    info.converged = rel <= tol
    info.rel_resid_recursive = rel
    info.rel_resid_true = norm(rhs - apply_A(x)) / bnorm
    return x, info


def source_rhs(U, eta, p: Params):
    """rho = D_1(1) P b with b = (eta, 0, ..., 0) (eq.(tosolve)): the right-hand
    side is always built with alpha = 1 and mass 1."""
    b5 = mobius.embed_source(eta, p.Ls)
    return mobius.apply_D(U, mobius.apply_P(b5), p.M5, 1.0, 1.0, p.b, p.c, p.dims,
                          p.antiperiodic_t)


def extract_y1(psi5):
    """y_1 = z_1 with z = P^-1 psi (eq.(tosolve1)); z_1 = P- psi_1 + P+ psi_Ls."""
    return mobius.apply_P_inv(psi5)[0]


def propagator(U, eta, p: Params, tol=1e-10, maxiter=100000, return_psi=False):
    """The 4D propagator y_1 through D_alpha(m) P z = D_1(1) P b, solved with the
    red-black form of eq.(redblack) and CGLS; psi = P z is the 5D solution."""
    rb = RedBlack(U, p)
    rho = source_rhs(U, eta, p)
    phi = rb.schur_rhs(rho)
    psi_b, info = cgls(rb.Dbb, rb.Dbb_dag, phi, tol, maxiter)
    psi = psi_b + rb.reconstruct_red(psi_b, rho)
    y1 = extract_y1(psi)
    if return_psi:
        return y1, info, psi
    return y1, info


def propagator_form(U, eta, p: Params, form, tol=1e-10, maxiter=100000):
    """y_1 with the Schur system in form 0, 1 or 2 (see RedBlack.schur_form), CGLS stopping
    on that form's own residual."""
    rb = RedBlack(U, p)
    rho = source_rhs(U, eta, p)
    phi = rb.schur_rhs(rho)
    A, Ad, to_rhs = rb.schur_form(form)
    psi_b, info = cgls(A, Ad, to_rhs(phi), tol, maxiter)
    psi = psi_b + rb.reconstruct_red(psi_b, rho)
    return extract_y1(psi), info


def solve_unpreconditioned(U, rho, p: Params, tol=1e-12, maxiter=100000):
    """CGLS on the full 5D system D_alpha(m) psi = rho, without red-black."""
    rb = RedBlack(U, p)
    return cgls(rb.D, rb.D_dag, rho, tol, maxiter)


def chiral_parts(psi):
    return spin_apply(P_PLUS, psi), spin_apply(P_MINUS, psi)
