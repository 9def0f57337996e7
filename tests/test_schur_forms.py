"""The alternative Schur forms of Sec. 3: eq.(redblack1), D'_bb = I_bb - D_br I_rr^-1 D_rb,
and its row-scaled version, in the oracle (pinned against eq.(redblack) and the dense
system) and in the library's site-local tables (CPU, through the C-ABI)."""

import numpy as np
import pytest

from oracle import redblack
from paper_1501_04950_amd import dwa, synth


def _case(bc="random"):
    dims, Ls = (2, 2, 2, 4), 4
    rng = np.random.default_rng(1750)
    if bc == "random":
        b, c = rng.uniform(0.5, 2.5, Ls), rng.uniform(0.1, 1.9, Ls)
    else:
        b = c = np.array([0.4, 1.7, 2.9, 0.8])
    U = synth.su3_field(dims, 0.5, 1751)
    p = redblack.Params.make(dims, Ls, -1.7, 0.1, 0.8, b, c)
    return U, p, redblack.RedBlack(U, p)


def _bf(rb, p, seed):
    return synth.gaussian_field5(p.dims, p.Ls, seed) * rb.black


def test_redblack1_is_I_times_redblack():
    U, p, rb = _case()
    x = _bf(rb, p, 1)
    lhs = rb.Dbb1(x)
    rhs = rb.black * rb.I(rb.Dbb(x))
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


@pytest.mark.parametrize("form", [0, 1, 2])
def test_form_adjoints(form):
    U, p, rb = _case()
    A, Ad, _ = rb.schur_form(form)
    x, y = _bf(rb, p, 2), _bf(rb, p, 3)
    a = redblack.vdot(y, A(x))
    b = redblack.vdot(Ad(y), x)
    assert abs(a - b) <= 1e-13 * abs(a)


@pytest.mark.parametrize("bc", ["random", "zolotarev_like"])
def test_forms_share_the_solution(bc):
    """CGLS on each form reaches the solution of eq.(redblack) (and its residual); the
    row weights divide exactly the rows whose coefficient exceeds one."""
    U, p, rb = _case(bc)
    phi = _bf(rb, p, 4)
    x0, _ = redblack.cgls(rb.Dbb, rb.Dbb_dag, phi, 1e-13, 5000)
    w = rb.row_weights()
    big = np.maximum(p.b, p.c) > 1.0
    assert np.allclose(w[big], 1.0 / np.maximum(p.b, p.c)[big]) and np.all(w[~big] == 1.0)
    for form in (1, 2):
        A, Ad, to_rhs = rb.schur_form(form)
        x, info = redblack.cgls(A, Ad, to_rhs(phi), 1e-13, 5000)
        assert info.converged
        assert np.linalg.norm(x - x0) <= 1e-9 * np.linalg.norm(x0)
        assert np.linalg.norm(phi - rb.Dbb(x)) <= 1e-11 * np.linalg.norm(phi)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_row_weights_bound_every_row(seed):
    """The row scaling after eq.(redblack1): each row of the scaled operator keeps its D_w
    coefficients at most one, and rows already within one are left alone.  The
    coefficients of row s are read off the oracle's D_w-coefficient matrix of the block
    list of eq.(mobius1) (alpha = 1, so that row's largest entry is max(b_s, c_s)), with
    rows dominated by b and rows dominated by c both present."""
    dims, Ls = (2, 2, 2, 2), 8
    rng = np.random.default_rng(1760 + seed)
    b, c = rng.uniform(0.3, 2.0, Ls), rng.uniform(0.3, 2.5, Ls)
    b[0], c[0] = 1.6, 2.2   # c dominates, above one
    b[1], c[1] = 2.1, 0.4   # b dominates, above one
    b[2], c[2] = 0.7, 0.9   # within one
    p = redblack.Params.make(dims, Ls, -1.7, 0.1, 1.0, b, c)
    rb = redblack.RedBlack(synth.unit_field(dims), p)
    w = rb.row_weights()
    rowmax = np.abs(rb.bg_matrix()).reshape(Ls, 4, 4 * Ls).max(axis=(1, 2))
    assert np.all(w * rowmax <= 1.0 + 1e-14)
    assert np.allclose((w * rowmax)[rowmax > 1.0], 1.0, atol=1e-14)
    assert np.all(w[rowmax <= 1.0] == 1.0)


@pytest.mark.skipif(not __import__("os").path.exists(dwa.LIB_PATH), reason="libdwa.so not built")
def test_library_tables_for_the_forms():
    """Kinds 9..11 of dwa_debug_smatrix: (I_1 G)^T, W I_1 G and its transpose, with W the
    row weights of the oracle; kind 8 (I_1 G) is pinned to the oracle's literal I in
    test_abi."""
    U, p, rb = _case("zolotarev_like")
    kw = dict(dims=p.dims, Ls=p.Ls, M5=p.M5, m=p.m, alpha=p.alpha, b=p.b, c=p.c)
    I = dwa.dwa_debug_smatrix(kind="I_alpha", **kw)
    IT = dwa.dwa_debug_smatrix(kind="I_alpha_T", **kw)
    WI = dwa.dwa_debug_smatrix(kind="W_I", **kw)
    WIT = dwa.dwa_debug_smatrix(kind="W_I_T", **kw)
    w = rb.row_weights()
    for ch in range(2):
        assert np.allclose(IT[ch], I[ch].T, rtol=0, atol=1e-15)
        assert np.allclose(WI[ch], w[:, None] * I[ch], rtol=0, atol=1e-15)
        assert np.allclose(WIT[ch], WI[ch].T, rtol=0, atol=1e-15)
