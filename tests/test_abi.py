"""Host-side checks of libdwa that need no GPU: exported symbols, argument
validation, and the fifth-dimension matrices the kernels apply (compared with
the oracle's literal D_alpha)."""

import ctypes
import subprocess

import numpy as np
import pytest

from oracle import gamma, redblack, wilson
from paper_1501_04950_amd import dwa, synth

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(dwa.LIB_PATH),
                                reason="libdwa.so not built")


def test_exports_every_declared_symbol():
    declared = dwa.header_functions()
    assert "dwa_apply_Dbb" in declared and "dwa_propagator" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", dwa.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    L = dwa.lib()
    for f in declared:
        assert getattr(L, f) is not None


def _create(**kw):
    base = dict(dims=(4, 4, 4, 4), Ls=8, M5=-1.8, m=0.05, alpha=0.8, b=1.5, c=0.5)
    base.update(kw)
    p = dwa.make_params(**base)
    h = ctypes.c_void_p()
    rc = dwa.lib().dwa_create(ctypes.byref(h), ctypes.byref(p), None)
    if rc == 0:
        dwa.lib().dwa_destroy(h)
    return rc


@pytest.mark.parametrize("kw", [dict(dims=(5, 4, 4, 4)), dict(dims=(4, 4, 3, 4)),
                                dict(dims=(0, 4, 4, 4)), dict(Ls=1), dict(Ls=33),
                                dict(alpha=0.0), dict(alpha=float("nan")), dict(m=float("inf")),
                                # FP64 half field of 16 * 12 * 2^21 * 16 B = 6 GiB > 4 GiB
                                dict(dims=(64, 64, 32, 32), Ls=16)])
def test_create_rejects_bad_arguments(kw):
    assert _create(**kw) == dwa.DWA_EINVAL
    assert dwa.lib().dwa_last_error().decode()


def test_create_rejects_null_coefficients():
    p = dwa.make_params((4, 4, 4, 4), 4, -1.8, 0.1, 1.0, 1.5, 0.5)
    p.b = ctypes.POINTER(ctypes.c_double)()
    h = ctypes.c_void_p()
    assert dwa.lib().dwa_create(ctypes.byref(h), ctypes.byref(p), None) == dwa.DWA_EINVAL
    assert dwa.lib().dwa_create(None, ctypes.byref(p), None) == dwa.DWA_EINVAL


def test_calls_reject_null_context():
    L = dwa.lib()
    assert L.dwa_set_alpha(None, 0.5) == dwa.DWA_EINVAL
    assert L.dwa_alpha_sweep(None, None, 1, None, None, None, None) == dwa.DWA_EINVAL
    assert L.dwa_propagator_adjoint(None, None, None, None, None, None, None, None, None, None,
                                    None, None) == dwa.DWA_EINVAL
    assert L.dwa_reserve_batch(None, 4) == dwa.DWA_EINVAL
    assert L.dwa_propagator_batch(None, 1, None, None, None, None) == dwa.DWA_EINVAL
    assert L.dwa_propagator_multi(None, 0, None, None, None, None, None) == dwa.DWA_EINVAL
    assert L.dwa_cgne_solve_batch(None, 0, 1, None, None, None, None) == dwa.DWA_EINVAL
    assert L.dwa_apply_Dbb(None, 0, None, None) == dwa.DWA_EINVAL
    assert L.dwa_set_links(None, None) == dwa.DWA_EINVAL
    assert L.dwa_propagator(None, None, None, None, None, None) == dwa.DWA_EINVAL
    assert L.dwa_autotune(None, 0, 1, None, 0, None) == dwa.DWA_EINVAL
    assert L.dwa_set_tuning(None, 0, 16, 0, 1, 0) == dwa.DWA_EINVAL
    assert L.dwa_get_tuning(None, 0, None, None, None, None) == dwa.DWA_EINVAL
    assert L.dwa_field_bytes(None, 0, 1) == 0
    assert L.dwa_strerror(dwa.DWA_ENOCONV).decode() == "solver did not converge"


def test_singular_site_block_is_rejected():
    # 4 + M5 = 0 makes I_1 = C, whose determinant is 1 + m per chirality
    assert _create(M5=-4.0, m=-1.0, b=1.0, c=1.0, Ls=4) == dwa.DWA_EINVAL


def test_no_device_is_reported_as_hip_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _create() == dwa.DWA_EHIP


# ------------------------------------------------------------------- s-matrices
def _params(Ls, seed, alpha, m=0.07, M5=-1.8):
    rng = np.random.default_rng(seed)
    return dict(dims=(2, 2, 2, 2), Ls=Ls, M5=M5, m=m, alpha=alpha,
                b=rng.uniform(1.0, 2.0, Ls), c=rng.uniform(0.1, 0.9, Ls))


def _mats(pr):
    return {k: dwa.dwa_debug_smatrix(kind=k, **pr) for k in dwa.MIX_KINDS}


@pytest.mark.parametrize("Ls", [2, 3, 8])
def test_site_block_matches_oracle(Ls):
    """The site-local block I of eq.(redblack) (D_alpha with zero links) equals I_1 G."""
    pr = _params(Ls, Ls, 0.7)
    op = redblack.Params.make(pr["dims"], Ls, pr["M5"], pr["m"], pr["alpha"], pr["b"], pr["c"])
    rb = redblack.RedBlack(synth.unit_field(pr["dims"]), op)
    I4 = rb.I_mat.reshape(Ls, 4, Ls, 4)
    M = _mats(pr)
    for spin in range(4):
        ch = 0 if spin < 2 else 1
        assert np.abs(I4[:, spin, :, spin] - M["I_alpha"][ch]).max() < 1e-14
        for other in range(4):
            if other != spin:
                assert np.abs(I4[:, spin, :, other]).max() == 0.0


@pytest.mark.parametrize("Ls", [2, 5])
def test_hopping_split_matches_oracle(Ls):
    """D_alpha psi = D_w (B G psi) + (I_alpha - (4 + M5) B G) psi slice by slice, with the
    library's B G and I_1 G and the oracle's literal D_alpha and D_w."""
    pr = _params(Ls, 10 + Ls, 0.6)
    dims = (4, 2, 2, 2)
    pr["dims"] = dims
    M = _mats(pr)
    U = synth.su3_field(dims, 0.5, 3)
    psi = synth.gaussian_field5(dims, Ls, 4)
    op = redblack.Params.make(dims, Ls, pr["M5"], pr["m"], pr["alpha"], pr["b"], pr["c"])
    lhs = redblack.RedBlack(U, op).D(psi)

    def smix(mat, f):
        out = np.empty_like(f)
        out[:, :, :2] = np.einsum("ij,jxsc->ixsc", mat[0], f[:, :, :2])
        out[:, :, 2:] = np.einsum("ij,jxsc->ixsc", mat[1], f[:, :, 2:])
        return out

    bg = smix(M["BG"], psi)
    rhs = wilson.dw(U, bg, pr["M5"], dims) + smix(M["I_alpha"], psi) - (4 + pr["M5"]) * bg
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)


@pytest.mark.parametrize("Ls", [2, 3, 7])
@pytest.mark.parametrize("kind", ["identity", "BG", "N", "NT", "Ginv_Iinv", "G_BT_g5", "I_alpha"])
def test_mix_tables_match_oracle(Ls, kind):
    """Every fifth-dimension matrix the kernels apply (per chirality, Ls x Ls) equals the
    oracle's site matrix of the same operator, built from the block list of eq.(mobius1),
    and acts as the identity on spin within each chirality."""
    pr = _params(Ls, 30 + Ls, 0.8)
    op = redblack.Params.make(pr["dims"], Ls, pr["M5"], pr["m"], pr["alpha"], pr["b"], pr["c"])
    O = redblack.RedBlack(synth.unit_field(pr["dims"]), op).mix_matrix(kind).reshape(Ls, 4, Ls, 4)
    M = dwa.dwa_debug_smatrix(kind=kind, **pr)
    for spin in range(4):
        ch = 0 if spin < 2 else 1
        assert np.abs(O[:, spin, :, spin] - M[ch]).max() < 1e-13
        for other in range(4):
            if other != spin:
                assert np.abs(O[:, spin, :, other]).max() == 0.0


@pytest.mark.parametrize("Ls", [2, 6])
def test_matrix_identities(Ls):
    """N = B I_1^-1, G^-1 I_1^-1 = (I_1 G)^-1, the adjoint premixes, from the same B, G, I_1."""
    pr = _params(Ls, 20 + Ls, 1.3)
    M = _mats(pr)
    sgn = [1.0, -1.0]
    for ch in range(2):
        I1inv = M["Iinv"][ch]
        G = I1inv @ M["I_alpha"][ch]
        assert np.allclose(G, np.diag(np.diag(G)), atol=1e-14)
        g = np.diag(G)
        expect_g = np.full(Ls, pr["alpha"])
        if ch == 0:
            expect_g[-1] = 1.0
        else:
            expect_g[0] = 1.0
        assert np.allclose(g, expect_g, atol=1e-13)
        B = M["BG"][ch] @ np.diag(1 / g)
        assert np.allclose(M["N"][ch], B @ I1inv, atol=1e-13)
        assert np.allclose(M["Ginv_Iinv"][ch], np.linalg.inv(M["I_alpha"][ch]), atol=1e-12)
        assert np.allclose(M["NT"][ch], M["N"][ch].T, atol=1e-15)
        assert np.allclose(M["g5_IinvT_Ginv"][ch], sgn[ch] * I1inv.T @ np.diag(1 / g), atol=1e-13)
        assert np.allclose(M["G_BT_g5"][ch], sgn[ch] * np.diag(g) @ B.T, atol=1e-13)
        assert np.allclose(M["identity"][ch], np.eye(Ls))
