"""GPU gradients of L = Re <eta', y_1> (dwa_propagator_adjoint) against the oracle's
adjoint-state gradients (small lattices) and against central finite differences of
GPU solves on the 8^4, Ls = 8 workload."""

import sys

import numpy as np
import pytest

from oracle import adjoint, redblack
from oracle.gamma import GAMMA5, spin_apply
from paper_1501_04950_amd import dwa, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("dims,Ls", [((2, 2, 2, 4), 4), ((4, 2, 2, 4), 5)])
def test_gradients_match_oracle(dims, Ls):
    """Every gradient against the oracle (unpreconditioned adjoint solve, literal block
    terms) with per-slice b_i, c_i without symmetry; both solves at 1e-13."""
    dev = gpu()
    rng = np.random.default_rng(21 + Ls)
    b, c = rng.uniform(1.0, 2.0, Ls), rng.uniform(0.1, 0.9, Ls)
    U = synth.su3_field(dims, 0.5, 31 + Ls)
    p = redblack.Params.make(dims, Ls, -1.8, 0.1, 0.8, b, c)
    eta = synth.gaussian_source(dims, 41)
    eta_p = synth.gaussian_source(dims, 42)
    ref = adjoint.gradients(U, eta, eta_p, p, tol=1e-13)
    L_ref = adjoint.loss(U, eta, eta_p, p)
    say(f"[gpu] gradients {dims} Ls={Ls}")
    ctx = dwa.Context(dims, Ls, -1.8, 0.1, 0.8, b, c)
    ctx.set_links(torch.from_numpy(U).to(dev))
    g = ctx.propagator_adjoint(torch.from_numpy(eta).to(dev), torch.from_numpy(eta_p).to(dev),
                               tol=1e-13, check_every=1)
    say(f"    L gpu {g['L']:.15e} oracle {L_ref:.15e}; iters fwd {g['stats'][0]['iters']} "
        f"adj {g['stats'][1]['iters']} adj resid {g['stats'][1]['rel_resid']:.1e}")
    assert g["status"] == dwa.DWA_OK
    assert g["stats"][1]["rel_resid"] <= 1e-12
    assert abs(g["L"] - L_ref) <= 1e-11 * abs(L_ref)
    errs = {"U": rel(g["U"].cpu().numpy(), ref["U"]), "eta": rel(g["eta"].cpu().numpy(), ref["eta"]),
            "b": rel(g["b"], ref["b"]), "c": rel(g["c"], ref["c"])}
    say(f"    rel errors {errs}; alpha gpu {g['alpha']:.2e} oracle {ref['alpha']:.2e}")
    for k, e in errs.items():
        assert e < 1e-9, (k, e)
    assert abs(g["alpha"]) <= 1e-9 * abs(L_ref)
    ctx.close()


@pytest.fixture(scope="module")
def c5():
    name = "c5_8x8x8x8_ls8"
    w = synth.WORKLOADS[name]
    dev = gpu()
    U = synth.workload_links(name)
    eta = synth.gaussian_source(w["dims"], 51)
    eta_p = synth.gaussian_source(w["dims"], 52)
    alpha = w["alphas"][0]
    ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], alpha, w["b"], w["c"])
    Ud = torch.from_numpy(U).to(dev)
    ctx.set_links(Ud)
    e, ep = torch.from_numpy(eta).to(dev), torch.from_numpy(eta_p).to(dev)
    say("[gpu] c5 adjoint gradients")
    g = ctx.propagator_adjoint(e, ep, tol=1e-13, check_every=5)
    assert g["status"] == dwa.DWA_OK
    yield dict(w=w, U=U, Ud=Ud, eta=e, eta_p=ep, ctx=ctx, g=g, alpha=alpha)
    ctx.close()


def _loss(ctx, eta, eta_p):
    y, st, rc = ctx.propagator(eta, tol=1e-13, check_every=5)
    assert rc == dwa.DWA_OK
    return float(torch.sum(torch.conj(eta_p) * y).real)


def _close(fd, adj, L):
    assert abs(fd - adj) <= 1e-6 * max(abs(adj), abs(L)), (fd, adj)


def test_c5_link_gradient_finite_differences(c5):
    """16 random complex link directions, central differences with step 1e-6."""
    ctx, g, Ud = c5["ctx"], c5["g"], c5["Ud"]
    gen = torch.Generator(device="cpu").manual_seed(61)
    L = g["L"]
    for k in range(16):
        d = torch.complex(torch.randn(Ud.shape, generator=gen, dtype=torch.float64),
                          torch.randn(Ud.shape, generator=gen, dtype=torch.float64)).to(Ud.device)
        vals = []
        for sgn in (1.0, -1.0):
            ctx.set_links((Ud + sgn * 1e-6 * d).contiguous())
            vals.append(_loss(ctx, c5["eta"], c5["eta_p"]))
        fd = (vals[0] - vals[1]) / 2e-6
        adj = float(torch.sum(torch.conj(g["U"]) * d).real)
        say(f"    link dir {k}: fd {fd:.9e} adjoint {adj:.9e}")
        _close(fd, adj, L)
    ctx.set_links(Ud)


def test_c5_coefficient_and_alpha_gradients_finite_differences(c5):
    """8 directions in (b, c) and 8 in (alpha, b): new contexts for b and c, set_alpha
    for alpha.  dL/dalpha itself is zero (y_1 does not depend on alpha)."""
    w, g = c5["w"], c5["g"]
    Ls = w["Ls"]
    rng = np.random.default_rng(71)
    b0, c0 = np.full(Ls, w["b"]), np.full(Ls, w["c"])
    L = g["L"]

    def loss_at(b, c, alpha):
        ctx = dwa.Context(w["dims"], Ls, w["M5"], w["m"], alpha, b, c)
        ctx.set_links(c5["Ud"])
        v = _loss(ctx, c5["eta"], c5["eta_p"])
        ctx.close()
        return v

    for k in range(8):
        db, dc = rng.normal(size=Ls), rng.normal(size=Ls)
        fd = (loss_at(b0 + 1e-6 * db, c0 + 1e-6 * dc, c5["alpha"])
              - loss_at(b0 - 1e-6 * db, c0 - 1e-6 * dc, c5["alpha"])) / 2e-6
        adj = float(g["b"] @ db + g["c"] @ dc)
        say(f"    (b, c) dir {k}: fd {fd:.9e} adjoint {adj:.9e}")
        _close(fd, adj, L)
    for k in range(8):
        da, db = rng.normal(), rng.normal(size=Ls)
        fd = (loss_at(b0 + 1e-6 * db, c0, c5["alpha"] + 1e-6 * da)
              - loss_at(b0 - 1e-6 * db, c0, c5["alpha"] - 1e-6 * da)) / 2e-6
        adj = float(g["alpha"] * da + g["b"] @ db)
        say(f"    (alpha, b) dir {k}: fd {fd:.9e} adjoint {adj:.9e}")
        _close(fd, adj, L)
    assert abs(g["alpha"]) <= 1e-8 * abs(L)


def test_c5_source_gradient(c5):
    """dL/deta against finite differences and against g5 y_1[g5 eta'] (b, c constant,
    so the 4D operator is g5-Hermitian)."""
    ctx, g = c5["ctx"], c5["g"]
    gen = torch.Generator(device="cpu").manual_seed(81)
    eta = c5["eta"]
    for k in range(4):
        d = torch.complex(torch.randn(eta.shape, generator=gen, dtype=torch.float64),
                          torch.randn(eta.shape, generator=gen, dtype=torch.float64)).to(eta.device)
        fd = (_loss(ctx, (eta + 1e-6 * d).contiguous(), c5["eta_p"])
              - _loss(ctx, (eta - 1e-6 * d).contiguous(), c5["eta_p"])) / 2e-6
        adj = float(torch.sum(torch.conj(g["eta"]) * d).real)
        _close(fd, adj, g["L"])
    g5 = torch.from_numpy(np.diag(GAMMA5).real.copy()).to(eta.device)[None, :, None]
    y5, _, rc = ctx.propagator((g5 * c5["eta_p"]).contiguous(), tol=1e-13, check_every=5)
    r = float(torch.linalg.vector_norm(g["eta"] - g5 * y5) / torch.linalg.vector_norm(g["eta"]))
    say(f"    g5 identity rel diff {r:.2e}")
    assert r < 1e-9


def test_autograd_function(c5):
    """The differentiable propagator: for L = Re <eta', y_1> its backward gives the
    library's adjoint gradients; for the nonlinear L2 = |y_1|^2 a link direction agrees
    with central differences."""
    from paper_1501_04950_amd import autograd as dag
    w, ctx, g = c5["w"], c5["ctx"], c5["g"]
    dev = c5["Ud"].device
    U = c5["Ud"].clone().requires_grad_(True)
    eta = c5["eta"].clone().requires_grad_(True)
    alpha = torch.tensor(c5["alpha"], dtype=torch.float64, device=dev, requires_grad=True)
    b = torch.full((w["Ls"],), w["b"], dtype=torch.float64, device=dev, requires_grad=True)
    c = torch.full((w["Ls"],), w["c"], dtype=torch.float64, device=dev, requires_grad=True)
    y = dag.propagator(ctx, U, eta, alpha, b, c, tol=1e-13, check_every=5)
    L = torch.sum(torch.conj(c5["eta_p"]) * y).real
    L.backward()
    assert rel(U.grad.cpu().numpy(), g["U"].cpu().numpy()) < 1e-10
    assert rel(eta.grad.cpu().numpy(), g["eta"].cpu().numpy()) < 1e-10
    assert rel(b.grad.cpu().numpy(), g["b"]) < 1e-10 and rel(c.grad.cpu().numpy(), g["c"]) < 1e-10
    assert abs(float(alpha.grad)) <= 1e-8 * abs(float(L))

    U2 = c5["Ud"].clone().requires_grad_(True)
    y2 = dag.propagator(ctx, U2, c5["eta"], tol=1e-13, check_every=5)
    L2 = torch.sum(torch.abs(y2) ** 2)
    L2.backward()
    gen = torch.Generator(device="cpu").manual_seed(91)
    d = torch.complex(torch.randn(U2.shape, generator=gen, dtype=torch.float64),
                      torch.randn(U2.shape, generator=gen, dtype=torch.float64)).to(dev)
    vals = []
    for sgn in (1.0, -1.0):
        ctx.set_links((c5["Ud"] + sgn * 1e-6 * d).contiguous())
        yy, _, _ = ctx.propagator(c5["eta"], tol=1e-13, check_every=5)
        vals.append(float(torch.sum(torch.abs(yy) ** 2)))
    ctx.set_links(c5["Ud"])
    fd = (vals[0] - vals[1]) / 2e-6
    adj = float(torch.sum(torch.conj(U2.grad) * d).real)
    say(f"    |y|^2 link dir: fd {fd:.9e} autograd {adj:.9e}")
    _close(fd, adj, float(L2))


def test_autograd_lazy_conjugate_gradient(c5):
    """L = Re sum(conj(y_1) * eta') is the same loss as Re <eta', y_1>, but autograd hands
    the backward a lazily conjugated gradient of y_1 (the value lives in memory
    conjugated, with a flag on the tensor).  The backward must resolve it: its gradients
    equal the library's adjoint gradients of Re <eta', y_1>.  The forward inputs may be
    such views as well (eta passed as conj(conj(eta)))."""
    from paper_1501_04950_amd import autograd as dag
    ctx, g = c5["ctx"], c5["g"]
    U = c5["Ud"].clone().requires_grad_(True)
    eta = c5["eta"].clone().requires_grad_(True)
    y = dag.propagator(ctx, U, eta.conj().conj(), tol=1e-13, check_every=5)
    L = torch.sum(torch.conj(y) * c5["eta_p"]).real
    L.backward()
    say(f"    L {float(L):.12e} library {g['L']:.12e}")
    assert abs(float(L) - g["L"]) <= 1e-10 * abs(g["L"])
    assert rel(U.grad.cpu().numpy(), g["U"].cpu().numpy()) < 1e-10
    assert rel(eta.grad.cpu().numpy(), g["eta"].cpu().numpy()) < 1e-10
    with pytest.raises(ValueError):
        ctx.propagator(c5["eta"].conj(), tol=1e-6)


@pytest.mark.parametrize("inner,delta", [("f32", 0.05), ("bf16", 0.3)])
def test_c5_mixed_precision_gradients(c5, inner, delta):
    """Both solves in FP32 or BF16 storage with FP64 reliable updates (tol 1e-10): the
    adjoint solve's FP64 residual meets the tolerance and every gradient agrees with
    the FP64 solves' (tol 1e-13) to the accuracy that tolerance allows."""
    ctx, ref = c5["ctx"], c5["g"]
    say(f"[gpu] c5 adjoint gradients, {inner} inner")
    g = ctx.propagator_adjoint(c5["eta"], c5["eta_p"], tol=1e-10, inner_prec=inner, delta=delta,
                               check_every=5)
    st = g["stats"]
    say(f"    iters fwd {st[0]['iters']} adj {st[1]['iters']} (FP64 {ref['stats'][1]['iters']}); "
        f"adj resid {st[1]['rel_resid']:.1e}")
    assert g["status"] == dwa.DWA_OK
    assert st[1]["rel_resid"] <= 1e-10
    assert abs(g["L"] - ref["L"]) <= 1e-8 * abs(ref["L"])
    errs = {"U": rel(g["U"].cpu().numpy(), ref["U"].cpu().numpy()),
            "eta": rel(g["eta"].cpu().numpy(), ref["eta"].cpu().numpy()),
            "b": rel(g["b"], ref["b"]), "c": rel(g["c"], ref["c"])}
    say(f"    rel errors vs FP64 solves {errs}")
    for k, e in errs.items():
        assert e < 1e-7, (k, e)
