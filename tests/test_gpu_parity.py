"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the
same seeded inputs.

FP64 operators must agree with the oracle to 1e-12 relative (they agree to
rounding, ~1e-15).  FP32 and BF16 storage state their error against the FP64
oracle.  Solves are compared through their residuals and the kappa * tol bound.
"""

import sys
import zlib

import numpy as np
import pytest

from oracle import redblack, wilson
from paper_1501_04950_amd import dwa, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    # name: dims, Ls, M5, m, alpha, b, c  (b, c None -> per-slice random)
    "tiny_2x2x2x2_ls4": ((2, 2, 2, 2), 4, -1.8, 0.1, 0.7, None, None),
    "ragged_2x2x2x6_ls2": ((2, 2, 2, 6), 2, -1.7, 0.2, 1.3, None, None),
    "c1_4x4x4x4_ls8": ((4, 4, 4, 4), 8, -1.8, 0.05, 0.8, 1.5, 0.5),
    "ls20_4x2x2x4": ((4, 2, 2, 4), 20, -1.6, 0.03, 0.9, None, None),
    "odd_4x2x2x4_ls5": ((4, 2, 2, 4), 5, -1.8, 0.1, 0.8, None, None),
    # the largest Ls the library takes (generic kernel, register arrays of 32 slices)
    "lsmax32_2x2x2x4_ls32": ((2, 2, 2, 4), 32, -1.8, 0.05, 0.8, None, None),
    "c2_8x8x8x16_ls12": ((8, 8, 8, 16), 12, -1.8, 0.02, 0.6, 1.5, 0.5),
    # L_s = 16 (the bench's) with 24 black sites: every tile size has a partly filled
    # last block
    "ls16_ragged_2x2x2x6": ((2, 2, 2, 6), 16, -1.8, 0.05, 0.8, 1.5, 0.5),
    "ls16_4x4x4x4": ((4, 4, 4, 4), 16, -1.7, 0.03, 1.2, None, None),
    "ls12_ragged_2x2x2x6": ((2, 2, 2, 6), 12, -1.8, 0.05, 0.7, None, None),
    # the other sign of M5 (taken literally in the (4 + M5) of eq.(wilson))
    "posM5_4x2x2x4_ls6": ((4, 2, 2, 4), 6, 1.8, 0.05, 0.9, None, None),
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


# unit roundoff of the storage precision (FP32: 24-bit significand; BF16: 8-bit)
UNIT = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8}
# element-wise bound k of |got - ref| <= k * u * |ref spinor at that (slice, site)|, about
# 4x the largest ratio measured on the parity cases below (FP32 3.2, BF16 1.3, both on the
# full-size 16^3 x 32, L_s = 16 workload)
ELEM_K = {"f32": 13.0, "bf16": 6.0}


def elem_ratio(got, ref, prec):
    """max over elements of |got - ref| / (u |ref spinor at (slice, site)|), over the
    (slice, site) pairs where the reference spinor is non-zero."""
    Ls, V = ref.shape[0], ref.shape[1]
    nrm = np.linalg.norm(ref.reshape(Ls, V, 12), axis=2)
    err = np.abs(got - ref).reshape(Ls, V, 12).max(axis=2)
    live = nrm > 0
    assert np.all(err[~live] == 0.0)
    return float(np.max(err[live] / (UNIT[prec] * nrm[live])))


def check_elementwise(got, ref, prec, what):
    r = elem_ratio(got, ref, prec)
    say(f"    {what}: max element error / (u |ref spinor|) = {r:.2f} (bound {ELEM_K[prec]:.0f})")
    assert r <= ELEM_K[prec], (what, r)


class Case:
    def __init__(self, name):
        dims, Ls, M5, m, alpha, b, c = CASES[name]
        rng = np.random.default_rng(zlib.crc32(name.encode()))
        self.b = np.full(Ls, b) if b is not None else rng.uniform(1.0, 2.0, Ls)
        self.c = np.full(Ls, c) if c is not None else rng.uniform(0.1, 0.9, Ls)
        self.name, self.dims, self.Ls, self.M5, self.m, self.alpha = name, dims, Ls, M5, m, alpha
        self.U = synth.su3_field(dims, 0.5, 7 + Ls)
        self.p = redblack.Params.make(dims, Ls, M5, m, alpha, self.b, self.c)
        self.rb = None

    def oracle(self):
        if self.rb is None:
            self.rb = redblack.RedBlack(self.U, self.p)
        return self.rb

    def ctx(self, alpha=None):
        dev = gpu()
        say(f"[gpu] create context {self.name} alpha={alpha or self.alpha}")
        ctx = dwa.Context(self.dims, self.Ls, self.M5, self.m, alpha or self.alpha, self.b, self.c)
        ctx.set_links(torch.from_numpy(self.U).to(dev))
        return ctx

    def black_field(self, seed):
        f = synth.gaussian_field5(self.dims, self.Ls, seed)
        return f * self.oracle().black


_cases = {}


def case(name):
    if name not in _cases:
        _cases[name] = Case(name)
    return _cases[name]


@pytest.mark.parametrize("prec,tol", [("f64", 0.0), ("f32", 1e-7), ("bf16", 5e-3)])
def test_pack_roundtrip(prec, tol):
    cs = case("ragged_2x2x2x6_ls2")
    ctx = cs.ctx()
    f = synth.gaussian_field5(cs.dims, cs.Ls, 3)
    ft = torch.from_numpy(f).to(gpu())
    say(f"[gpu] pack/unpack {prec}")
    out = torch.zeros_like(ft)
    for par in (0, 1):
        half = ctx.pack(ft, par, prec)
        ctx.unpack(half, par, prec, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if tol == 0.0:
        assert np.array_equal(got, f)
    else:
        assert np.abs(got - f).max() <= tol * np.abs(f).max() * 2
    ctx.close()


@pytest.mark.parametrize("name", ["tiny_2x2x2x2_ls4", "ragged_2x2x2x6_ls2", "c1_4x4x4x4_ls8"])
def test_dw_matches_oracle(name):
    cs = case(name)
    ctx = cs.ctx()
    n = 3
    f = synth.gaussian_source(cs.dims, 5, leading=(n,))
    say(f"[gpu] apply_Dw {name} n={n}")
    out = ctx.apply_Dw(torch.from_numpy(f).to(gpu())).cpu().numpy()
    ref = wilson.dw(cs.U, f, cs.M5, cs.dims)
    assert rel(out, ref) < 1e-13
    ctx.close()


def _gpu_dbb(cs, ctx, x_full, prec="f64", dagger=False):
    xt = torch.from_numpy(np.ascontiguousarray(x_full)).to(gpu())
    half = ctx.pack(xt, 0, prec)
    say(f"[gpu] apply_Dbb{'_dag' if dagger else ''} {cs.name} {prec}")
    out = ctx.apply_Dbb(half, prec, dagger=dagger)
    full = torch.zeros_like(xt)
    ctx.unpack(out, 0, prec, out=full)
    return full.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_dbb_matches_oracle(name):
    cs = case(name)
    ctx = cs.ctx()
    x = cs.black_field(11)
    got = _gpu_dbb(cs, ctx, x)
    ref = cs.oracle().Dbb(x)
    r = rel(got, ref)
    say(f"    D_bb rel err {r:.2e}")
    assert r < 1e-13
    got_d = _gpu_dbb(cs, ctx, x, dagger=True)
    ref_d = cs.oracle().Dbb_dag(x)
    rd = rel(got_d, ref_d)
    say(f"    D_bb^dag rel err {rd:.2e}")
    assert rd < 1e-13
    ctx.close()


def test_full_size_dbb_matches_oracle():
    """The bench workload at its full size (16^3 x 32, L_s = 16, APE-smeared links,
    alpha = 1) in the configuration bench.py times (autotuned tile and block order):
    the FP64, FP32 and BF16 D_bb of one seeded black field against the oracle's, element
    by element (one oracle application, about 35 s of host time), and <y, D_bb x> =
    <D_bb^dag y, x> for the GPU operators (FP64, and FP32 / BF16 to their rounding)."""
    name = "c3_16x16x16x32_ls16"
    w = synth.WORKLOADS[name]
    dev = gpu()
    U = synth.workload_links(name)
    p = redblack.Params.make(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
    say("[gpu] full-size D_bb: oracle set-up")
    rb = redblack.RedBlack(U, p)
    x = synth.gaussian_field5(w["dims"], w["Ls"], 1603) * rb.black
    y = synth.gaussian_field5(w["dims"], w["Ls"], 1604) * rb.black
    ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
    ctx.set_links(torch.from_numpy(U).to(dev))
    for prec in ("f64", "f32", "bf16"):
        ctx.autotune(prec, reps=3)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    yt = torch.from_numpy(np.ascontiguousarray(y)).to(dev)
    xh, yh = ctx.pack(xt, 0, "f64"), ctx.pack(yt, 0, "f64")
    got = torch.zeros_like(xt)
    ctx.unpack(ctx.apply_Dbb(xh, "f64"), 0, "f64", out=got)
    say("[gpu] full-size D_bb: oracle application")
    ref = rb.Dbb(x)
    r = rel(got.cpu().numpy(), ref)
    say(f"    full-size D_bb rel err {r:.2e} (tuning f64 {ctx.get_tuning('f64')})")
    assert r < 1e-13
    # the low-precision operators in the tuned configurations the solves use
    for prec, tol in (("f32", 2e-6), ("bf16", 2e-2)):
        lo = torch.zeros_like(xt)
        ctx.unpack(ctx.apply_Dbb(ctx.pack(xt, 0, prec), prec), 0, prec, out=lo)
        lo = lo.cpu().numpy()
        rl = rel(lo, ref)
        say(f"    full-size {prec} D_bb rel err vs FP64 oracle {rl:.2e} (tuning {ctx.get_tuning(prec)})")
        assert rl < tol
        check_elementwise(lo, ref, prec, f"full-size {prec} D_bb")
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6), ("bf16", 2e-2)):
        xp, yp = ctx.pack(xt, 0, prec), ctx.pack(yt, 0, prec)
        lhs = torch.zeros_like(xt)
        rhs = torch.zeros_like(xt)
        ctx.unpack(ctx.apply_Dbb(xp, prec), 0, prec, out=lhs)
        ctx.unpack(ctx.apply_Dbb(yp, prec, dagger=True), 0, prec, out=rhs)
        a = complex(torch.sum(torch.conj(yt) * lhs))
        b = complex(torch.sum(torch.conj(rhs) * xt))
        d = abs(a - b) / abs(a)
        say(f"    {prec}: |<y, D x> - <D^dag y, x>| / |<y, D x>| = {d:.1e}")
        assert d < tol
    ctx.close()


def test_full_size_propagator_solves_full_system():
    """End to end at full size, as bench.py runs it: the BF16-inner solve (delta 0.3,
    host check every 5, autotuned kernels) of the Z2 source on 16^3 x 32, L_s = 16
    returns a 5D psi that satisfies the oracle's literal D_alpha psi = D_1(1) P eta
    (eq.(mobius1), eq.(tosolve1)) to the accuracy of the 1e-10 Schur solve, and y_1 is
    its wall projection."""
    name = "c3_16x16x16x32_ls16"
    w = synth.WORKLOADS[name]
    dev = gpu()
    U = synth.workload_links(name)
    eta = synth.z2_source(w["dims"], w["seed"] + 100)
    ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
    ctx.set_links(torch.from_numpy(U).to(dev))
    for prec in ("f64", "bf16"):
        ctx.autotune(prec, reps=3)
    say("[gpu] full-size BF16-inner propagator with psi")
    y, st, rc, psi = ctx.propagator(torch.from_numpy(eta).to(dev), want_psi=True, tol=1e-10,
                                    inner_prec="bf16", delta=0.3, check_every=5)
    assert rc == dwa.DWA_OK and st["rel_resid"] <= 1e-10
    psi = psi.cpu().numpy()
    ctx.close()
    p = redblack.Params.make(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
    say("    oracle: D_alpha psi against D_1(1) P eta")
    rho = redblack.source_rhs(U, eta, p)
    res = rel(redblack.RedBlack(U, p).D(psi), rho)
    say(f"    full-system relative residual {res:.2e} (Schur residual {st['rel_resid']:.2e})")
    assert res < 1e-8
    assert rel(y.cpu().numpy(), redblack.extract_y1(psi)) < 1e-15


@pytest.mark.parametrize("prec,bound", [("f32", 2e-6), ("bf16", 2e-2)])
def test_dbb_low_precision_error(prec, bound):
    cs = case("c1_4x4x4x4_ls8")
    ctx = cs.ctx()
    x = cs.black_field(12)
    ref = cs.oracle().Dbb(x)
    got = _gpu_dbb(cs, ctx, x, prec)
    r = rel(got, ref)
    say(f"    D_bb {prec} rel err vs FP64 oracle {r:.2e}")
    assert r < bound
    check_elementwise(got, ref, prec, f"c1 {prec} D_bb")
    got_d = _gpu_dbb(cs, ctx, x, prec, dagger=True)
    check_elementwise(got_d, cs.oracle().Dbb_dag(x), prec, f"c1 {prec} D_bb^dag")
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("name", ["tiny_2x2x2x2_ls4", "c1_4x4x4x4_ls8", "ls12_ragged_2x2x2x6",
                                  "ls16_ragged_2x2x2x6", "ls16_4x4x4x4"])
def test_dbb_tiles_match_oracle(name, prec, tol):
    """D_bb and D_bb^dag in each storage precision with every L_s that has its own
    kernels (4, 8, 12, 16), against the FP64 oracle for every tile size and block order,
    and bitwise the same result from each of them.  The small lattices leave every tile
    size with a partly filled last block."""
    cs = case(name)
    ctx = cs.ctx()
    x = cs.black_field(21)
    ref = cs.oracle().Dbb(x)
    ref_d = cs.oracle().Dbb_dag(x)
    first = None
    for ns in (8, 16, 32):
        for order in ("slab", "lex"):
            ctx.set_tuning(prec, ns, order)
            got = _gpu_dbb(cs, ctx, x, prec)
            got_d = _gpu_dbb(cs, ctx, x, prec, dagger=True)
            r, rd = rel(got, ref), rel(got_d, ref_d)
            say(f"    ns={ns} {order}: {prec} D_bb rel err {r:.2e}, dagger {rd:.2e}")
            assert r < tol and rd < tol
            if prec != "f64" and first is None:
                check_elementwise(got, ref, prec, f"{name} {prec} D_bb")
                check_elementwise(got_d, ref_d, prec, f"{name} {prec} D_bb^dag")
            if first is None:
                first = (got, got_d)
            else:
                assert np.array_equal(got, first[0]) and np.array_equal(got_d, first[1])
    ctx.close()


def test_cgne_matches_oracle_cgls():
    """Same CGLS, same stopping rule: iteration counts agree within one and the
    solutions agree to the accuracy both residuals allow."""
    cs = case("c1_4x4x4x4_ls8")
    rb = cs.oracle()
    rhs = cs.black_field(13)
    x_ref, info = redblack.cgls(rb.Dbb, rb.Dbb_dag, rhs, 1e-10, 2000)
    ctx = cs.ctx()
    say("[gpu] cgne_solve c1 f64")
    half = ctx.pack(torch.from_numpy(rhs).to(gpu()), 0, "f64")
    x, st, rc = ctx.cgne_solve(half, tol=1e-10, maxiter=2000, check_every=1)
    assert rc == dwa.DWA_OK and st["converged"]
    full = torch.zeros((cs.Ls,) + rhs.shape[1:], dtype=torch.complex128, device=gpu())
    ctx.unpack(x, 0, "f64", out=full)
    xg = full.cpu().numpy()
    say(f"    iters gpu {st['iters']} oracle {info.iters}; true resid gpu {st['rel_resid']:.2e}; "
        f"x diff {rel(xg, x_ref):.2e}")
    assert abs(st["iters"] - info.iters) <= 1
    assert st["rel_resid"] <= 1.5e-10
    assert rel(rb.Dbb(xg), rhs) <= 1.5e-10
    assert rel(xg, x_ref) < 1e-8
    ctx.close()


@pytest.mark.parametrize("name", ["c1_4x4x4x4_ls8", "posM5_4x2x2x4_ls6"])
def test_propagator_matches_oracle(name):
    """y_1 for a point source (site 0, spin 0, colour 0) on the 4^4, Ls=8 lattice, and
    with M5 = +1.8 on 4x2x2x4, Ls = 6."""
    cs = case(name)
    eta = synth.point_source(cs.dims, 0, 0, 0)
    y_ref, info = redblack.propagator(cs.U, eta, cs.p, tol=1e-12)
    ctx = cs.ctx()
    say(f"[gpu] propagator {name} f64 tol 1e-12")
    y, st, rc = ctx.propagator(torch.from_numpy(eta).to(gpu()), tol=1e-12, check_every=1)
    yg = y.cpu().numpy()
    r = rel(yg, y_ref)
    say(f"    y1 rel diff {r:.2e} iters gpu {st['iters']} oracle {info.iters}")
    assert rc == dwa.DWA_OK
    assert abs(st["iters"] - info.iters) <= 1
    assert r < 1e-12
    ctx.close()


def test_propagator_psi_solves_full_system():
    """The returned 5D psi satisfies D_alpha psi = D_1(1) P b (oracle's literal operators)."""
    cs = case("tiny_2x2x2x2_ls4")
    eta = synth.gaussian_source(cs.dims, 21)
    ctx = cs.ctx()
    say("[gpu] propagator tiny with psi")
    y, st, rc, psi = ctx.propagator(torch.from_numpy(eta).to(gpu()), want_psi=True, tol=1e-13)
    psi = psi.cpu().numpy()
    rho = redblack.source_rhs(cs.U, eta, cs.p)
    assert rel(cs.oracle().D(psi), rho) < 1e-11
    assert rel(y.cpu().numpy(), redblack.extract_y1(psi)) < 1e-15
    ctx.close()


def test_y1_alpha_independent_on_gpu():
    cs = case("c1_4x4x4x4_ls8")
    eta = torch.from_numpy(synth.gaussian_source(cs.dims, 22)).to(gpu())
    ys = []
    for alpha in (0.6, 1.0, 1.3):
        ctx = cs.ctx(alpha)
        say(f"[gpu] propagator alpha={alpha}")
        y, st, rc = ctx.propagator(eta, tol=1e-12, check_every=10)
        assert rc == dwa.DWA_OK
        ys.append(y.cpu().numpy())
        ctx.close()
    assert rel(ys[0], ys[1]) < 1e-9 and rel(ys[2], ys[1]) < 1e-9


def test_alpha_sweep_matches_oracle():
    """The alpha study on one context (dwa_set_alpha between solves): each alpha's
    iteration count is the oracle CGLS count at that alpha (within one), every y_1
    is the oracle's alpha = 1 propagator, and the context's alpha is restored."""
    cs = case("c1_4x4x4x4_ls8")
    eta = synth.point_source(cs.dims, 0, 1, 0)
    alphas = [0.5, 0.8, 1.0, 1.2]
    ref_iters = []
    y_ref = None
    for a in alphas:
        y_a, info = redblack.propagator(cs.U, eta, cs.p.with_(alpha=a), tol=1e-10)
        ref_iters.append(info.iters)
        if a == 1.0:
            y_ref = y_a
    ctx = cs.ctx()
    say(f"[gpu] alpha sweep c1 {alphas}")
    y, stats, rc = ctx.alpha_sweep(torch.from_numpy(eta).to(gpu()), alphas, tol=1e-10, check_every=1)
    assert rc == dwa.DWA_OK
    iters = [st["iters"] for st in stats]
    say(f"    iters gpu {iters} oracle {ref_iters}")
    for a, i, r, st, yy in zip(alphas, iters, ref_iters, stats, y.cpu().numpy()):
        assert abs(i - r) <= 1, (a, i, r)
        assert st["rel_resid"] <= 1.5e-10
        assert rel(yy, y_ref) < 1e-8
    # restored: a plain solve reproduces the context's own alpha count
    _, st0, _ = ctx.propagator(torch.from_numpy(eta).to(gpu()), tol=1e-10, check_every=1)
    assert abs(st0["iters"] - ref_iters[alphas.index(cs.alpha)]) <= 1
    with pytest.raises(dwa.DwaError) as e:
        ctx.set_alpha(0.0)
    assert e.value.status == dwa.DWA_EINVAL
    ctx.close()


def test_alpha_sweep_8x8x8x16_fp64_and_f32():
    """The alpha study on 8^3 x 16, Ls = 12 (spread 0.5, m = 0.02) for the 12 spin-colour
    point sources at site 0, FP64 and FP32-inner with FP64 reliable updates, both to a
    1e-10 residual.  Properties that hold at any size: every solve converges, y_1 is the
    same for every alpha and both precisions (within kappa * tol), and the FP32 path
    needs about as many iterations as FP64.  The iteration counts are printed (the
    paper's MILC fields are not here, so their values are not pinned)."""
    name = "c2_8x8x8x16_ls12"
    w = synth.WORKLOADS[name]
    dev = gpu()
    ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
    ctx.set_links(torch.from_numpy(synth.workload_links(name)).to(dev))
    alphas = list(w["alphas"])
    n = {"f64": np.zeros((12, len(alphas)), int), "f32": np.zeros((12, len(alphas)), int)}
    for src in range(12):
        eta = torch.from_numpy(synth.point_source(w["dims"], 0, src // 3, src % 3)).to(dev)
        say(f"[gpu] c2 alpha sweep source {src}")
        y64, st64, rc64 = ctx.alpha_sweep(eta, alphas, tol=1e-10, check_every=10)
        y32, st32, rc32 = ctx.alpha_sweep(eta, alphas, tol=1e-10, inner_prec="f32", delta=0.05,
                                          check_every=10)
        assert rc64 == dwa.DWA_OK and rc32 == dwa.DWA_OK
        ref = y64[alphas.index(1.0)]
        for k in range(len(alphas)):
            assert st64[k]["rel_resid"] <= 1e-10 and st32[k]["rel_resid"] <= 1e-10
            for y in (y64[k], y32[k]):
                d = float(torch.linalg.vector_norm(y - ref) / torch.linalg.vector_norm(ref))
                assert d < 1e-7, (src, alphas[k], d)
            n["f64"][src, k] = st64[k]["iters"]
            n["f32"][src, k] = st32[k]["iters"]
    for prec in ("f64", "f32"):
        rel_n = n[prec] / n[prec][:, [alphas.index(1.0)]]
        say(f"    {prec}: mean n(alpha)/n(1) " +
            ", ".join(f"{a}: {m:.3f}+-{sd:.3f}" for a, m, sd in zip(alphas, rel_n.mean(0), rel_n.std(0))))
    assert np.all(n["f32"] <= 1.3 * n["f64"] + 20)
    ctx.close()


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_mixed_precision_reaches_fp64_accuracy(inner):
    cs = case("c1_4x4x4x4_ls8")
    eta = torch.from_numpy(synth.point_source(cs.dims, 0, 1, 2)).to(gpu())
    ctx = cs.ctx()
    say(f"[gpu] propagator f64 reference")
    y64, st64, rc = ctx.propagator(eta, tol=1e-10, check_every=5)
    say(f"[gpu] propagator mixed {inner}")
    y, st, rc = ctx.propagator(eta, tol=1e-10, inner_prec=inner, delta=0.1 if inner == "f32" else 0.3,
                               check_every=5)
    say(f"    {inner}: iters {st['iters']} outer {st['outer']} resid {st['rel_resid']:.2e}; "
        f"f64 iters {st64['iters']}")
    assert rc == dwa.DWA_OK and st["rel_resid"] <= 1e-10
    assert rel(y.cpu().numpy(), y64.cpu().numpy()) < 1e-8
    ctx.close()


@pytest.mark.parametrize("inner,mode,delta", [("bf16", "reliable", 0.3), ("f32", "reliable", 0.05),
                                              ("bf16", "defect", 0.3)])
def test_mixed_precision_bench_workload(inner, mode, delta):
    """At the 16^3 x 32, Ls = 16 workload the mixed solves reach the FP64 solve's
    accuracy: true FP64 residual <= 1e-10 and y_1 within kappa * tol of the FP64 y_1.
    The FP64 D_bb that measures the residual is the one checked against the oracle
    element by element on the smaller lattices."""
    dev = gpu()
    w = synth.WORKLOADS["c3_16x16x16x32_ls16"]
    say(f"[gpu] bench workload, mixed {inner} {mode} delta={delta}")
    ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
    ctx.set_links(torch.from_numpy(synth.workload_links("c3_16x16x16x32_ls16")).to(dev))
    eta = torch.from_numpy(synth.z2_source(w["dims"], w["seed"] + 100)).to(dev)
    y64, st64, rc64 = ctx.propagator(eta, tol=1e-10, check_every=10)
    y, st, rc = ctx.propagator(eta, tol=1e-10, inner_prec=inner, delta=delta, check_every=10,
                               mixed_mode=mode)
    say(f"    {inner}/{mode}: iters {st['iters']} outer {st['outer']} resid {st['rel_resid']:.2e}; "
        f"f64 iters {st64['iters']}")
    assert rc64 == dwa.DWA_OK and rc == dwa.DWA_OK
    assert st["rel_resid"] <= 1e-10
    # both solutions within ~kappa * 1e-10 of the exact one
    d = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))
    say(f"    |y - y64| / |y64| = {d:.2e}")
    assert d < 1e-7
    ctx.close()


@pytest.mark.parametrize("inner,check_every", [("f64", 1), ("f64", 4), ("bf16", 5), ("f32", 3)])
def test_solver_graph_replay_equals_eager(inner, check_every, monkeypatch):
    """The single-field solvers replay one CG iteration from a hipGraph between host
    checks (with the reliable updates and checks run eagerly in between); with
    DWA_SOLVE_NO_GRAPH the same launches are issued one by one.  Every replay must give
    what the eager launches give: y_1, the iteration count and the final residual are
    bitwise the same, for the propagator and for its adjoint solve (gradients)."""
    cs = case("c1_4x4x4x4_ls8")
    ctx = cs.ctx()
    eta = torch.from_numpy(synth.point_source(cs.dims, 0, 2, 2)).to(gpu())
    etp = torch.from_numpy(synth.gaussian_source(cs.dims, 77)).to(gpu())
    kw = dict(tol=1e-10, inner_prec=inner, check_every=check_every)
    if inner != "f64":
        kw["delta"] = 0.3 if inner == "bf16" else 0.05
    res = {}
    for mode in ("graph", "eager"):
        if mode == "eager":
            monkeypatch.setenv("DWA_SOLVE_NO_GRAPH", "1")
        say(f"[gpu] solver {mode} {inner} check_every={check_every}")
        y, st, rc = ctx.propagator(eta, **kw)
        g = ctx.propagator_adjoint(eta, etp, want=("U",), **kw)
        assert rc == dwa.DWA_OK and g["status"] == dwa.DWA_OK
        res[mode] = (y.cpu().numpy(), st, g["U"].cpu().numpy(), g["stats"])
    (yg, sg, ug, gg), (ye, se, ue, ge) = res["graph"], res["eager"]
    say(f"    iters {sg['iters']} / {se['iters']}, adjoint {gg[1]['iters']} / {ge[1]['iters']}")
    assert np.array_equal(yg, ye) and np.array_equal(ug, ue)
    assert sg["iters"] == se["iters"] and sg["rel_resid"] == se["rel_resid"]
    assert gg[1]["iters"] == ge[1]["iters"] and gg[1]["rel_resid"] == ge[1]["rel_resid"]
    ctx.close()


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_zero_source_gives_zero(inner):
    """eta = 0: the solve stops at once with y_1 = 0 and status ok (degenerate case)."""
    cs = case("c1_4x4x4x4_ls8")
    ctx = cs.ctx()
    eta = torch.zeros((int(np.prod(cs.dims)), 4, 3), dtype=torch.complex128, device=gpu())
    y, st, rc = ctx.propagator(eta, tol=1e-10, inner_prec=inner)
    assert rc == dwa.DWA_OK and st["converged"] and st["iters"] == 0
    assert float(torch.max(torch.abs(y))) == 0.0
    ctx.close()


def test_error_paths():
    cs = case("tiny_2x2x2x2_ls4")
    dev = gpu()
    ctx = dwa.Context(cs.dims, cs.Ls, cs.M5, cs.m, cs.alpha, cs.b, cs.c)
    say("[gpu] error paths")
    half = ctx.half_field("f64")
    with pytest.raises(dwa.DwaError) as e:
        ctx.apply_Dbb(half)
    assert e.value.status == dwa.DWA_ESTATE
    ctx.set_links(torch.from_numpy(cs.U).to(dev))
    eta = synth.gaussian_source(cs.dims, 3)
    eta[5, 1, 2] = np.nan
    with pytest.raises(dwa.DwaError) as e:
        ctx.propagator(torch.from_numpy(eta).to(dev))
    assert e.value.status == dwa.DWA_ENAN
    eta = torch.from_numpy(synth.gaussian_source(cs.dims, 4)).to(dev)
    y, st, rc = ctx.propagator(eta, tol=1e-14, maxiter=2)
    assert rc == dwa.DWA_ENOCONV and st["iters"] == 2 and not st["converged"]
    with pytest.raises(dwa.DwaError) as e:
        ctx.propagator(eta, inner_prec="bf16", mixed_mode=7)
    assert e.value.status == dwa.DWA_EINVAL
    ctx.close()


@pytest.mark.parametrize("name", ["ragged_2x2x2x6_ls2", "c1_4x4x4x4_ls8", "ls20_4x2x2x4"])
@pytest.mark.parametrize("kind", ["identity", "N", "NT", "Ginv_Iinv", "G_BT_g5"])
def test_single_hop_launch(name, kind):
    """dwa_apply_hop: out = M_kind H_rb x_b with H the hopping sum of eq.(wilson) without
    its -1/2 (on red sites D_w x_b = -1/2 H_rb x_b for a black-only x_b), and M_kind built
    from the oracle's own site matrices of eq.(mobius1)."""
    cs = case(name)
    ctx = cs.ctx()
    x = cs.black_field(31)
    h = -2.0 * wilson.dw(cs.U, x, cs.M5, cs.dims) * cs.oracle().red
    ref = cs.oracle().site_apply(cs.oracle().mix_matrix(kind), h)
    xt = torch.from_numpy(x).to(gpu())
    say(f"[gpu] apply_hop {name} {kind}")
    out = ctx.apply_hop(ctx.pack(xt, 0, "f64"), 1, kind, "f64")
    full = torch.zeros_like(xt)
    ctx.unpack(out, 1, "f64", out=full)
    assert rel(full.cpu().numpy(), ref) < 1e-13
    ctx.close()
