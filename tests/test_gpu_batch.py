"""Batched solves (dwa_propagator_batch / dwa_propagator_multi): many sources, and
several lattices, in one solve whose CGNE iteration is replayed from a hipGraph."""

import sys

import numpy as np
import pytest

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


def spin_colour_sources(dims, site=0):
    """The 12 point sources at one site, [12, V, 4, 3]."""
    return np.stack([synth.point_source(dims, site, k // 3, k % 3) for k in range(12)])


def rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def _ctx(name, alpha=None):
    w = synth.WORKLOADS[name]
    ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], alpha if alpha is not None else 1.0,
                      w["b"], w["c"])
    ctx.set_links(torch.from_numpy(synth.workload_links(name)).to(gpu()))
    return ctx, w


def test_batch_fp64_equals_single_solves():
    """Each field of a batch follows the single-source CGLS exactly: same iteration
    count (host check every iteration) and the same y_1 (same reduction order)."""
    ctx, w = _ctx("c1_4x4x4x4_ls8", 0.8)
    eta = torch.from_numpy(spin_colour_sources(w["dims"])).to(gpu())
    ctx.reserve_batch(12)
    say("[gpu] batch of 12 on 4^4 Ls=8, FP64")
    y, stats, rc = ctx.propagator_batch(eta, tol=1e-12, check_every=1)
    assert rc == dwa.DWA_OK
    for k in range(12):
        ys, st, rc1 = ctx.propagator(eta[k].contiguous(), tol=1e-12, check_every=1)
        assert rc1 == dwa.DWA_OK
        d = rel(y[k], ys)
        assert stats[k]["iters"] == st["iters"], (k, stats[k]["iters"], st["iters"])
        assert stats[k]["rel_resid"] <= 1e-12
        assert d < 1e-13, (k, d)
    # a second call on the same reservation reproduces the first (graph rebuilt per call)
    y2, stats2, rc2 = ctx.propagator_batch(eta, tol=1e-12, check_every=1)
    assert rc2 == dwa.DWA_OK and float(torch.max(torch.abs(y2 - y))) == 0.0
    ctx.close()


@pytest.mark.parametrize("inner,mode,delta", [("f32", "reliable", 0.05), ("bf16", "reliable", 0.3),
                                              ("f32", "defect", 0.1), ("bf16", "defect", 0.1)])
def test_batch_mixed_precision(inner, mode, delta):
    """12 sources on 8^3 x 16, Ls = 12 with low-precision inner CGNE and FP64 reliable
    updates or defect correction: every field reaches 1e-10 and matches the FP64 batch.
    With reliable updates the iteration counts stay within 10% (+10) of single-source
    solves with the same options."""
    ctx, w = _ctx("c2_8x8x8x16_ls12", 0.8)
    eta = torch.from_numpy(spin_colour_sources(w["dims"])).to(gpu())
    ctx.reserve_batch(12)
    say(f"[gpu] batch of 12 on 8^3x16 Ls=12, inner {inner}, {mode}")
    kw = dict(tol=1e-10, inner_prec=inner, delta=delta, check_every=10, mixed_mode=mode)
    y64, st64, rc64 = ctx.propagator_batch(eta, tol=1e-10, check_every=10)
    y, st, rc = ctx.propagator_batch(eta, **kw)
    assert rc64 == dwa.DWA_OK and rc == dwa.DWA_OK
    say("    iters fp64 " + str([s["iters"] for s in st64]) + f" {inner} " + str([s["iters"] for s in st])
        + " outer " + str([s["outer"] for s in st]))
    for k in range(12):
        assert st[k]["rel_resid"] <= 1e-10 and st64[k]["rel_resid"] <= 1e-10
        assert rel(y[k], y64[k]) < 1e-7
    if mode == "reliable":
        for k in (0, 5, 11):
            ys, s1, rc1 = ctx.propagator(eta[k].contiguous(), **kw)
            assert rc1 == dwa.DWA_OK
            say(f"    field {k}: batch {st[k]['iters']} single {s1['iters']} iterations")
            assert st[k]["iters"] <= 1.1 * s1["iters"] + 10
            assert rel(y[k], ys) < 1e-7
    ctx.close()


def test_multi_lattice_batch():
    """Three lattices (8^4 / Ls 8, 12^3 x 24 / Ls 12, 16^3 x 32 / Ls 16; spread 0.6,
    alpha 0.8, m 0.02) with 12 point sources each in one solve, FP32 inner and FP64
    outer to 1e-10.  Every field converges, and one source per lattice matches a
    single-source FP64 solve of its own context."""
    bw = synth.BATCH_WORKLOAD
    dev = gpu()
    batches, singles = [], []
    for k, lat in enumerate(bw["lattices"]):
        dims, Ls = lat["dims"], lat["Ls"]
        U = torch.from_numpy(synth.su3_field(dims, bw["spread"], bw["seed"] + k)).to(dev)
        ctx = dwa.Context(dims, Ls, bw["M5"], bw["m"], bw["alpha"], bw["b"], bw["c"])
        ctx.set_links(U)
        ctx.reserve_batch(12)
        eta = torch.from_numpy(spin_colour_sources(dims)).to(dev)
        batches.append((ctx, eta))
    say("[gpu] multi-lattice batch: 3 lattices x 12 sources, FP32 inner")
    ys, stats, rc = dwa.propagator_multi(batches, tol=1e-10, inner_prec="f32", delta=0.1,
                                         check_every=10)
    assert rc == dwa.DWA_OK
    for (ctx, eta), y, st in zip(batches, ys, stats):
        say(f"    {ctx.dims} Ls={ctx.Ls}: iters {[s['iters'] for s in st]}")
        assert all(s["rel_resid"] <= 1e-10 for s in st)
        y0, st0, rc0 = ctx.propagator(eta[5].contiguous(), tol=1e-10, check_every=10)
        assert rc0 == dwa.DWA_OK
        assert rel(y[5], y0) < 1e-7
    for ctx, _ in batches:
        ctx.close()


def test_batch_validation():
    ctx, w = _ctx("c1_4x4x4x4_ls8")
    eta = torch.from_numpy(spin_colour_sources(w["dims"])).to(gpu())
    with pytest.raises(dwa.DwaError) as e:
        ctx.propagator_batch(eta)  # nothing reserved
    assert e.value.status == dwa.DWA_EINVAL
    ctx.reserve_batch(4)
    with pytest.raises(dwa.DwaError) as e:
        ctx.propagator_batch(eta)  # 12 > 4
    assert e.value.status == dwa.DWA_EINVAL
    y, st, rc = ctx.propagator_batch(eta[:4].contiguous(), tol=1e-10)
    assert rc == dwa.DWA_OK and len(st) == 4
    ctx.close()


@pytest.mark.parametrize("Ls,nb", [(12, 1), (8, 2)])
def test_dbb_norm_epilogue_keeps_outputs(Ls, nb):
    """D_bb with the |out|^2 partial sums of the second hop writes the same fields as
    without them, bit for bit, on every repetition (16^3 x 32, FP64).  Guards the wide
    store whose data registers the norm epilogue must not overwrite too early."""
    dev = gpu()
    dims = (16, 16, 16, 32)
    ctx = dwa.Context(dims, Ls, -1.8, 0.02, 0.8, 1.5, 0.5)
    ctx.set_links(torch.from_numpy(synth.su3_field(dims, 0.5, 9)).to(dev))
    ctx.reserve_batch(nb)
    gen = torch.Generator(device=dev).manual_seed(5)
    x = torch.stack([ctx.half_field("f64") for _ in range(nb)]).contiguous()
    x.copy_(torch.randn(x.shape, dtype=x.dtype, device=dev, generator=gen))
    say(f"[gpu] D_bb norm epilogue 16^3x32 Ls={Ls} nb={nb}")
    ref = ctx.apply_Dbb_batch(x, "f64")
    ref_n = [float(torch.sum(torch.abs(ref[k]) ** 2)) for k in range(nb)]
    for rep in range(8):
        y, nrm = ctx.apply_Dbb_batch(x, "f64", norms=True)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), rep
        for k in range(nb):
            assert abs(nrm[k] - ref_n[k]) <= 1e-12 * ref_n[k]
    ctx.close()


def _dbb_pair(ctx, x, prec):
    return ctx.apply_Dbb(x, prec), ctx.apply_Dbb_dag(x, prec)


def _ctx_dims(dims, Ls, seed):
    ctx = dwa.Context(dims, Ls, -1.8, 0.05, 0.8, 1.5, 0.5)
    ctx.set_links(torch.from_numpy(synth.su3_field(dims, 0.5, seed)).to(gpu()))
    return ctx


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 8), ((8, 8, 8, 16), 12), ((4, 2, 2, 4), 5)])
def test_autotune_configurations_agree(dims, Ls):
    """Every tile / traversal gives bitwise the same D_bb and D_bb^dag in all three
    precisions; the autotuner keeps the fastest it timed; set_tuning validates; a solve
    after tuning agrees with one on the default configuration."""
    dev = gpu()
    ctx = _ctx_dims(dims, Ls, 17)
    gen = torch.Generator(device=dev).manual_seed(11)
    say(f"[gpu] autotune {dims} Ls={Ls}")
    for prec in ("f64", "f32", "bf16"):
        x = ctx.half_field(prec)
        if prec == "bf16":
            x.copy_(torch.randn(x.shape, device=dev, generator=gen).to(torch.bfloat16))
        else:
            x.copy_(torch.randn(x.shape, dtype=x.dtype, device=dev, generator=gen))
        ref = _dbb_pair(ctx, x, prec)
        res = ctx.autotune(prec, reps=3)
        timed = [c for c in res["candidates"] if c["us"] >= 0]
        say(f"    {prec}: chose ns={res['ns']} {res['order']} dense={res['dense']} ({res['us']:.1f} us of "
            + ", ".join(f"{c['ns']}/{c['order']}{'/dense' if c['dense'] else ''} {c['us']:.1f}"
                        for c in timed) + ")")
        assert timed and res["us"] == min(c["us"] for c in timed)
        assert any(c["dense"] for c in timed) and any(not c["dense"] for c in timed)
        tol = {"f64": 1e-13, "f32": 2e-6, "bf16": 2e-2}[prec]
        for c in timed:
            ctx.set_tuning(prec, c["ns"], c["order"], 1, c["dense"])
            got = _dbb_pair(ctx, x, prec)
            if not c["dense"]:  # the sweeps: the same arithmetic per site, so bitwise
                assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), (prec, c)
            else:  # the dense matrices: the same operator to rounding
                for g, r in zip(got, ref):
                    gf, rf = (g.float(), r.float()) if prec == "bf16" else (g, r)
                    assert float(torch.linalg.vector_norm(gf - rf) / torch.linalg.vector_norm(rf)) < tol, c
        ctx.set_tuning(prec, res["ns"], res["order"], res["nf"], res["dense"])
        if Ls not in (4, 8, 12, 16):
            assert {c["ns"] for c in res["candidates"]} == {8}
            with pytest.raises(dwa.DwaError):
                ctx.set_tuning(prec, 16, "slab")
    with pytest.raises(dwa.DwaError):
        ctx.set_tuning("f64", 24, "slab")
    with pytest.raises(dwa.DwaError):
        ctx.set_tuning("f64", 8, 3)
    eta = torch.from_numpy(synth.gaussian_source(dims, 3)).to(dev)
    y1, st, rc = ctx.propagator(eta, tol=1e-12, check_every=1)
    ctx2 = _ctx_dims(dims, Ls, 17)
    y0, st0, rc0 = ctx2.propagator(eta, tol=1e-12, check_every=1)
    assert rc == rc0 == dwa.DWA_OK
    assert rel(y1, y0) < 1e-10
    ctx.close()
    ctx2.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_fields_per_block_agree(prec):
    """A batched hop whose blocks apply their staged links to nf fields in turn gives,
    for every nf, bitwise the D_bb (and |D_bb x|^2 per field) of one field per block;
    with a batch reserved the autotuner times the fields per block too."""
    dev = gpu()
    dims, Ls, nb = (8, 8, 8, 16), 12, 12
    ctx = _ctx_dims(dims, Ls, 23)
    ctx.reserve_batch(nb)
    gen = torch.Generator(device=dev).manual_seed(29)
    x = torch.stack([ctx.half_field(prec) for _ in range(nb)]).contiguous()
    if prec == "bf16":
        x.copy_(torch.randn(x.shape, device=dev, generator=gen).to(torch.bfloat16))
    else:
        x.copy_(torch.randn(x.shape, dtype=x.dtype, device=dev, generator=gen))
    ns, order, _, dense = ctx.get_tuning(prec)
    ctx.set_tuning(prec, ns, order, 1, dense)
    ref, ref_n = ctx.apply_Dbb_batch(x, prec, norms=True)
    for nf in (2, 3, 4, 5, 12, 16):
        ctx.set_tuning(prec, ns, order, nf, dense)
        y, nrm = ctx.apply_Dbb_batch(x, prec, norms=True)
        assert torch.equal(y, ref), nf
        assert nrm == ref_n, nf
    res = ctx.autotune(prec, reps=3)
    batch = [c for c in res["candidates"] if c["nrhs"] > 1]
    say(f"[gpu] {prec} batched hop pair: " + ", ".join(f"nf={c['nf']} {c['us']:.1f} us" for c in batch)
        + f"; chose nf={res['nf']}")
    assert {c["nf"] for c in batch} == {1, 2, 3, 4, 6, 12}
    assert res["nf"] == min((c for c in batch if c["us"] >= 0), key=lambda c: c["us"])["nf"]
    y, nrm = ctx.apply_Dbb_batch(x, prec, norms=True)
    if not res["dense"]:
        assert torch.equal(y, ref)
    with pytest.raises(dwa.DwaError):
        ctx.set_tuning(prec, ns, order, 0, dense)
    ctx.close()


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_batch_with_zero_source(inner):
    """A zero source inside a batch gives y_1 = 0 at iteration 0; the other fields solve
    as they do alone."""
    ctx, w = _ctx("c1_4x4x4x4_ls8", 0.8)
    eta = torch.from_numpy(spin_colour_sources(w["dims"])[:4].copy()).to(gpu())
    eta[2].zero_()
    ctx.reserve_batch(4)
    y, st, rc = ctx.propagator_batch(eta, tol=1e-10, inner_prec=inner, check_every=1)
    assert rc == dwa.DWA_OK
    assert st[2]["iters"] == 0 and float(torch.max(torch.abs(y[2]))) == 0.0
    for k in (0, 1, 3):
        ys, s1, rc1 = ctx.propagator(eta[k].contiguous(), tol=1e-10, inner_prec=inner, check_every=1)
        assert rc1 == dwa.DWA_OK and st[k]["rel_resid"] <= 1e-10
        assert rel(y[k], ys) < 1e-8
    ctx.close()


def test_graph_replay_equals_eager(monkeypatch):
    """The batched CGNE replayed from a hipGraph (many replays, host checks and eager
    reliable updates between them) gives bitwise the result of the same launches issued
    one by one (DWA_BATCH_NO_GRAPH), for an FP64 and a BF16-inner batch."""
    ctx, w = _ctx("c2_8x8x8x16_ls12", 0.8)
    eta = torch.from_numpy(spin_colour_sources(w["dims"])[:6].copy()).to(gpu())
    ctx.reserve_batch(6)
    for kw in (dict(tol=1e-10, check_every=7), dict(tol=1e-10, inner_prec="bf16", delta=0.3, check_every=7)):
        y_g, st_g, rc_g = ctx.propagator_batch(eta, **kw)
        monkeypatch.setenv("DWA_BATCH_NO_GRAPH", "1")
        y_e, st_e, rc_e = ctx.propagator_batch(eta, **kw)
        monkeypatch.delenv("DWA_BATCH_NO_GRAPH")
        say(f"[gpu] graph vs eager {kw.get('inner_prec', 'f64')}: iters {[s['iters'] for s in st_g]}")
        assert rc_g == rc_e == dwa.DWA_OK
        assert [s["iters"] for s in st_g] == [s["iters"] for s in st_e]
        assert torch.equal(y_g, y_e)
        # the same solve with 3 fields per hop block: partial sums are grouped per field
        # and chunk either way, so the result is bitwise the same
        prec = kw.get("inner_prec", "f64")
        ns, order, nf0, dense = ctx.get_tuning(prec)
        ctx.set_tuning(prec, ns, order, 3, dense)
        y_m, st_m, rc_m = ctx.propagator_batch(eta, **kw)
        ctx.set_tuning(prec, ns, order, nf0, dense)
        assert rc_m == dwa.DWA_OK and torch.equal(y_m, y_g)
    ctx.close()


def test_dense_matrices_and_tuning_cache(tmp_path):
    """The dense fifth-dimension matrices (a tuning choice) against the oracle: FP64 D_bb
    and a full FP64 solve; and the JSON tuning cache: a second autotune with the same key
    applies the stored configuration without timing."""
    from oracle import redblack
    dev = gpu()
    dims, Ls = (4, 4, 4, 4), 8
    U = synth.su3_field(dims, 0.5, 31)
    p = redblack.Params.make(dims, Ls, -1.8, 0.05, 0.8, 1.5, 0.5)
    rb = redblack.RedBlack(U, p)
    ctx = dwa.Context(dims, Ls, -1.8, 0.05, 0.8, 1.5, 0.5)
    ctx.set_links(torch.from_numpy(U).to(dev))
    ctx.set_tuning("f64", 8, "slab", 1, True)
    assert ctx.get_tuning("f64")[3] is True
    x = synth.gaussian_field5(dims, Ls, 37) * rb.black
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    got = torch.zeros_like(xt)
    ctx.unpack(ctx.apply_Dbb(ctx.pack(xt, 0, "f64"), "f64"), 0, "f64", out=got)
    r = float(np.linalg.norm(got.cpu().numpy() - rb.Dbb(x)) / np.linalg.norm(rb.Dbb(x)))
    say(f"[gpu] dense D_bb rel err vs oracle {r:.1e}")
    assert r < 1e-13
    eta = synth.gaussian_source(dims, 41)
    y, st, rc = ctx.propagator(torch.from_numpy(eta).to(dev), tol=1e-12)
    y_ref, _ = redblack.propagator(U, eta, p, tol=1e-12)
    assert rc == dwa.DWA_OK
    assert float(np.linalg.norm(y.cpu().numpy() - y_ref) / np.linalg.norm(y_ref)) < 1e-9
    with pytest.raises(dwa.DwaError):
        ctx.set_tuning("f64", 16, "slab", 1, True)  # dense runs the 8-site kernel
    cache = str(tmp_path / "tune.json")
    first = ctx.autotune("bf16", reps=2, cache=cache)
    assert not first["cached"]
    ctx.set_tuning("bf16", 32 if first["ns"] != 32 else 16, "lex")
    second = ctx.autotune("bf16", reps=2, cache=cache)
    assert second["cached"] and second["us"] is None
    assert ctx.get_tuning("bf16") == (first["ns"], first["order"], first["nf"], first["dense"])
    ctx.close()
