#!/usr/bin/env python3
"""Benchmark of the alpha-Moebius domain-wall propagator on one MI355X.

Workload (the paper-shaped configuration): 16^3 x 32 lattice, Ls = 16, seeded
SU(3) links of spread 0.7 after two APE-like smearing steps (coefficient 0.5),
M5 = -1.8 (Wilson diagonal 2.2), m = 0.01, b = 1.5, c = 0.5, Z2-noise source.

One step is one full pass of the hot path: source rho = D_1(1) P b, Schur
right-hand side, CG on the normal equations of D_bb to a 1e-10 relative residual
(mixed precision: CGLS with low-precision storage and FP64 reliable updates),
reconstruction and extraction of y_1.  Inputs are resident in HBM before the timed
region.  The JSON line reports the mixed-precision time to 1e-10 as `value`, the
FP64 time beside it, D_bb bandwidth per precision, the roofline of the fused hop
kernel (HIP events on the library's stream), and the CPU oracle on a bounded sample.
"""

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

METRIC = "CGNE time-to-1e-10 + D_bb HBM GB/s, mixed vs FP64, 16^3x32 L_s=16"
HBM_PEAK_GBS = 8000.0
FLOPS_PER_SITE_DW = 1320


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_16x16x16x32_ls16")
    ap.add_argument("--inner", default="bf16", choices=["f32", "bf16"])
    ap.add_argument("--delta", type=float, default=None)
    ap.add_argument("--mixed-mode", default="reliable", choices=["reliable", "defect"])
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--check-every", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference solve")
    ap.add_argument("--no-sweep", action="store_true", help="skip the alpha sweep")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient (adjoint) timing")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default hop tiles instead of running the autotuner")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched 3-lattice x 12-source solve")
    ap.add_argument("--no-zolo", action="store_true",
                    help="skip the Zolotarev-coefficient study")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the eq.(redblack) vs eq.(redblack1) comparison")
    ap.add_argument("--no-overlap", action="store_true",
                    help="skip the overlap-operator application")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 4^4 and 8^3x16 time-to-solution runs")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 512 MiB device copy (scale reference for HBM counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): a solve is not "
              "split across GPUs in this library", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1501_04950_amd import dwa, synth

    w = synth.WORKLOADS[args.workload]
    dims, Ls = w["dims"], w["Ls"]
    V = int(np.prod(dims))
    Vh = V // 2
    log(f"generating links {dims} Ls={Ls}")
    U = synth.workload_links(args.workload)
    plaq = synth.plaquette(U, dims)
    eta = synth.z2_source(dims, w["seed"] + 100)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    ctx = dwa.Context(dims, Ls, w["M5"], w["m"], args.alpha, w["b"], w["c"])
    Ud = torch.from_numpy(U).to(dev)
    ctx.set_links(Ud)
    eta_d = torch.from_numpy(eta).to(dev)
    torch.cuda.synchronize()

    # --- autotuner: tile and block traversal of the fused hop, per precision --------
    tuning = {}
    for prec in ("f64", "f32", "bf16"):
        if args.no_tune:
            ns, order, _, _ = ctx.get_tuning(prec)
            tuning[prec] = {"ns": ns, "order": order, "tuned": False}
            continue
        t0 = time.perf_counter()
        res = ctx.autotune(prec, reps=10)
        tuning[prec] = {"ns": res["ns"], "order": res["order"], "dense": res["dense"],
                        "pair_us": round(res["us"], 2),
                        "tuned": True, "tune_s": round(time.perf_counter() - t0, 3),
                        "candidates": [[c["ns"], c["order"], "dense" if c["dense"] else "sweep",
                                        round(c["us"], 2)] for c in res["candidates"]]}
        log(f"autotune {prec}: ns={res['ns']} order={res['order']} pair {res['us']:.1f} us")

    eb = {"f64": 16, "f32": 8, "bf16": 4}
    S = {p: Ls * 12 * Vh * eb[p] for p in eb}
    L = {p: 4 * V * 9 * eb[p] for p in eb}

    def ev_time(fn, reps):
        """Average milliseconds of fn() over reps, HIP events on the library stream."""
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for i in range(reps):
            fn(i)
        end.record(stream)
        end.synchronize()
        return start.elapsed_time(end) / reps

    # --- kernel and operator bandwidth (rotating buffers, > 512 MiB per set) ------
    kern = {}
    for prec in ("f64", "f32", "bf16"):
        nset = max(2, int(np.ceil(600e6 / (2 * S[prec]))))
        ins = [ctx.half_field(prec) for _ in range(nset)]
        for t in ins:
            if prec == "bf16":
                t.copy_(torch.randn(t.shape, device=dev).to(torch.bfloat16))
            else:
                t.copy_(torch.randn(t.shape, dtype=t.dtype, device=dev))
        outs = [ctx.half_field(prec) for _ in range(nset)]
        reds = [ctx.half_field(prec) for _ in range(nset)]
        log(f"timing {prec}: {nset} buffer sets")
        for i in range(3):
            ctx.apply_hop(ins[i % nset], 1, "N", prec, out=reds[i % nset])
        # cold: rotating buffer sets, so inputs come from HBM, not the 256 MB Infinity Cache
        hop_cold_ms = ev_time(lambda i: ctx.apply_hop(ins[i % nset], 1, "N", prec, out=reds[i % nset]),
                              args.kernel_reps)
        # as inside a solve: the input was written just before (one buffer set)
        ctx.apply_hop(ins[0], 1, "N", prec, out=reds[0])
        hop_ms = ev_time(lambda i: ctx.apply_hop(ins[0], 1, "N", prec, out=reds[0]), args.kernel_reps)
        dbb_ms = ev_time(lambda i: ctx.apply_Dbb(ins[i % nset], prec, out=outs[i % nset]),
                         args.kernel_reps)
        dag_ms = ev_time(lambda i: ctx.apply_Dbb_dag(ins[i % nset], prec, out=outs[i % nset]),
                         args.kernel_reps)
        hop_bytes = 2 * S[prec] + L[prec]
        dbb_bytes = 5 * S[prec] + 2 * L[prec]
        kern[prec] = {
            "hop_us": hop_ms * 1e3, "hop_gbs": hop_bytes / hop_ms / 1e6,
            "hop_cold_us": hop_cold_ms * 1e3, "hop_cold_gbs": hop_bytes / hop_cold_ms / 1e6,
            "dbb_us": dbb_ms * 1e3, "dbb_gbs": dbb_bytes / dbb_ms / 1e6,
            "dbb_dag_us": dag_ms * 1e3, "dbb_dag_gbs": dbb_bytes / dag_ms / 1e6,
            "dbb_gflops": FLOPS_PER_SITE_DW * V * Ls / dbb_ms / 1e6,
        }
        log(f"  {prec}: hop {kern[prec]['hop_us']:.1f} us {kern[prec]['hop_gbs']:.0f} GB/s "
            f"(cold {kern[prec]['hop_cold_us']:.1f} us) | "
            f"D_bb {kern[prec]['dbb_us']:.1f} us {kern[prec]['dbb_gbs']:.0f} GB/s")
        del ins, outs, reds
        torch.cuda.empty_cache()

    stream_gbs = stream_reference_gbs(torch, dev)
    log(f"  streaming reference (torch add, 3 x 256 MiB): {stream_gbs:.0f} GB/s")

    if args.copy_probe:
        a = torch.empty(512 * 2**20 // 4, dtype=torch.float32, device=dev).normal_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # --- FP64 reference solve ---------------------------------------------------------
    fp64 = None
    y64 = None
    if not args.no_fp64:
        log("FP64 propagator solve (warm-up, then median of 3)")
        kw64 = dict(tol=args.tol, inner_prec="f64", check_every=args.check_every)
        ctx.propagator(eta_d, **kw64)
        t64 = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            y64, st64, rc = ctx.propagator(eta_d, **kw64)
            torch.cuda.synchronize()
            t64.append(time.perf_counter() - t0)
        fp64 = {"time_s": round(statistics.median(t64), 4), "runs_s": [round(t, 4) for t in t64],
                "iters": st64["iters"], "n_Dbb": st64["n_Dbb"], "rel_resid": st64["rel_resid"],
                "status": rc}
        log(f"  FP64: {fp64['time_s']:.3f} s, {st64['iters']} iters, resid {st64['rel_resid']:.2e}")

    # --- mixed-precision steps (timed) ------------------------------------------------
    # delta: the reliable-update threshold, or the inner tolerance of a defect-correction
    # restart (both picked by sweeps on this workload)
    default_delta = {("reliable", "bf16"): 0.3, ("reliable", "f32"): 0.02,
                     ("defect", "bf16"): 0.01, ("defect", "f32"): 0.01}
    delta = args.delta if args.delta is not None else default_delta[(args.mixed_mode, args.inner)]
    kw = dict(tol=args.tol, inner_prec=args.inner, delta=delta, check_every=args.check_every,
              mixed_mode=args.mixed_mode)
    for i in range(args.warmup):
        log(f"warmup {i}")
        ctx.propagator(eta_d, **kw)
    torch.cuda.synchronize()
    times, stats = [], []
    y = None
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y, st, rc = ctx.propagator(eta_d, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(st)
        log(f"step {i}: {times[-1]:.3f} s, iters {st['iters']} outer {st['outer']} "
            f"resid {st['rel_resid']:.2e} status {rc}")
    mixed_s = statistics.mean(times)
    # the other FP64 outer scheme on the same solve: restarted defect correction beside
    # reliable updates (or the reverse), median of 3 after a warm-up
    other_mode = "defect" if args.mixed_mode == "reliable" else "reliable"
    okw = dict(kw, mixed_mode=other_mode, delta=default_delta[(other_mode, args.inner)])
    ctx.propagator(eta_d, **okw)
    ots = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ost, orc = ctx.propagator(eta_d, **okw)
        torch.cuda.synchronize()
        ots.append(time.perf_counter() - t0)
    other = {"mixed_mode": other_mode, "delta": okw["delta"], "time_s": round(statistics.median(ots), 4),
             "iters": ost["iters"], "outer": ost["outer"], "rel_resid": ost["rel_resid"], "status": orc}
    log(f"other outer scheme ({other_mode}, delta {okw['delta']}): {other['time_s']:.3f} s, "
        f"iters {ost['iters']} outer {ost['outer']}")
    y_err = None
    if y64 is not None:
        y_err = float(torch.linalg.vector_norm(y - y64) / torch.linalg.vector_norm(y64))

    # --- gradients of L = Re <eta', y_1> (adjoint state): forward solve, adjoint solve
    # on D_bb^dag and the force kernels, with the mixed solves and with FP64 solves ----
    grad = None
    if not args.no_grad:
        eta_p = torch.from_numpy(synth.gaussian_source(dims, w["seed"] + 200)).to(dev)
        grad = {}
        for inner in (args.inner, "f64"):
            gkw = dict(kw, inner_prec=inner) if inner != "f64" else dict(tol=args.tol, inner_prec="f64",
                                                                          check_every=args.check_every)
            ctx.propagator_adjoint(eta_d, eta_p, **gkw)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g = ctx.propagator_adjoint(eta_d, eta_p, **gkw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            grad[inner] = {"time_s": round(dt, 4), "fwd_iters": g["stats"][0]["iters"],
                           "adj_iters": g["stats"][1]["iters"],
                           "adj_rel_resid": g["stats"][1]["rel_resid"], "status": g["status"]}
            log(f"gradients ({inner} solves): {dt:.3f} s, iters fwd {g['stats'][0]['iters']} "
                f"adj {g['stats'][1]['iters']}, adj resid {g['stats'][1]['rel_resid']:.1e}")
            if inner == args.inner:
                gU = g["U"]
        grad["ratio_to_forward_solve"] = round(grad[args.inner]["time_s"] / mixed_s, 3)
        grad["U_rel_diff_mixed_vs_f64"] = float(torch.linalg.vector_norm(gU - g["U"]) /
                                                torch.linalg.vector_norm(g["U"]))
        del g, gU

    # --- alpha study (Sec. 3): FP64 CGNE iteration counts n(alpha) -------------------
    sweep = None
    if not args.no_sweep:
        alphas = [round(0.5 + 0.1 * i, 2) for i in range(11)]
        log(f"alpha sweep {alphas[0]}..{alphas[-1]} (FP64)")
        ys, sts, rc = ctx.alpha_sweep(eta_d, alphas, tol=args.tol, inner_prec="f64",
                                      check_every=1)
        iters = [st["iters"] for st in sts]
        n1 = iters[alphas.index(1.0)]
        best = min(range(len(alphas)), key=lambda i: iters[i])
        ratio = iters[best] / n1
        y_ref = ys[alphas.index(1.0)]
        spread = max(float(torch.linalg.vector_norm(ys[i] - y_ref) / torch.linalg.vector_norm(y_ref))
                     for i in range(len(alphas)))
        sweep = {"alpha": alphas, "iters": iters, "rel_iters": [round(i / n1, 4) for i in iters],
                 "time_s": [round(st["time_ms"] / 1e3, 4) for st in sts],
                 "best_alpha": alphas[best], "best_rel_iters": round(ratio, 4),
                 "speedup_1_minus_ratio": round(1 - ratio, 4),
                 "speedup_inverse_ratio_minus_1": round(1 / ratio - 1, 4),
                 "y1_max_rel_diff_across_alpha": spread}
        log(f"  iters {iters}; best alpha {alphas[best]} ratio {ratio:.3f}; y1 spread {spread:.1e}")
        del ys
        # the mixed-precision solve again at the best alpha (same y_1, fewer iterations):
        # a warm-up, then the median of 3, as for the other solve times
        ctx.set_alpha(alphas[best])
        ctx.propagator(eta_d, **kw)
        tb = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            yb, stb, rcb = ctx.propagator(eta_d, **kw)
            torch.cuda.synchronize()
            tb.append(time.perf_counter() - t0)
        sweep["mixed_at_best_alpha"] = {
            "alpha": alphas[best], "time_s": round(statistics.median(tb), 4),
            "runs_s": [round(v, 4) for v in tb],
            "speedup_vs_alpha1": round(mixed_s / statistics.median(tb), 3),
            "iters": stb["iters"], "rel_resid": stb["rel_resid"],
            "y1_rel_diff_vs_alpha1": float(torch.linalg.vector_norm(yb - y) / torch.linalg.vector_norm(y))}
        ctx.set_alpha(args.alpha)
        log(f"  mixed at alpha {alphas[best]}: {sweep['mixed_at_best_alpha']['time_s']} s, "
            f"{stb['iters']} iters")

    # --- batched solve: 3 lattices x 12 spin-colour sources against 36 single solves -
    batch = None
    if not args.no_batch:
        batch = batch_bench(torch, dwa, synth, dev, stream, args)

    # --- Zolotarev coefficients with the concave ordering, and their alpha sweep -------
    zolo = None
    if not args.no_zolo:
        zolo = zolotarev_study(torch, dwa, Ud, w, args)

    # --- the Schur forms of Sec. 3: eq.(redblack) against eq.(redblack1) -------------
    forms = None
    if not args.no_forms:
        forms = schur_form_study(torch, dwa, Ud, w, zolo)

    # --- the overlap operator through the 5D engine ---------------------------------
    ovl = None
    if not args.no_overlap:
        ovl = overlap_study(torch, dwa, Ud, w, eta_d, y if y is not None else None)

    # --- the small workloads (launch-latency bound): time to solution ----------------
    small = None
    if not args.no_small:
        log("small workloads: 4^4 Ls=8 and 8^3x16 Ls=12 solves")
        small = small_solves(torch, dwa, synth, dev)

    # --- CPU oracle on a bounded sample ---------------------------------------------
    cpu = None
    if not args.no_cpu:
        c1_gpu = None
        if small is not None:
            g = small["c1_4x4x4x4_ls8"]["f64"]
            c1_gpu = {"gpu_s": g["time_s"], "gpu_iters": g["iters"]}
        cpu = cpu_baseline(U, dims, Ls, w, args.alpha, fp64, c1_gpu)

    roofline = make_roofline(kern, tuning, args.inner, dims, Ls, S, L, stream_gbs)
    result = {
        "metric": METRIC,
        "value": round(mixed_s, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed_s * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{dims[0]}^3x{dims[3]} Ls={Ls} m={w['m']} alpha={args.alpha} "
                               f"M5={w['M5']} b={w['b']} c={w['c']} Z2 source, tol {args.tol}",
                   "plaquette": round(plaq, 6), "storage": args.inner, "arithmetic": "f32",
                   "outer": "f64 reliable updates" if args.mixed_mode == "reliable" else "f64 defect correction",
                   "inner": args.inner, "delta": delta,
                   "mixed_mode": args.mixed_mode},
        "other_outer_scheme": other,
        "mixed": {"time_s": round(mixed_s, 4), "iters": stats[-1]["iters"],
                  "outer": stats[-1]["outer"], "rel_resid": stats[-1]["rel_resid"],
                  "y1_rel_diff_vs_fp64": y_err},
        "fp64": fp64,
        "speedup_mixed_vs_fp64": round(fp64["time_s"] / mixed_s, 3) if fp64 else None,
        "dbb": {p: {k: round(v, 2) for k, v in kern[p].items()} for p in kern},
        "roofline": roofline,
        "tuning": tuning,
        "small_workloads": small,
        "zolotarev": zolo,
        "schur_forms": forms,
        "overlap": ovl,
        "gradients": grad,
        "alpha_sweep": sweep,
        "batch": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)
    ctx.close()


def batch_bench(torch, dwa, synth, dev, stream, args):
    """The batched workload: 8^4 / Ls 8, 12^3x24 / Ls 12 and 16^3x32 / Ls 16 with the 12
    spin-colour point sources each, solved to 1e-10 with FP32 inner solves and again with
    BF16 inner solves, all 36 systems in one dwa_propagator_multi call, against the same
    36 systems solved one at a time.  Also the batched D_bb of 12 FP32 fields on
    16^3x32 against 12 single applications."""
    bw = synth.BATCH_WORKLOAD
    batches = []
    for k, lat in enumerate(bw["lattices"]):
        dims, Ls = lat["dims"], lat["Ls"]
        ctx = dwa.Context(dims, Ls, bw["M5"], bw["m"], bw["alpha"], bw["b"], bw["c"])
        ctx.set_links(torch.from_numpy(synth.su3_field(dims, bw["spread"], bw["seed"] + k)).to(dev))
        ctx.reserve_batch(12)
        if not args.no_tune:
            for prec in ("f64", "f32", "bf16"):
                ctx.autotune(prec, reps=5)
        eta = torch.from_numpy(np.stack([synth.point_source(dims, 0, j // 3, j % 3)
                                         for j in range(12)])).to(dev)
        batches.append((ctx, eta))

    def solve_both(kw, label):
        log(f"batch: 3 lattices x 12 sources, {label} inner (warmup)")
        dwa.propagator_multi(batches, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ys, sts, rc = dwa.propagator_multi(batches, **kw)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        log(f"  batched: {t_batch:.3f} s, status {rc}")
        for ctx, eta in batches:  # warm each context's single-solve path
            ctx.propagator(eta[0].contiguous(), **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq, seq_iters = [], []
        for ctx, eta in batches:
            ylat, it = [], []
            for j in range(12):
                y, st, _ = ctx.propagator(eta[j].contiguous(), **kw)
                ylat.append(y)
                it.append(st["iters"])
            seq.append(ylat)
            seq_iters.append(it)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        log(f"  sequential: {t_seq:.3f} s")
        diff = max(float(torch.linalg.vector_norm(ys[i][j] - seq[i][j]) / torch.linalg.vector_norm(seq[i][j]))
                   for i in range(3) for j in range(12))
        lat = []
        for (ctx, _), st, it in zip(batches, sts, seq_iters):
            lat.append({"dims": list(ctx.dims), "Ls": ctx.Ls,
                        "batch_iters": [s["iters"] for s in st], "single_iters": it,
                        "max_rel_resid": max(s["rel_resid"] for s in st)})
        return {"inner": kw["inner_prec"], "delta": kw["delta"], "status": rc,
                "batched_s": round(t_batch, 4), "sequential_s": round(t_seq, 4),
                "speedup": round(t_seq / t_batch, 3), "max_y1_rel_diff_batch_vs_single": diff,
                "lattices": lat}

    r32 = solve_both(dict(tol=args.tol, inner_prec="f32", delta=0.1, check_every=args.check_every), "FP32")
    r16 = solve_both(dict(tol=args.tol, inner_prec="bf16", delta=0.3, check_every=args.check_every), "BF16")
    # the same 36 systems batched in plain FP64 (one timed run): the time the mixed
    # batches are measured against at equal accuracy
    log("batch: 3 lattices x 12 sources, FP64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sts64, rc64 = dwa.propagator_multi(batches, tol=args.tol, inner_prec="f64", check_every=args.check_every)
    torch.cuda.synchronize()
    f64_batched = {"batched_s": round(time.perf_counter() - t0, 4), "status": rc64,
                   "iters": [max(s["iters"] for s in st) for st in sts64],
                   "max_rel_resid": max(s["rel_resid"] for st in sts64 for s in st)}
    log(f"  FP64 batched: {f64_batched['batched_s']:.3f} s")
    # batched D_bb, 12 FP32 fields on the largest lattice
    ctx = batches[2][0]
    x = torch.stack([ctx.half_field("f32") for _ in range(12)]).contiguous()
    x.copy_(torch.randn(x.shape, dtype=x.dtype, device=dev))
    out = torch.empty_like(x)
    ctx.apply_Dbb_batch(x, "f32", out=out)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(5):
        ctx.apply_Dbb_batch(x, "f32", out=out)
    end.record(stream)
    end.synchronize()
    batch_ms = start.elapsed_time(end) / 5
    ns, order, nf, dense = ctx.get_tuning("f32")
    ctx.set_tuning("f32", ns, order, 1, dense)
    ctx.apply_Dbb_batch(x, "f32", out=out)
    start.record(stream)
    for _ in range(5):
        ctx.apply_Dbb_batch(x, "f32", out=out)
    end.record(stream)
    end.synchronize()
    batch_nf1_ms = start.elapsed_time(end) / 5
    ctx.set_tuning("f32", ns, order, nf, dense)
    start.record(stream)
    for _ in range(5):
        for j in range(12):
            ctx.apply_Dbb(x[j], "f32", out=out[j])
    end.record(stream)
    end.synchronize()
    single_ms = start.elapsed_time(end) / 5
    Vh = ctx.Vh
    S = ctx.Ls * 12 * Vh * 8
    Lb = 4 * 2 * Vh * 9 * 8
    dbb = {"fields": 12, "fields_per_block": nf, "batched_ms": round(batch_ms, 3),
           "batched_one_field_per_block_ms": round(batch_nf1_ms, 3), "single_x12_ms": round(single_ms, 3),
           "batched_gbs_per_field_model": round(12 * (5 * S + 2 * Lb) / batch_ms / 1e6, 1)}
    log(f"  D_bb x12 FP32 16^3x32: batched {batch_ms:.3f} ms ({nf} fields per block; 1: "
        f"{batch_nf1_ms:.3f} ms), 12 single {single_ms:.3f} ms")
    for c, _ in batches:
        c.close()
    out = {"workload": "8^4/Ls8 + 12^3x24/Ls12 + 16^3x32/Ls16, 12 point sources each, "
                       f"spread {bw['spread']}, alpha {bw['alpha']}, m {bw['m']}, tol {args.tol}"}
    out.update(r32)  # FP32 inner at the top level, as before
    out["bf16_inner"] = r16
    out["f64"] = f64_batched
    out["dbb_batch"] = dbb
    return out


# Per-site-slice algorithmic flops of the roofline kernel (a hop of eq.(wilson) followed by
# the fifth-dimension matrix N = B I_1^-1): the Wilson hop at the usual 1320 flops per
# site, and the O(L_s) sweeps of N, 16 flops per complex value and slice (a cyclic
# bidiagonal solve: scale, one FMA pair and the closure correction; a bidiagonal
# multiply: scale and one FMA pair) for the 12 colour-spin components.
HOP_FLOPS = 1320
MIX_N_FLOPS = 16 * 12
# gfx950: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; a wave64 VALU instruction occupies a SIMD
# for 4 cycles, so 39.3e12 lane-instructions/s, i.e. 78.6 TFLOP/s of FP32 FMA without
# packed-FP32 instructions (which this build does not emit)
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
FP32_FMA_PEAK_TFLOPS = 2 * VALU_LANE_OPS_PEAK / 1e12


def stream_reference_gbs(torch, dev, reps=20):
    """HBM bandwidth a plain streaming kernel reaches here: torch.add over three FP32
    tensors of 256 MiB (two read, one written; 768 MiB, beyond the 256 MB Infinity Cache),
    bytes moved / mean launch time over `reps` launches.  Context for the HBM fractions,
    which stay against the 8 TB/s peak."""
    n = 256 * 2**20 // 4
    a = torch.empty(n, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a).uniform_()
    c = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, b, out=c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(a, b, out=c)
    e1.record()
    e1.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 3 * n * 4 / s / 1e9


def make_roofline(kern, tuning, inner, dims, Ls, S, L, stream_gbs=None):
    """Roofline record of the dominant kernel (the first hop of D_bb in the inner
    precision, hop_mix_kernel MODE 0 with the N mix), against both resources it can be
    bound by: HBM bytes (algorithmic 2S + L per launch, timed as inside a solve and cold)
    and VALU arithmetic (algorithmic flops; beside them the VALU issue fraction from the
    committed SQ_INSTS_VALU count per launch, when it was taken on the kernel source built
    here).  `bound` follows the classical roofline: "alu" when the kernel's arithmetic
    intensity (algorithmic flops per algorithmic byte) exceeds the machine balance (FP32
    vector peak / HBM peak), else "hbm"; for "alu", achieved / peak are algorithmic FP32
    TFLOP/s against 78.6.  With stream_gbs (stream_reference_gbs) the HBM record also
    gives the in-solve hop and every precision's D_bb as a fraction of that rate."""
    V = int(np.prod(dims))
    dom = kern[inner]
    ns_dom = tuning[inner]["ns"]
    name = f"dwa::hop_mix_kernel<dwa::{inner.upper()}, {ns_dom}, {Ls}, 0, 2, false, false>"
    hop_s = dom["hop_us"] * 1e-6
    hbm_frac = dom["hop_gbs"] / HBM_PEAK_GBS
    valu = measured_valu(name)
    flops = (HOP_FLOPS + MIX_N_FLOPS) * V // 2 * Ls
    alu = {"algorithmic_flops_per_launch": flops,
           "achieved_tflops": round(flops / hop_s / 1e12, 2),
           "peak_tflops": round(FP32_FMA_PEAK_TFLOPS, 1),
           "frac_algorithmic": round(flops / hop_s / 1e12 / FP32_FMA_PEAK_TFLOPS, 4),
           "valu_insts_per_launch": valu,
           "valu_issue_frac": round(valu * 64 / (hop_s * VALU_LANE_OPS_PEAK), 4) if valu else None}
    per_prec = {p: {"hop_frac_in_solve": round(kern[p]["hop_gbs"] / HBM_PEAK_GBS, 4),
                    "hop_frac_cold": round(kern[p]["hop_cold_gbs"] / HBM_PEAK_GBS, 4),
                    "dbb_frac": round(kern[p]["dbb_gbs"] / HBM_PEAK_GBS, 4),
                    "dbb_dag_frac": round(kern[p]["dbb_dag_gbs"] / HBM_PEAK_GBS, 4)} for p in kern}
    if stream_gbs:
        for p in kern:
            per_prec[p]["dbb_frac_of_stream_ref"] = round(kern[p]["dbb_gbs"] / stream_gbs, 4)
    bytes_launch = 2 * S[inner] + L[inner]
    intensity = flops / bytes_launch
    balance = FP32_FMA_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    bound = "alu" if intensity > balance else "hbm"
    rec = {"bound": bound,
           "arithmetic_intensity_flop_per_byte": round(intensity, 2),
           "machine_balance_flop_per_byte": round(balance, 2),
           "kernel": f"hop_mix_kernel<{inner.upper()},{ns_dom},{Ls},0> (fused Wilson hop + N mix)",
           "traffic": measured_traffic(name),
           "bytes_per_launch": 2 * S[inner] + L[inner],
           "timing": "HIP events on the library stream, input written just before (as in the solve)",
           "hbm": {"achieved_gbs": round(dom["hop_gbs"], 1), "frac": round(hbm_frac, 4),
                   "achieved_cold_gbs": round(dom["hop_cold_gbs"], 1),
                   "frac_cold": round(dom["hop_cold_gbs"] / HBM_PEAK_GBS, 4),
                   "stream_ref_gbs": round(stream_gbs, 1) if stream_gbs else None,
                   "frac_of_stream_ref": round(dom["hop_gbs"] / stream_gbs, 4) if stream_gbs else None},
           "alu": alu,
           "per_precision": per_prec}
    if bound == "alu":
        rec.update(achieved=alu["achieved_tflops"], peak=alu["peak_tflops"], unit="TFLOP/s",
                   frac=alu["frac_algorithmic"])
    else:
        rec.update(achieved=round(dom["hop_gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=round(hbm_frac, 4))
    return rec


def _kernel_sha():
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in ("kcommon.h", "khop.h"):
        h.update(open(os.path.join(here, "paper_1501_04950_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _profile_value(fname, key, kernel):
    """The per-launch figure `key` of `kernel` from a committed counter summary, or None
    when the summary was taken on a different kernel source than the one built here."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        sha = _kernel_sha()
        for line in open(os.path.join(here, "profiles", fname)):
            f = line.split()
            if f[:1] == [key] and " ".join(f[1:-3]) == kernel:
                return float(f[-3]) if f[-1] == sha else None
    except OSError:
        pass
    return None


def measured_valu(kernel):
    return _profile_value("hop_mix_kernel_16x16x16x32_ls16_valu.md", "valu_insts_per_launch", kernel)


def measured_traffic(kernel):
    return _profile_value("hop_mix_kernel_16x16x16x32_ls16_traffic.md", "traffic_bytes_per_launch", kernel)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _timed(fn):
    """(result, wall seconds, threads used = CPU seconds / wall seconds) of fn()."""
    c0, t0 = time.process_time(), time.perf_counter()
    r = fn()
    wall = time.perf_counter() - t0
    return r, wall, (time.process_time() - c0) / wall


def cpu_baseline(U, dims, Ls, w, alpha, fp64, c1_gpu, dbb_reps=3):
    """The oracle as it stands, timed on this host's cores.

    value: one full oracle propagator solve, wall clock, on the 4^4, L_s = 8 workload
    (point source, alpha = 1, tol 1e-10): source, Schur right-hand side, CGLS,
    reconstruction and extraction, exactly as the tests call it.  The same solve on the
    GPU (FP64, host check every iteration) is reported beside it.  Also measured: the
    oracle's D_bb on the 16^3 x 32, L_s = 16 workload (median of dbb_reps
    applications); an estimate of an oracle solve of that workload (that median times
    the D_bb applications of the GPU FP64 solve) is reported separately, labelled as an
    estimate."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import redblack
    from paper_1501_04950_amd import synth

    c1 = synth.WORKLOADS["c1_4x4x4x4_ls8"]
    log("CPU oracle: full propagator solve on 4^4 Ls=8")
    p1 = redblack.Params.make(c1["dims"], c1["Ls"], c1["M5"], c1["m"], 1.0, c1["b"], c1["c"])
    U1 = synth.workload_links("c1_4x4x4x4_ls8")
    eta1 = synth.point_source(c1["dims"], 0, 0, 0)
    (y1, info), wall1, thr1 = _timed(lambda: redblack.propagator(U1, eta1, p1, tol=1e-10))
    log(f"  oracle 4^4 solve: {wall1:.2f} s, {info.iters} iterations, {thr1:.1f} threads")

    log(f"CPU oracle: {dbb_reps} D_bb applications on the full workload")
    p = redblack.Params.make(dims, Ls, w["M5"], w["m"], alpha, w["b"], w["c"])
    rb = redblack.RedBlack(U, p)
    x = synth.gaussian_field5(dims, Ls, 5) * rb.black
    walls, thr = [], []
    for _ in range(dbb_reps):
        _, wt, th = _timed(lambda: rb.Dbb(x))
        walls.append(wt)
        thr.append(th)
        log(f"  oracle D_bb: {wt:.1f} s")
    dbb_med = statistics.median(walls)
    n_dbb = fp64.get("n_Dbb") if fp64 else None
    est = dbb_med * n_dbb if n_dbb else None
    S = Ls * 12 * (int(np.prod(dims)) // 2) * 16
    L = 4 * int(np.prod(dims)) * 9 * 16
    return {"value": round(wall1, 3), "unit": "s",
            "cores": max(1, round(max([thr1] + thr))),
            "host_cores_available": len(os.sched_getaffinity(0)),
            "cpu_model": _cpu_model(),
            "kind": "oracle",
            "sample": (f"one full oracle propagator solve (numpy, FP64) of the 4^4 Ls=8 workload, "
                       f"point source, alpha 1, tol 1e-10: {info.iters} CGLS iterations, wall clock"),
            "c1_solve": {"oracle_s": round(wall1, 3), "oracle_iters": info.iters,
                         "oracle_threads": round(thr1, 2), **(c1_gpu or {})},
            "c3_dbb": {"oracle_median_s": round(dbb_med, 2), "oracle_runs_s": [round(v, 2) for v in walls],
                       "oracle_threads": round(statistics.median(thr), 2),
                       "oracle_model_gbs": round((5 * S + 2 * L) / dbb_med / 1e9, 3)},
            "c3_solve_estimate": {"value_s": round(est, 1) if est else None, "estimate": True,
                                  "how": f"oracle D_bb median x {n_dbb} D_bb applications of the GPU "
                                         "FP64 solve of the same system (not a timed solve)"}}


def zolotarev_study(torch, dwa, Ud, w, args, Ls=10, m=0.06, steps=300):
    """The Zolotarev row of the paper's table (m = 0.06, Ls = 10) on the paper-shaped
    field: spectral bounds of |gamma_5 D_w| by Lanczos on the GPU, Zolotarev coefficients
    b_i = c_i = omega_i for them, FP64 CGNE iteration counts (host check every iteration,
    tol 1e-10) for the concave, increasing and decreasing orders at alpha = 1, and the
    alpha sweep with the concave order; beside it the constant b = c = 1 of the table's
    other rows at the same m and Ls.  Iteration counts on synthetic fields: parity
    unpinned (the paper's are for MILC fields)."""
    from paper_1501_04950_amd import synth
    dims = w["dims"]
    eta = torch.from_numpy(synth.z2_source(dims, w["seed"] + 100)).to(Ud.device)
    probe = dwa.Context(dims, Ls, w["M5"], m, 1.0, 1.0, 1.0)
    probe.set_links(Ud)
    t0 = time.perf_counter()
    lo, hi = probe.wilson_bounds(steps)
    t_bounds = time.perf_counter() - t0
    probe.close()
    log(f"Zolotarev: |gamma5 D_w| in [{lo:.5f}, {hi:.5f}] ({steps} Lanczos steps, {t_bounds:.2f} s)")
    out = {"workload": f"{dims[0]}^3x{dims[3]} Ls={Ls} m={m} M5={w['M5']} Z2 source, FP64 CGNE to 1e-10",
           "lanczos_steps": steps, "lambda_min": lo, "lambda_max": hi, "bounds_s": round(t_bounds, 3)}
    kw = dict(tol=1e-10, inner_prec="f64", check_every=1)
    alphas = [0.15, 0.2, 0.25, 0.3, 0.4, 0.5, 0.6, 0.8, 1.0, 1.2]

    def sweep(ctx):
        ys, sts, rc = ctx.alpha_sweep(eta, alphas, **kw)
        it = [s_["iters"] for s_ in sts]
        n1 = it[alphas.index(1.0)]
        best = min(range(len(alphas)), key=lambda i: it[i])
        return ys[alphas.index(1.0)], {
            "alpha": alphas, "iters": it, "rel_iters": [round(i / n1, 4) for i in it],
            "best_alpha": alphas[best], "best_iters": it[best], "best_rel_iters": round(it[best] / n1, 4),
            "speedup_1_minus_ratio": round(1 - it[best] / n1, 4), "status": rc}

    y_ref = None
    for order in ("concave", "increasing", "decreasing"):
        om, delta = dwa.zolotarev(lo, hi, Ls, order)
        ctx = dwa.Context(dims, Ls, w["M5"], m, 1.0, om, om)
        ctx.set_links(Ud)
        y1, rec = sweep(ctx)
        ctx.close()
        if order == "concave":
            out["omega_concave"] = [round(v, 6) for v in om]
            out["delta"] = delta
            y_ref = y1
        else:
            rec["y1_rel_diff_vs_concave"] = float(torch.linalg.vector_norm(y1 - y_ref) /
                                                  torch.linalg.vector_norm(y_ref))
        out[order] = rec
        log(f"  {order}: iters {rec['iters']}; best alpha {rec['best_alpha']}")
    ctx = dwa.Context(dims, Ls, w["M5"], m, 1.0, 1.0, 1.0)
    ctx.set_links(Ud)
    _, out["constant_b1_c1"] = sweep(ctx)
    ctx.close()
    log(f"  constant b = c = 1: iters {out['constant_b1_c1']['iters']}")
    return out


def schur_form_study(torch, dwa, Ud, w, zolo):
    """Sec. 3's comparison of the Schur forms on the paper-shaped field: CGNE iteration
    counts (FP64, tol 1e-10 on each form's own residual, alpha = 1) of eq.(redblack),
    eq.(redblack1) and eq.(redblack1) with its rows scaled, for the bench's Moebius
    coefficients (b = 1.5, c = 0.5, Ls = 16, m = 0.01) and, when the Zolotarev study ran,
    its concave Zolotarev coefficients (Ls = 10, m = 0.06).  Every form reaches the same
    solution; the eq.(redblack) residual of each result is reported.  Counts on synthetic
    fields: parity unpinned."""
    from paper_1501_04950_amd import synth
    dims = w["dims"]
    eta = torch.from_numpy(synth.z2_source(dims, w["seed"] + 100)).to(Ud.device)
    cases = [("moebius b=1.5 c=0.5", w["Ls"], w["m"], w["b"], w["c"])]
    if zolo:
        om = np.array(zolo["omega_concave"])
        cases.append(("zolotarev concave", len(om), 0.06, om, om))
    out = {}
    for name, Ls, m, b, c in cases:
        ctx = dwa.Context(dims, Ls, w["M5"], m, 1.0, b, c)
        ctx.set_links(Ud)
        rec, y0 = {"Ls": Ls, "m": m}, None
        for form in ("redblack", "redblack1", "redblack1_scaled"):
            y, st, rc = ctx.propagator_form(eta, form, tol=1e-10, maxiter=20000)
            if y0 is None:
                y0 = y
            rec[form] = {"iters": st["iters"], "status": rc, "redblack_resid": st["rel_resid"],
                         "time_s": round(st["time_ms"] / 1e3, 3),
                         "y1_rel_diff_vs_redblack": float(torch.linalg.vector_norm(y - y0) /
                                                          torch.linalg.vector_norm(y0))}
            log(f"Schur form {form} ({name}): {st['iters']} iters, eq.(redblack) resid {st['rel_resid']:.1e}")
        out[name] = rec
        ctx.close()
    return out


def overlap_study(torch, dwa, Ud, w, eta, y_mixed):
    """The 4D overlap operator D_OV(m) through one 5D solve of mass 1 (App. A,
    eq.(startprop)) on the paper-shaped field: the time of one application (FP64 CGNE to
    1e-10) and the residual |D_OV(m) y_1 - eta| / |eta| of the bench's mixed-precision y_1."""
    dims = w["dims"]
    ctx = dwa.Context(dims, w["Ls"], w["M5"], 1.0, 1.0, w["b"], w["c"])
    ctx.set_links(Ud)
    ctx.overlap_apply(eta, w["m"], tol=1e-10, check_every=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, st, rc = ctx.overlap_apply(eta, w["m"], tol=1e-10, check_every=5)
    torch.cuda.synchronize()
    rec = {"workload": f"D_OV(m={w['m']}) on the Z2 source, mass-1 solve in FP64 to 1e-10",
           "time_s": round(time.perf_counter() - t0, 4), "iters": st["iters"], "status": rc}
    if y_mixed is not None:
        back, st2, rc2 = ctx.overlap_apply(y_mixed, w["m"], tol=1e-12, check_every=5)
        rec["residual_of_mixed_y1"] = float(torch.linalg.vector_norm(back - eta) / torch.linalg.vector_norm(eta))
    log(f"overlap apply: {rec['time_s']} s, {st['iters']} iters; D_OV y_1 residual "
        f"{rec.get('residual_of_mixed_y1')}")
    ctx.close()
    return rec


def small_solves(torch, dwa, synth, dev):
    """Time to solution of the two small workloads (launch-latency bound): the 4^4, L_s =
    8 point source (FP64; a host check every iteration, which stops at the oracle's
    iteration, and every 5, which replays 5 iterations from the graph per check) and the
    8^3 x 16, L_s = 12 point source (FP64 and FP32 inner), tol 1e-10, median of 5 after a
    warm-up."""
    out = {}
    for name, inners in (("c1_4x4x4x4_ls8", ("f64", "f64_check5")), ("c2_8x8x8x16_ls12", ("f64", "f32"))):
        w = synth.WORKLOADS[name]
        ctx = dwa.Context(w["dims"], w["Ls"], w["M5"], w["m"], 1.0, w["b"], w["c"])
        ctx.set_links(torch.from_numpy(synth.workload_links(name)).to(dev))
        eta = torch.from_numpy(synth.point_source(w["dims"], 0, 0, 0)).to(dev)
        res = {}
        for key in inners:
            inner = key.split("_")[0]
            check = 1 if key == "f64" and name.startswith("c1") else 5
            kw = dict(tol=1e-10, inner_prec=inner, check_every=check)
            if inner != "f64":
                kw["delta"] = 0.05
            ctx.propagator(eta, **kw)
            ts = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                y, st, rc = ctx.propagator(eta, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[key] = {"time_s": round(statistics.median(ts), 5), "iters": st["iters"],
                        "rel_resid": st["rel_resid"], "status": rc, "check_every": kw["check_every"]}
            log(f"  {name} {key}: {res[key]['time_s'] * 1e3:.2f} ms, {st['iters']} iters")
        out[name] = res
        ctx.close()
    return out


if __name__ == "__main__":
    main()
