"""The roofline record of bench.py, checked on the CPU: the bound follows the kernel's
arithmetic intensity against the machine balance, the fractions are achieved / peak, and
the committed counter summaries are read only while they match the kernel source."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

DIMS, LS = (16, 16, 16, 32), 16
V = 16 * 16 * 16 * 32
VH = V // 2
EB = {"f64": 16, "f32": 8, "bf16": 4}  # bytes per complex value
S = {p: LS * 12 * VH * b for p, b in EB.items()}  # one half-lattice 5D field
L = {p: 4 * V * 9 * b for p, b in EB.items()}  # all links
ROOF_KERNEL = "dwa::hop_mix_kernel<dwa::BF16, 32, 16, 0, 2, false, false>"


def kern_record(hop_us):
    # a hop that moves its algorithmic bytes 2S + L in hop_us
    out = {}
    for p in EB:
        gbs = (2 * S[p] + L[p]) / (hop_us[p] * 1e-6) / 1e9
        out[p] = {"hop_us": hop_us[p], "hop_gbs": gbs, "hop_cold_us": 1.1 * hop_us[p],
                  "hop_cold_gbs": gbs / 1.1, "dbb_us": 3 * hop_us[p], "dbb_gbs": gbs / 1.2,
                  "dbb_dag_us": 3 * hop_us[p], "dbb_dag_gbs": gbs / 1.2}
    return out


TUNING = {"f64": {"ns": 16}, "f32": {"ns": 32}, "bf16": {"ns": 32}}
HOP_US = {"f64": 160.0, "f32": 80.0, "bf16": 48.0}


def test_bf16_hop_sits_under_the_alu_roof():
    rec = bench.make_roofline(kern_record(HOP_US), TUNING, "bf16", DIMS, LS, S, L, 6000.0)
    # Wilson hop (1320 flops per site) and the N sweeps (16 flops per complex value and
    # slice, 12 components) on V/2 sites and L_s slices, over 2S + L bytes
    flops = (1320 + 16 * 12) * VH * LS
    nbytes = 2 * S["bf16"] + L["bf16"]
    balance = 78.6e12 / 8e12
    assert flops / nbytes > balance  # 13.3 against 9.8 flop/B
    assert rec["bound"] == "alu" and rec["unit"] == "TFLOP/s"
    assert rec["peak"] == pytest.approx(78.6, abs=0.05)
    assert rec["achieved"] == pytest.approx(flops / 48e-6 / 1e12, rel=1e-3)
    assert rec["frac"] == pytest.approx(rec["achieved"] / rec["peak"], rel=1e-3)
    assert rec["bytes_per_launch"] == nbytes
    # HBM view beside it: achieved bytes against 8 TB/s and against the streaming rate
    hbm = rec["hbm"]
    assert hbm["frac"] == pytest.approx(nbytes / 48e-6 / 8e12, rel=1e-3)
    assert hbm["stream_ref_gbs"] == 6000.0
    assert hbm["frac_of_stream_ref"] == pytest.approx(nbytes / 48e-6 / 6e12, rel=1e-3)
    for p in EB:
        assert rec["per_precision"][p]["dbb_frac_of_stream_ref"] == pytest.approx(
            (2 * S[p] + L[p]) / (HOP_US[p] * 1e-6) / 1.2 / 6e12, rel=1e-3)


def test_fp64_hop_sits_under_the_hbm_roof():
    rec = bench.make_roofline(kern_record(HOP_US), TUNING, "f64", DIMS, LS, S, L)
    flops = (1320 + 16 * 12) * VH * LS
    nbytes = 2 * S["f64"] + L["f64"]
    assert flops / nbytes < 78.6e12 / 8e12
    assert rec["bound"] == "hbm" and rec["unit"] == "GB/s" and rec["peak"] == 8000.0
    assert rec["achieved"] == pytest.approx(nbytes / 160e-6 / 1e9, rel=1e-3)
    assert rec["frac"] == pytest.approx(rec["achieved"] / 8000.0, rel=1e-3)
    assert rec["hbm"]["stream_ref_gbs"] is None


def test_committed_counters_match_the_kernel_source():
    # the summaries under profiles/ were taken on the kernel source in the tree: bench.py
    # reports their traffic and VALU counts for the roofline kernel
    assert bench.measured_traffic(ROOF_KERNEL) == 157855829.0
    assert bench.measured_valu(ROOF_KERNEL) == 22315008.0
    rec = bench.make_roofline(kern_record(HOP_US), TUNING, "bf16", DIMS, LS, S, L)
    assert rec["traffic"] == 157855829.0
    assert rec["alu"]["valu_insts_per_launch"] == 22315008.0


def test_counters_of_another_kernel_source_are_not_reported(monkeypatch):
    monkeypatch.setattr(bench, "_kernel_sha", lambda: "0" * 16)
    assert bench.measured_traffic(ROOF_KERNEL) is None
    assert bench.measured_valu(ROOF_KERNEL) is None
    rec = bench.make_roofline(kern_record(HOP_US), TUNING, "bf16", DIMS, LS, S, L)
    assert rec["traffic"] is None
    assert rec["alu"]["valu_issue_frac"] is None
