"""dwa_apply_Dbb_static: D_bb with its intermediate fields in the library's static device
array (no allocation, no context workspace) equals dwa_apply_Dbb bit for bit, through the
C-ABI, on two calls in a row (the second on a smaller lattice), in every precision; a
lattice whose fields do not fit is rejected."""

import ctypes
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


def _ctx(dims, Ls, seed):
    rng = np.random.default_rng(seed)
    ctx = dwa.Context(dims, Ls, -1.8, 0.03, 0.9, rng.uniform(1.0, 2.0, Ls), rng.uniform(0.1, 0.9, Ls))
    ctx.set_links(torch.from_numpy(synth.su3_field(dims, 0.5, seed)).to(gpu()))
    return ctx


def _random_half(ctx, prec, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    h = ctx.half_field(prec, zero=False)
    if prec == "bf16":
        h.copy_(torch.randn(h.shape, generator=g).to(torch.bfloat16))
    else:
        h.copy_(torch.randn(h.shape, generator=g, dtype=h.dtype))
    return h


def _static(ctx, prec, x):
    out = ctx.half_field(prec)
    rc = dwa.lib().dwa_apply_Dbb_static(ctx._h, dwa.PREC[prec], ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()))
    return out, rc


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_static_dbb_equals_dbb_two_calls(prec):
    big = _ctx((8, 8, 8, 16), 12, 1601)   # FP64: 2 x 9.4 MB of the 64 MiB
    small = _ctx((4, 4, 2, 6), 8, 1602)   # ragged: 48 black sites
    for k, ctx in enumerate((big, small)):
        x = _random_half(ctx, prec, 1610 + k)
        say(f"[gpu] dwa_apply_Dbb_static {prec} {ctx.dims} Ls={ctx.Ls} (call {k + 1})")
        got, rc = _static(ctx, prec, x)
        torch.cuda.synchronize()
        assert rc == dwa.DWA_OK, dwa.lib().dwa_last_error()
        ref = ctx.apply_Dbb(x, prec)
        torch.cuda.synchronize()
        same = torch.equal(got.view(torch.uint8), ref.view(torch.uint8))
        say(f"    bitwise equal to dwa_apply_Dbb: {same}")
        assert same
    big.close()
    small.close()


def test_static_dbb_rejects_large_lattice():
    """Two FP32 half fields of 16^4, L_s = 16 take 2 x 50.3 MB > 64 MiB: DWA_EINVAL with a
    message, and nothing launched."""
    big = dwa.Context((16, 16, 16, 16), 16, -1.8, 0.03, 0.9, 1.5, 0.5)
    big.set_links(torch.from_numpy(synth.su3_field((16, 16, 16, 16), 0.5, 1604)).to(gpu()))
    xb = big.half_field("f32")
    say("[gpu] dwa_apply_Dbb_static on 16^4 Ls=16 f32 (2 x 50 MB): rejected")
    _, rc = _static(big, "f32", xb)
    assert rc == dwa.DWA_EINVAL
    assert b"static scratch" in dwa.lib().dwa_last_error()
    big.close()
