"""The Schur forms of Sec. 3 on the GPU (dwa_propagator_form): eq.(redblack),
eq.(redblack1) and its row-scaled version give the oracle's y_1, and each form takes the
oracle's CGLS iteration count for that form (within one).  The counts themselves -- the
paper's reason for choosing eq.(redblack) with coefficients above one -- are printed;
their values on synthetic fields are parity unpinned."""

import sys

import numpy as np
import pytest

from oracle import pool, redblack
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


C1 = synth.WORKLOADS["c1_4x4x4x4_ls8"]


@pytest.mark.parametrize("coefs", ["moebius_1.5_0.5", "zolotarev"])
def test_schur_forms_match_oracle(coefs):
    dev = gpu()
    U = synth.workload_links("c1_4x4x4x4_ls8")
    Ls = C1["Ls"]
    if coefs == "zolotarev":
        probe = dwa.Context(C1["dims"], Ls, C1["M5"], C1["m"], 1.0, 1.0, 1.0)
        probe.set_links(torch.from_numpy(U).to(dev))
        lo, hi = probe.wilson_bounds(300)
        probe.close()
        b = c = dwa.zolotarev(lo, hi, Ls, "concave")[0]
    else:
        b, c = np.full(Ls, 1.5), np.full(Ls, 0.5)
    alpha = 0.8
    p = redblack.Params.make(C1["dims"], Ls, C1["M5"], C1["m"], alpha, b, c)
    eta = synth.point_source(C1["dims"], 0, 2, 1)
    say(f"[gpu] Schur forms, {coefs}: oracle solves")
    ref = pool.propagators(U, [eta] * 3, p, tol=1e-10, forms=[0, 1, 2])
    ctx = dwa.Context(C1["dims"], Ls, C1["M5"], C1["m"], alpha, b, c)
    ctx.set_links(torch.from_numpy(U).to(dev))
    e = torch.from_numpy(eta).to(dev)
    y_ref = ref[0][0]
    for form, (y_o, it_o) in zip(("redblack", "redblack1", "redblack1_scaled"), ref):
        y, st, rc = ctx.propagator_form(e, form, tol=1e-10)
        d = rel(y.cpu().numpy(), y_ref)
        say(f"    {form}: iters gpu {st['iters']} oracle {it_o}; eq.(redblack) residual "
            f"{st['rel_resid']:.1e}; y1 vs oracle {d:.1e}")
        assert rc == dwa.DWA_OK
        assert abs(st["iters"] - it_o) <= 1
        assert rel(y.cpu().numpy(), y_o) < 1e-8 and d < 1e-7
    with pytest.raises(dwa.DwaError) as ex:
        ctx.propagator_form(e, 3)
    assert ex.value.status == dwa.DWA_EINVAL
    ctx.close()
