"""The propagator y_1 as a differentiable torch operation.

``propagator(ctx, U, eta, alpha, b, c, **opts)`` returns y_1 for the context's lattice
and parameters, with the links U and the source eta taken from the arguments.  Its
backward runs ``dwa_propagator_adjoint`` with the incoming gradient of y_1 as eta':
for a real loss L, torch's gradient of a complex tensor is dL/dRe + i dL/dIm, which is
the convention of the library, so d L / d y_1 is exactly the eta' of
L = Re <eta', y_1> for the linearised loss.  alpha, b and c are real tensors holding the
context's values (the context is built with them); they receive ordinary derivatives.
All arithmetic runs in libdwa; this module only moves tensors.
"""

import torch

from . import dwa


def _plain(t):
    """t detached, with any lazy conjugate / negative bit applied to the values, and
    contiguous: the library reads the memory, not the tensor's flags.  Autograd hands
    over such views, e.g. the gradient of Re sum(y.conj() * w) is a lazy conjugate."""
    return t.detach().resolve_conj().resolve_neg().contiguous()


class _Propagator(torch.autograd.Function):
    @staticmethod
    def forward(fctx, U, eta, alpha, b, c, holder, opts):
        holder.set_links(_plain(U))
        y1, st, rc = holder.propagator(_plain(eta), **opts)
        fctx.holder, fctx.opts = holder, opts
        fctx.save_for_backward(U, eta)
        fctx.stats = st
        return y1

    @staticmethod
    def backward(fctx, gy):
        U, eta = fctx.saved_tensors
        holder = fctx.holder
        need = fctx.needs_input_grad
        want = tuple(k for k, i in (("U", 0), ("eta", 1), ("alpha", 2), ("b", 3), ("c", 4)) if need[i])
        holder.set_links(_plain(U))
        g = holder.propagator_adjoint(_plain(eta), _plain(gy), want=want, **fctx.opts)
        dev = eta.device
        out = [None] * 7
        if need[0]:
            out[0] = g["U"]
        if need[1]:
            out[1] = g["eta"]
        if need[2]:
            out[2] = torch.tensor(g["alpha"], dtype=torch.float64, device=dev)
        if need[3]:
            out[3] = torch.from_numpy(g["b"]).to(dev)
        if need[4]:
            out[4] = torch.from_numpy(g["c"]).to(dev)
        return tuple(out)


def propagator(holder: dwa.Context, U, eta, alpha=None, b=None, c=None, **opts):
    """y_1 of eta for the links U on the context ``holder``; differentiable in U, eta
    and (when given as tensors that require grad) alpha, b, c.  alpha, b and c must hold
    the values the context was created with (or set by ``set_alpha``)."""
    p = holder.params
    dev = eta.device
    if alpha is None:
        alpha = torch.tensor(p.alpha, dtype=torch.float64, device=dev)
    if b is None:
        b = torch.tensor([p.b[i] for i in range(holder.Ls)], dtype=torch.float64, device=dev)
    if c is None:
        c = torch.tensor([p.c[i] for i in range(holder.Ls)], dtype=torch.float64, device=dev)
    if abs(float(alpha) - p.alpha) > 1e-15 * max(1.0, abs(p.alpha)):
        raise ValueError("alpha differs from the context's alpha (use Context.set_alpha)")
    for name, t, ref in (("b", b, p.b), ("c", c, p.c)):
        vals = t.detach().cpu().tolist()
        if len(vals) != holder.Ls or any(abs(v - ref[i]) > 1e-15 * max(1.0, abs(ref[i]))
                                         for i, v in enumerate(vals)):
            raise ValueError(f"{name} differs from the context's {name} (create a new context)")
    return _Propagator.apply(U, eta, alpha, b, c, holder, opts)
