"""ctypes binding of libdwa (include/dwa.h).

Argument marshalling only: every arithmetic step runs in the HIP library.  Device
memory and streams come from PyTorch; fields are passed as ``tensor.data_ptr()``.
If ``libdwa.so`` has not been built this module raises on first use; there is no
fallback path.

Tensor shapes used by the wrappers:
  links            complex128 (4, V, 3, 3)
  4D field         complex128 (V, 4, 3)
  5D field         complex128 (Ls, V, 4, 3)
  half field F64   complex128 (Ls, 12, Vh)
  half field F32   complex64  (Ls, 12, Vh)
  half field BF16  bfloat16   (Ls, 12, Vh, 2)   (re, im)
"""

from __future__ import annotations

import ctypes
import json
import os
import re
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwa.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "dwa.h")

DWA_OK, DWA_EINVAL, DWA_ENOMEM, DWA_EHIP, DWA_ENOCONV, DWA_EBREAKDOWN, DWA_ENAN, DWA_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
DWA_F64, DWA_F32, DWA_BF16 = 0, 1, 2
PREC = {"f64": DWA_F64, "f32": DWA_F32, "bf16": DWA_BF16}
PREC_NAMES = {v: k for k, v in PREC.items()}
MIXED_MODES = {"reliable": 0, "defect": 1}

MIX_KINDS = {"identity": 0, "BG": 1, "N": 2, "Ginv_Iinv": 3, "g5_IinvT_Ginv": 4, "NT": 5,
             "G_BT_g5": 6, "Iinv": 7, "I_alpha": 8, "I_alpha_T": 9, "W_I": 10, "W_I_T": 11}
SCHUR_FORMS = {"redblack": 0, "redblack1": 1, "redblack1_scaled": 2}


class dwa_params(ctypes.Structure):
    _fields_ = [("dims", c_int * 4), ("Ls", c_int), ("M5", c_double), ("m", c_double),
                ("alpha", c_double), ("b", POINTER(c_double)), ("c", POINTER(c_double)),
                ("antiperiodic_t", c_int)]


class dwa_solve_opts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("maxiter", c_int), ("inner_prec", c_int), ("delta", c_double),
                ("check_every", c_int), ("warm_start", c_int), ("mixed_mode", c_int)]


class dwa_solve_stats(ctypes.Structure):
    _fields_ = [("iters", c_int), ("outer", c_int), ("converged", c_int), ("rel_resid", c_double),
                ("time_ms", c_double), ("n_Dbb", c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DwaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libdwa status {status}: {msg}")
        self.status = status


def _load_tune_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


class dwa_tune_entry(ctypes.Structure):
    _fields_ = [("prec", c_int), ("ns", c_int), ("order", c_int), ("nf", c_int), ("dense", c_int),
                ("nrhs", c_int), ("us", c_double)]


# block traversal orders of the fused hop (dwa_set_tuning)
HOP_ORDERS = {"slab": 0, "lex": 1, "zdom": 2}

_lib = None


def lib():
    """Load libdwa.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1501_04950_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "dwa_create": (c_int, [POINTER(c_void_p), POINTER(dwa_params), P]),
        "dwa_destroy": (c_int, [P]),
        "dwa_set_links": (c_int, [P, P]),
        "dwa_field_bytes": (c_size_t, [P, c_int, c_int]),
        "dwa_get_sizes": (c_int, [P, POINTER(c_longlong), POINTER(c_int)]),
        "dwa_pack_spinor5": (c_int, [P, c_int, P, P, c_int]),
        "dwa_unpack_spinor5": (c_int, [P, c_int, P, P, c_int]),
        "dwa_apply_Dw": (c_int, [P, P, P, c_int]),
        "dwa_apply_Dbb": (c_int, [P, c_int, P, P]),
        "dwa_apply_Dbb_dag": (c_int, [P, c_int, P, P]),
        "dwa_apply_Dbb_static": (c_int, [P, c_int, P, P]),
        "dwa_apply_hop": (c_int, [P, c_int, c_int, c_int, P, P]),
        "dwa_cgne_solve": (c_int, [P, P, P, POINTER(dwa_solve_opts), POINTER(dwa_solve_stats)]),
        "dwa_propagator": (c_int, [P, P, P, POINTER(dwa_solve_opts), POINTER(dwa_solve_stats), P]),
        "dwa_set_alpha": (c_int, [P, c_double]),
        "dwa_propagator_form": (c_int, [P, c_int, P, P, POINTER(dwa_solve_opts),
                                        POINTER(dwa_solve_stats)]),
        "dwa_overlap_apply": (c_int, [P, c_double, P, P, POINTER(dwa_solve_opts),
                                      POINTER(dwa_solve_stats)]),
        "dwa_alpha_sweep": (c_int, [P, POINTER(c_double), c_int, P, P, POINTER(dwa_solve_opts),
                                    POINTER(dwa_solve_stats)]),
        "dwa_propagator_adjoint": (c_int, [P, P, P, POINTER(c_double), POINTER(c_double),
                                           POINTER(c_double), POINTER(c_double), P, P, P,
                                           POINTER(dwa_solve_opts), POINTER(dwa_solve_stats)]),
        "dwa_reserve_batch": (c_int, [P, c_int]),
        "dwa_apply_Dbb_batch": (c_int, [P, c_int, c_int, P, P, POINTER(c_double)]),
        "dwa_propagator_batch": (c_int, [P, c_int, P, P, POINTER(dwa_solve_opts),
                                         POINTER(dwa_solve_stats)]),
        "dwa_propagator_multi": (c_int, [POINTER(c_void_p), c_int, POINTER(c_int), POINTER(c_void_p),
                                         POINTER(c_void_p), POINTER(dwa_solve_opts),
                                         POINTER(dwa_solve_stats)]),
        "dwa_cgne_solve_batch": (c_int, [POINTER(c_void_p), c_int, c_int, POINTER(c_void_p),
                                         POINTER(c_void_p), POINTER(dwa_solve_opts),
                                         POINTER(dwa_solve_stats)]),
        "dwa_zolotarev": (c_int, [c_double, c_double, c_int, c_int, POINTER(c_double),
                                  POINTER(c_double)]),
        "dwa_wilson_bounds": (c_int, [P, c_int, POINTER(c_double), POINTER(c_double)]),
        "dwa_autotune": (c_int, [P, c_int, c_int, POINTER(dwa_tune_entry), c_int, POINTER(c_int)]),
        "dwa_set_tuning": (c_int, [P, c_int, c_int, c_int, c_int, c_int]),
        "dwa_get_tuning": (c_int, [P, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                   POINTER(c_int)]),
        "dwa_strerror": (ctypes.c_char_p, [c_int]),
        "dwa_last_error": (ctypes.c_char_p, []),
        "dwa_debug_smatrix": (c_int, [POINTER(dwa_params), c_int, POINTER(c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/dwa.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dwa_[a-z0-9_A-Z]+)\s*\(", txt)))


def _raise(rc):
    L = lib()
    raise DwaError(rc, f"{L.dwa_strerror(rc).decode()} ({L.dwa_last_error().decode()})")


def check(rc, allow=()):
    if rc != DWA_OK and rc not in allow:
        _raise(rc)
    return rc


def make_params(dims, Ls, M5, m, alpha, b, c, antiperiodic_t=True):
    bb = np.ascontiguousarray(np.broadcast_to(np.asarray(b, dtype=np.float64), (Ls,)))
    cc = np.ascontiguousarray(np.broadcast_to(np.asarray(c, dtype=np.float64), (Ls,)))
    p = dwa_params()
    p.dims = (c_int * 4)(*[int(d) for d in dims])
    p.Ls, p.M5, p.m, p.alpha = int(Ls), float(M5), float(m), float(alpha)
    p.b = bb.ctypes.data_as(POINTER(c_double))
    p.c = cc.ctypes.data_as(POINTER(c_double))
    p.antiperiodic_t = 1 if antiperiodic_t else 0
    p._keep = (bb, cc)
    return p


def dwa_debug_smatrix(dims, Ls, M5, m, alpha, b, c, kind):
    """Host-only: the [2][Ls][Ls] fifth-dimension matrix of the given kind."""
    p = make_params(dims, Ls, M5, m, alpha, b, c)
    out = np.zeros((2, Ls, Ls), dtype=np.float64)
    k = MIX_KINDS[kind] if isinstance(kind, str) else int(kind)
    check(lib().dwa_debug_smatrix(byref(p), k, out.ctypes.data_as(POINTER(c_double))))
    return out


ZOLO_ORDERS = {"increasing": 0, "concave": 1, "decreasing": 2}


def zolotarev(lmin, lmax, Ls, ordering="concave"):
    """Zolotarev coefficients omega_i (per slice i_5) for b_i = c_i = omega_i and the
    deviation delta = max |prod (1 - omega x)/(1 + omega x)| on [lmin, lmax]
    (dwa_zolotarev; host only)."""
    om = np.zeros(int(Ls))
    d = c_double(0.0)
    o = ZOLO_ORDERS[ordering] if isinstance(ordering, str) else int(ordering)
    check(lib().dwa_zolotarev(float(lmin), float(lmax), int(Ls), o,
                              om.ctypes.data_as(POINTER(c_double)), byref(d)))
    return om, d.value


def _torch():
    import torch
    return torch


def _ptr(t):
    return c_void_p(t.data_ptr())


def check_storage(t):
    """Reject tensors whose storage does not hold their values: a lazily conjugated or
    negated view (``x.conj()``, ``-x`` of a conjugate) keeps the unconjugated numbers in
    memory and a flag on the tensor, and the library reads memory.  Resolve such views
    first (``t.resolve_conj().resolve_neg()``)."""
    if t.is_conj() or t.is_neg():
        raise ValueError("tensor is a lazy conjugate or negative view; call resolve_conj() / "
                         "resolve_neg() before passing it to the library")


class Context:
    """One lattice, parameter set and gauge field on the current GPU (dwa_create)."""

    def __init__(self, dims, Ls, M5, m, alpha, b, c, antiperiodic_t=True, stream=None):
        torch = _torch()
        self.dims, self.Ls = tuple(int(d) for d in dims), int(Ls)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.params = make_params(dims, Ls, M5, m, alpha, b, c, antiperiodic_t)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._batch_nmax = 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._h = c_void_p()
        check(lib().dwa_create(byref(self._h), byref(self.params), c_void_p(stream.cuda_stream)))

    def close(self):
        if self._h:
            lib().dwa_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- fields -------------------------------------------------------------
    def field_bytes(self, prec="f64", nrhs=1):
        """Bytes of nrhs half fields of precision prec (dwa_field_bytes)."""
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        return int(lib().dwa_field_bytes(self._h, p, int(nrhs)))

    def half_field(self, prec="f64", zero=True):
        torch = _torch()
        p = PREC[prec] if isinstance(prec, str) else prec
        shape = (self.Ls, 12, self.Vh)
        f = torch.zeros if zero else torch.empty
        if p == DWA_F64:
            return f(shape, dtype=torch.complex128, device=self.device)
        if p == DWA_F32:
            return f(shape, dtype=torch.complex64, device=self.device)
        return f(shape + (2,), dtype=torch.bfloat16, device=self.device)

    def _check_half(self, t, prec):
        torch = _torch()
        p = PREC[prec] if isinstance(prec, str) else prec
        want = {DWA_F64: torch.complex128, DWA_F32: torch.complex64, DWA_BF16: torch.bfloat16}[p]
        n = self.Ls * 12 * self.Vh * (2 if p == DWA_BF16 else 1)
        if t.dtype != want or not t.is_contiguous() or t.numel() != n or t.device != self.device:
            raise ValueError(f"half field must be a contiguous {want} tensor of {n} elements on {self.device}")
        check_storage(t)
        return p

    def _check_canon(self, t, shape):
        torch = _torch()
        if (t.dtype != torch.complex128 or not t.is_contiguous() or tuple(t.shape) != tuple(shape)
                or t.device != self.device):
            raise ValueError(f"expected contiguous complex128 {tuple(shape)} on {self.device}")
        check_storage(t)

    def set_links(self, U):
        self._check_canon(U, (4, self.V, 3, 3))
        check(lib().dwa_set_links(self._h, _ptr(U)))

    def pack(self, canon5, parity, prec="f64"):
        self._check_canon(canon5, (self.Ls, self.V, 4, 3))
        out = self.half_field(prec, zero=False)
        p = self._check_half(out, prec)
        check(lib().dwa_pack_spinor5(self._h, p, _ptr(out), _ptr(canon5), int(parity)))
        return out

    def unpack(self, half, parity, prec="f64", out=None):
        torch = _torch()
        p = self._check_half(half, prec)
        if out is None:
            out = torch.zeros((self.Ls, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        self._check_canon(out, (self.Ls, self.V, 4, 3))
        check(lib().dwa_unpack_spinor5(self._h, p, _ptr(out), _ptr(half), int(parity)))
        return out

    # -- operators ------------------------------------------------------------
    def apply_Dw(self, inp):
        torch = _torch()
        n = inp.shape[0]
        self._check_canon(inp, (n, self.V, 4, 3))
        out = torch.empty_like(inp)
        check(lib().dwa_apply_Dw(self._h, _ptr(out), _ptr(inp), int(n)))
        return out

    def apply_Dbb(self, inp, prec="f64", out=None, dagger=False):
        p = self._check_half(inp, prec)
        if out is None:
            out = self.half_field(prec, zero=False)
        self._check_half(out, prec)
        fn = lib().dwa_apply_Dbb_dag if dagger else lib().dwa_apply_Dbb
        check(fn(self._h, p, _ptr(out), _ptr(inp)))
        return out

    def apply_Dbb_dag(self, inp, prec="f64", out=None):
        return self.apply_Dbb(inp, prec, out, dagger=True)

    def apply_hop(self, inp, parity_out, kind="N", prec="f64", out=None):
        """One fused hop launch: out = M_kind (H inp) from parity 1 - parity_out."""
        p = self._check_half(inp, prec)
        if out is None:
            out = self.half_field(prec, zero=False)
        self._check_half(out, prec)
        k = MIX_KINDS[kind] if isinstance(kind, str) else int(kind)
        check(lib().dwa_apply_hop(self._h, p, int(parity_out), k, _ptr(out), _ptr(inp)))
        return out

    # -- tuning ---------------------------------------------------------------
    def autotune(self, prec="f64", reps=10, cache=None):
        """Time every tile / traversal of the fused hop for one storage precision, the
        dense fifth-dimension matrices against the sweeps, and (with a batch reserved)
        the fields per block of the batched hop, and keep the fastest (dwa_autotune).

        cache: path of a JSON file keyed by (GPU architecture, lattice, L_s, precision,
        batch reservation); a hit applies the stored configuration without timing, a
        miss tunes and stores the result.  Returns {"ns", "order", "nf", "dense", "us",
        "candidates", "cached"}; us is the chosen configuration's single-field hop-pair
        time (None when cached)."""
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        key = None
        if cache is not None:
            torch = _torch()
            arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
            key = "|".join(str(v) for v in (arch, "x".join(map(str, self.dims)), self.Ls,
                                            PREC_NAMES[p], self._batch_nmax))
            data = _load_tune_cache(cache)
            if key in data:
                c = data[key]
                self.set_tuning(p, c["ns"], c["order"], c["nf"], c["dense"])
                return {**c, "us": None, "candidates": [], "cached": True}
        ent = (dwa_tune_entry * 48)()
        n = c_int(0)
        check(lib().dwa_autotune(self._h, p, int(reps), ent, 48, byref(n)))
        names = {v: k for k, v in HOP_ORDERS.items()}
        cands = [{"ns": ent[i].ns, "order": names[ent[i].order], "nf": ent[i].nf,
                  "dense": bool(ent[i].dense), "nrhs": ent[i].nrhs, "us": ent[i].us}
                 for i in range(n.value)]
        ns, order, nf, dense = self.get_tuning(prec)
        us = min((c["us"] for c in cands if c["nrhs"] == 1 and c["ns"] == ns and c["order"] == order
                  and c["dense"] == dense), default=None)
        res = {"ns": ns, "order": order, "nf": nf, "dense": dense}
        if key is not None:
            data = _load_tune_cache(cache)
            data[key] = res
            tmp = f"{cache}.tmp{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return {**res, "us": us, "candidates": cands, "cached": False}

    def set_tuning(self, prec, ns, order="slab", nf=1, dense=False):
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        o = HOP_ORDERS[order] if isinstance(order, str) else int(order)
        check(lib().dwa_set_tuning(self._h, p, int(ns), o, int(nf), 1 if dense else 0))

    def get_tuning(self, prec):
        """(sites per block, block order, fields per block of a batched hop, dense)."""
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        ns, o, nf, d = c_int(0), c_int(0), c_int(0), c_int(0)
        check(lib().dwa_get_tuning(self._h, p, byref(ns), byref(o), byref(nf), byref(d)))
        return ns.value, {v: k for k, v in HOP_ORDERS.items()}[o.value], nf.value, bool(d.value)

    # -- solvers --------------------------------------------------------------
    @staticmethod
    def opts(tol=1e-10, maxiter=100000, inner_prec="f64", delta=0.1, check_every=1,
             warm_start=False, mixed_mode="reliable"):
        o = dwa_solve_opts()
        o.tol, o.maxiter = float(tol), int(maxiter)
        o.inner_prec = PREC[inner_prec] if isinstance(inner_prec, str) else int(inner_prec)
        o.delta, o.check_every, o.warm_start = float(delta), int(check_every), int(bool(warm_start))
        o.mixed_mode = MIXED_MODES[mixed_mode] if isinstance(mixed_mode, str) else int(mixed_mode)
        return o

    def cgne_solve(self, rhs, x=None, **kw):
        """Returns (x, stats dict, status)."""
        self._check_half(rhs, "f64")
        if x is None:
            x = self.half_field("f64")
        self._check_half(x, "f64")
        o = self.opts(**kw)
        st = dwa_solve_stats()
        rc = check(lib().dwa_cgne_solve(self._h, _ptr(x), _ptr(rhs), byref(o), byref(st)),
                   allow=(DWA_ENOCONV,))
        return x, st.as_dict(), rc

    def propagator(self, eta, want_psi=False, **kw):
        """Returns (y1, stats dict, status[, psi5])."""
        torch = _torch()
        self._check_canon(eta, (self.V, 4, 3))
        y1 = torch.zeros((self.V, 4, 3), dtype=torch.complex128, device=self.device)
        psi = None
        if want_psi:
            psi = torch.zeros((self.Ls, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        o = self.opts(**kw)
        st = dwa_solve_stats()
        rc = check(lib().dwa_propagator(self._h, _ptr(y1), _ptr(eta), byref(o), byref(st),
                                        _ptr(psi) if psi is not None else None),
                   allow=(DWA_ENOCONV,))
        if want_psi:
            return y1, st.as_dict(), rc, psi
        return y1, st.as_dict(), rc

    def propagator_form(self, eta, form="redblack1", **kw):
        """y_1 with the Schur system in one of the forms of Sec. 3 (dwa_propagator_form).
        Returns (y1, stats dict, status)."""
        torch = _torch()
        self._check_canon(eta, (self.V, 4, 3))
        y1 = torch.zeros((self.V, 4, 3), dtype=torch.complex128, device=self.device)
        f = SCHUR_FORMS[form] if isinstance(form, str) else int(form)
        o = self.opts(**kw)
        st = dwa_solve_stats()
        rc = check(lib().dwa_propagator_form(self._h, f, _ptr(y1), _ptr(eta), byref(o), byref(st)),
                   allow=(DWA_ENOCONV,))
        return y1, st.as_dict(), rc

    def overlap_apply(self, x, m, **kw):
        """D_OV(m) x through one 5D solve on this (mass 1) context (dwa_overlap_apply).
        Returns (D_OV(m) x, stats dict, status)."""
        torch = _torch()
        self._check_canon(x, (self.V, 4, 3))
        out = torch.zeros_like(x)
        o = self.opts(**kw)
        st = dwa_solve_stats()
        rc = check(lib().dwa_overlap_apply(self._h, float(m), _ptr(out), _ptr(x), byref(o), byref(st)),
                   allow=(DWA_ENOCONV,))
        return out, st.as_dict(), rc

    def propagator_adjoint(self, eta, eta_prime, want=("U", "eta", "alpha", "b", "c"), **kw):
        """Gradients of L = Re <eta', y_1> (dwa_propagator_adjoint).  Returns a dict with
        the requested entries of 'U' [4, V, 3, 3], 'eta' [V, 4, 3] (device complex128),
        'alpha' (float), 'b', 'c' (numpy [Ls]) plus 'L', 'y1', 'stats' and 'status'."""
        torch = _torch()
        self._check_canon(eta, (self.V, 4, 3))
        self._check_canon(eta_prime, (self.V, 4, 3))
        dev = self.device
        gU = torch.zeros((4, self.V, 3, 3), dtype=torch.complex128, device=dev) if "U" in want else None
        geta = torch.zeros((self.V, 4, 3), dtype=torch.complex128, device=dev) if "eta" in want else None
        ga = c_double(0.0)
        gb = np.zeros(self.Ls) if "b" in want else None
        gc = np.zeros(self.Ls) if "c" in want else None
        L = c_double(0.0)
        y1 = torch.zeros((self.V, 4, 3), dtype=torch.complex128, device=dev)
        o = self.opts(**kw)
        st = (dwa_solve_stats * 2)()
        dp = lambda a: a.ctypes.data_as(POINTER(c_double)) if a is not None else None
        rc = check(lib().dwa_propagator_adjoint(
            self._h, _ptr(gU) if gU is not None else None, _ptr(geta) if geta is not None else None,
            byref(ga) if "alpha" in want else None, dp(gb), dp(gc), byref(L), _ptr(y1),
            _ptr(eta), _ptr(eta_prime), byref(o), st), allow=(DWA_ENOCONV,))
        out = {"L": L.value, "y1": y1, "stats": [st[0].as_dict(), st[1].as_dict()], "status": rc}
        if gU is not None:
            out["U"] = gU
        if geta is not None:
            out["eta"] = geta
        if "alpha" in want:
            out["alpha"] = ga.value
        if gb is not None:
            out["b"] = gb
        if gc is not None:
            out["c"] = gc
        return out

    def wilson_bounds(self, steps=200):
        """(lambda_min, lambda_max) estimates of |gamma_5 D_w| by Lanczos on the GPU
        (dwa_wilson_bounds)."""
        lo, hi = c_double(0.0), c_double(0.0)
        check(lib().dwa_wilson_bounds(self._h, int(steps), byref(lo), byref(hi)))
        return lo.value, hi.value

    def reserve_batch(self, nmax):
        check(lib().dwa_reserve_batch(self._h, int(nmax)))
        self._batch_nmax = int(nmax)

    def apply_Dbb_batch(self, x, prec="f64", out=None, norms=False):
        """D_bb on a batch of half fields x [n, ...] (dwa_apply_Dbb_batch); with norms,
        also |out|^2 per field from the kernel's partial sums."""
        if out is None:
            out = _torch().empty_like(x)
        n = int(x.shape[0])
        nrm = (c_double * n)() if norms else None
        check(lib().dwa_apply_Dbb_batch(self._h, PREC[prec], n, _ptr(out), _ptr(x), nrm))
        return (out, [nrm[i] for i in range(n)]) if norms else out

    def propagator_batch(self, eta, **kw):
        """y_1 for a batch of sources eta [n, V, 4, 3] (dwa_propagator_batch).
        Returns (y1 [n, V, 4, 3], list of stats dicts, status)."""
        y, st, rc = propagator_multi([(self, eta)], **kw)
        return y[0], st[0], rc

    def set_alpha(self, alpha):
        check(lib().dwa_set_alpha(self._h, float(alpha)))
        self.params.alpha = float(alpha)

    def alpha_sweep(self, eta, alphas, **kw):
        """The alpha study: y_1 and solve statistics for each alpha (Sec. 3).
        Returns (y1 [n, V, 4, 3], list of stats dicts, status)."""
        torch = _torch()
        self._check_canon(eta, (self.V, 4, 3))
        a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).ravel())
        n = a.size
        y1 = torch.zeros((n, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        o = self.opts(**kw)
        st = (dwa_solve_stats * n)()
        rc = check(lib().dwa_alpha_sweep(self._h, a.ctypes.data_as(POINTER(c_double)), n, _ptr(y1),
                                         _ptr(eta), byref(o), st), allow=(DWA_ENOCONV,))
        return y1, [st[i].as_dict() for i in range(n)], rc


def propagator_multi(batches, **kw):
    """Batched propagators over several contexts in one solve (dwa_propagator_multi).
    batches: list of (Context, eta [n_i, V_i, 4, 3]).  Returns (list of y1 batches,
    list of per-context stats lists, status)."""
    torch = _torch()
    nctx = len(batches)
    ctxs = (c_void_p * nctx)()
    nr = (c_int * nctx)()
    ys, etas = [], []
    for i, (ctx, eta) in enumerate(batches):
        if eta.dim() != 4:
            raise ValueError("eta must be [n, V, 4, 3]")
        ctx._check_canon(eta[0], (ctx.V, 4, 3))
        if not eta.is_contiguous():
            raise ValueError("eta must be contiguous")
        ctxs[i] = ctx._h.value
        nr[i] = eta.shape[0]
        ys.append(torch.zeros_like(eta))
        etas.append(eta)
    yp = (c_void_p * nctx)(*[y.data_ptr() for y in ys])
    ep = (c_void_p * nctx)(*[e.data_ptr() for e in etas])
    o = Context.opts(**kw)
    total = sum(nr)
    st = (dwa_solve_stats * total)()
    rc = check(lib().dwa_propagator_multi(ctxs, nctx, nr, yp, ep, byref(o), st), allow=(DWA_ENOCONV,))
    out, k = [], 0
    for i in range(nctx):
        out.append([st[k + j].as_dict() for j in range(nr[i])])
        k += nr[i]
    return ys, out, rc


def cgne_solve_batch(batches, **kw):
    """Batched Schur-level CGNE over several contexts (dwa_cgne_solve_batch): D_bb x = rhs
    for every right-hand side.  batches: list of (Context, rhs [n, Ls, 12, Vh] complex128
    black half fields), the same n for every context.  Returns (list of x batches, list of
    per-context stats lists, status)."""
    torch = _torch()
    nctx = len(batches)
    if nctx < 1:
        raise ValueError("no batches")
    n = int(batches[0][1].shape[0])
    ctxs = (c_void_p * nctx)()
    xs, rhss = [], []
    for i, (ctx, rhs) in enumerate(batches):
        if rhs.dim() != 4 or int(rhs.shape[0]) != n or not rhs.is_contiguous():
            raise ValueError("rhs must be a contiguous [n, Ls, 12, Vh] batch, the same n everywhere")
        ctx._check_half(rhs[0], "f64")
        check_storage(rhs)
        ctxs[i] = ctx._h.value
        xs.append(torch.zeros_like(rhs))
        rhss.append(rhs)
    xp = (c_void_p * nctx)(*[x.data_ptr() for x in xs])
    rp = (c_void_p * nctx)(*[r.data_ptr() for r in rhss])
    o = Context.opts(**kw)
    st = (dwa_solve_stats * (nctx * n))()
    rc = check(lib().dwa_cgne_solve_batch(ctxs, nctx, n, xp, rp, byref(o), st), allow=(DWA_ENOCONV,))
    return xs, [[st[i * n + j].as_dict() for j in range(n)] for i in range(nctx)], rc
