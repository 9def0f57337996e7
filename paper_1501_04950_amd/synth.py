"""Seeded synthetic inputs: SU(3) gauge fields, APE-like smearing and 4D sources.

This module holds input generation only.  It contains none of the domain-wall
method's arithmetic, and both the HIP path and the CPU oracle consume the
arrays it returns unchanged (host FP64 / complex128, canonical layouts):

* links   ``U[mu][site][a][b]``  shape ``(4, V, 3, 3)``, mu = 0..3 = x, y, z, t
* 4D field ``eta[site][spin][colour]`` shape ``(V, 4, 3)``
* sites are lexicographic, ``site = x + Lx*(y + Ly*(z + Lz*t))``

The paper measures on three MILC 16^3x32 gauge fields (Sec. 3, Results) that
are not available here; the seeded fields below stand in for them.
"""

from __future__ import annotations

import numpy as np

# Parameter sets of the five workloads this library is measured and tested on.
# M5 is the literal value in the Wilson diagonal (4 + M5) of eq.(wilson): the
# usual domain-wall height 1.8 enters as M5 = -1.8, which gives the Wilson
# kernel the negative mass that makes the free overlap operator tend to m at
# zero momentum (with +1.8 it tends to 1 and the quark mass drops out).
WORKLOADS = {
    "c1_4x4x4x4_ls8": dict(dims=(4, 4, 4, 4), Ls=8, spread=0.3, seed=1501, M5=-1.8,
                           m=0.05, b=1.5, c=0.5, alphas=(1.0, 0.8), ape_steps=0),
    "c2_8x8x8x16_ls12": dict(dims=(8, 8, 8, 16), Ls=12, spread=0.5, seed=1502, M5=-1.8,
                             m=0.02, b=1.5, c=0.5, alphas=(0.6, 0.8, 1.0, 1.2), ape_steps=0),
    "c3_16x16x16x32_ls16": dict(dims=(16, 16, 16, 32), Ls=16, spread=0.7, seed=1503,
                                M5=-1.8, m=0.01, b=1.5, c=0.5,
                                alphas=tuple(round(0.5 + 0.1 * k, 1) for k in range(11)),
                                ape_steps=2, ape_coeff=0.5),
    "c5_8x8x8x8_ls8": dict(dims=(8, 8, 8, 8), Ls=8, spread=0.4, seed=1505, M5=-1.8,
                           m=0.05, b=1.5, c=0.5, alphas=(0.9,), ape_steps=0),
}
# Batched workload: three lattices with 12 point sources each, alpha = 0.8, m = 0.02.
BATCH_WORKLOAD = dict(
    lattices=[dict(dims=(8, 8, 8, 8), Ls=8), dict(dims=(12, 12, 12, 24), Ls=12),
              dict(dims=(16, 16, 16, 32), Ls=16)],
    spread=0.6, seed=1504, M5=-1.8, m=0.02, b=1.5, c=0.5, alpha=0.8)


def volume(dims) -> int:
    lx, ly, lz, lt = dims
    return lx * ly * lz * lt


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_su3(n: int, spread: float, rng: np.random.Generator) -> np.ndarray:
    """n matrices U = exp(i*spread*H), H a Gaussian traceless Hermitian 3x3."""
    a = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)[None]
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * spread * w)
    return np.einsum("nab,nb,ncb->nac", v, ph, np.conj(v))


def su3_field(dims, spread: float, seed: int) -> np.ndarray:
    """Seeded SU(3) links in canonical order [mu][t][z][y][x] -> shape (4, V, 3, 3)."""
    vol = volume(dims)
    u = random_su3(4 * vol, spread, _rng(seed))
    return np.ascontiguousarray(u.reshape(4, vol, 3, 3))


def unit_field(dims) -> np.ndarray:
    """Free field U = 1."""
    vol = volume(dims)
    u = np.zeros((4, vol, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def _grid(u, dims):
    lx, ly, lz, lt = dims
    return u.reshape(4, lt, lz, ly, lx, 3, 3)


_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # mu -> axis of a (t, z, y, x) grid


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _project_su3(v: np.ndarray) -> np.ndarray:
    """Polar projection V (V^dag V)^(-1/2), then divide by det^(1/3) (principal branch)."""
    vv = np.einsum("...ba,...bc->...ac", np.conj(v), v)
    w, q = np.linalg.eigh(vv)
    inv_sqrt = np.einsum("...ab,...b,...cb->...ac", q, 1.0 / np.sqrt(w), np.conj(q))
    unit = v @ inv_sqrt
    det = np.linalg.det(unit)
    return unit / (det ** (1.0 / 3.0))[..., None, None]


def ape_smear(u: np.ndarray, dims, coeff: float = 0.5, steps: int = 1) -> np.ndarray:
    """APE-like smearing: V = (1-coeff) U + coeff/6 * sum of the six staples, then
    projection back to SU(3); all links are updated together each step.  Gauge
    links are periodic in every direction."""
    g = _grid(u, dims).copy()
    for _ in range(steps):
        new = np.empty_like(g)
        for mu in range(4):
            am = _AXIS[mu]
            st = np.zeros_like(g[mu])
            for nu in range(4):
                if nu == mu:
                    continue
                an = _AXIS[nu]
                u_mu_xpnu = np.roll(g[mu], -1, axis=an)          # U_mu(x+nu)
                u_nu_xpmu = np.roll(g[nu], -1, axis=am)          # U_nu(x+mu)
                st += g[nu] @ u_mu_xpnu @ _dag(u_nu_xpmu)        # upper staple
                u_nu_xmnu = np.roll(g[nu], 1, axis=an)           # U_nu(x-nu)
                u_mu_xmnu = np.roll(g[mu], 1, axis=an)           # U_mu(x-nu)
                u_nu_xmnupmu = np.roll(u_nu_xmnu, -1, axis=am)   # U_nu(x-nu+mu)
                st += _dag(u_nu_xmnu) @ u_mu_xmnu @ u_nu_xmnupmu  # lower staple
            new[mu] = _project_su3((1.0 - coeff) * g[mu] + (coeff / 6.0) * st)
        g = new
    return np.ascontiguousarray(g.reshape(u.shape))


def plaquette(u: np.ndarray, dims) -> float:
    """Mean of Re tr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag) / 3 over x, mu<nu."""
    g = _grid(u, dims)
    acc, n = 0.0, 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            p = (g[mu] @ np.roll(g[nu], -1, axis=_AXIS[mu])
                 @ _dag(np.roll(g[mu], -1, axis=_AXIS[nu])) @ _dag(g[nu]))
            acc += np.trace(p, axis1=-2, axis2=-1).real.mean() / 3.0
            n += 1
    return acc / n


def workload_links(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    u = su3_field(w["dims"], w["spread"], w["seed"])
    if w.get("ape_steps", 0):
        u = ape_smear(u, w["dims"], w.get("ape_coeff", 0.5), w["ape_steps"])
    return u


def point_source(dims, site: int = 0, spin: int = 0, colour: int = 0) -> np.ndarray:
    eta = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    eta[site, spin, colour] = 1.0
    return eta


def z2_source(dims, seed: int) -> np.ndarray:
    """Each component (+-1 +- i)/sqrt(2)."""
    rng = _rng(seed)
    shape = (volume(dims), 4, 3)
    re = rng.integers(0, 2, size=shape) * 2 - 1
    im = rng.integers(0, 2, size=shape) * 2 - 1
    return (re + 1j * im) / np.sqrt(2.0)


def gaussian_source(dims, seed: int, leading=()) -> np.ndarray:
    rng = _rng(seed)
    shape = tuple(leading) + (volume(dims), 4, 3)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def gaussian_field5(dims, Ls: int, seed: int) -> np.ndarray:
    """Random 5D field [s][site][spin][colour] for operator-level tests."""
    return gaussian_source(dims, seed, leading=(Ls,))

