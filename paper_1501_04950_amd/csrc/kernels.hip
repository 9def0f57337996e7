// gfx950 kernels of libdwa.
//
// Field layout (one parity, "SoA"): element (s, comp, cb) of a 5D half field sits at
// (s * 12 + comp) * Vh + cb, comp = spin * 3 + colour, so a wavefront of consecutive
// checkerboard sites reads or writes one contiguous run per (s, comp).  Links of one
// precision are [parity][mu][row*3+col][cb] with the antiperiodic time phase folded in.
// nbr[p][dir][cb] is the checkerboard index (in the other parity) of the neighbour
// x + mu (dir = mu) or x - mu (dir = 4 + mu) of the output site cb of parity p.
#include <hip/hip_runtime.h>

#include "dwa_internal.h"

namespace dwa {

namespace {

constexpr int RED_THREADS = 256;

template <typename S>
using RealOf = typename S::real;

// the value a complex number has after a store/load round trip in storage S
template <typename S>
__device__ __forceinline__ cpx<RealOf<S>> as_stored(cpx<RealOf<S>> v) {
  if constexpr (S::prec == DWA_BF16) {
    return cmk<float>(bf16_to_f32(f32_to_bf16_rne(v.re)), bf16_to_f32(f32_to_bf16_rne(v.im)));
  } else {
    return v;
  }
}

// ---------------------------------------------------------------------------
// wave64 + LDS block reduction of a double, fixed order (deterministic)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void block_sum_to(double v, double* out_slot) {
  __shared__ double wsum[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  if (lane == 0) wsum[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += wsum[i];
    *out_slot = t;
  }
}

// ---------------------------------------------------------------------------
// One site of the Wilson hopping sum H psi (eq.(wilson) without the -1/2):
//   H psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu),
// in the chiral basis with the two-spinor projection: for each direction the
// upper spins carry v = U h (or U^dag h) of the projected h, the lower spins a
// fixed +-1/+-i recombination of v.
template <typename S>
__device__ __forceinline__ void hop_site(const typename S::elem* __restrict__ in,
                                         const typename S::elem* __restrict__ links,
                                         const int* __restrict__ nbr, int p, unsigned site,
                                         unsigned s, unsigned Vh, cpx<RealOf<S>> acc[12]) {
  using R = RealOf<S>;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = cmk<R>(0, 0);
  const unsigned plane = 12u * Vh;
  const typename S::elem* ins = in + size_t(s) * plane;
  // the direction loop stays rolled: unrolled, the scheduler hoists all eight gathers
  // (8 x 12 spinor + 8 x 9 link complex numbers) and the kernel spills in FP64
#pragma unroll 1
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    const unsigned nb = (unsigned)nbr[(p * 8 + dir) * Vh + site];
    cpx<R> ps[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int co = 0; co < 3; ++co) ps[sp][co] = ld<S>(ins, (sp * 3 + co) * Vh + nb);
    // projection h = psi_u -+ A psi_l
    cpx<R> h[2][3];
#pragma unroll
    for (int co = 0; co < 3; ++co) {
      const cpx<R> p0 = ps[0][co], p1 = ps[1][co], p2 = ps[2][co], p3 = ps[3][co];
      if (mu == 0) {
        h[0][co] = fwd ? p0 + mul_i(p3) : p0 - mul_i(p3);
        h[1][co] = fwd ? p1 + mul_i(p2) : p1 - mul_i(p2);
      } else if (mu == 1) {
        h[0][co] = fwd ? p0 + p3 : p0 - p3;
        h[1][co] = fwd ? p1 - p2 : p1 + p2;
      } else if (mu == 2) {
        h[0][co] = fwd ? p0 + mul_i(p2) : p0 - mul_i(p2);
        h[1][co] = fwd ? p1 - mul_i(p3) : p1 + mul_i(p3);
      } else {
        h[0][co] = fwd ? p0 - p2 : p0 + p2;
        h[1][co] = fwd ? p1 - p3 : p1 + p3;
      }
    }
    // link: U_mu(x) from this parity, or U_mu(x-mu) from the other parity
    const unsigned lsite = fwd ? site : nb;
    const int lpar = fwd ? p : 1 - p;
    const typename S::elem* L = links + size_t((lpar * 4 + mu) * 9) * Vh;
    cpx<R> u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = ld<S>(L, k * Vh + lsite);
    cpx<R> v[2][3];
#pragma unroll
    for (int hs = 0; hs < 2; ++hs)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cpx<R> t = cmk<R>(0, 0);
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          if (fwd) cmac(t, u[a * 3 + bb], h[hs][bb]);        // (U h)_a
          else cmac_conj(t, u[bb * 3 + a], h[hs][bb]);       // (U^dag h)_a
        }
        v[hs][a] = t;
      }
    // reconstruct: upper spins += v; lower spins += fixed recombination of v
#pragma unroll
    for (int co = 0; co < 3; ++co) {
      acc[0 * 3 + co] = acc[0 * 3 + co] + v[0][co];
      acc[1 * 3 + co] = acc[1 * 3 + co] + v[1][co];
      cpx<R> l0, l1;
      if (mu == 0) {
        l0 = fwd ? mul_mi(v[1][co]) : mul_i(v[1][co]);
        l1 = fwd ? mul_mi(v[0][co]) : mul_i(v[0][co]);
      } else if (mu == 1) {
        l0 = fwd ? cmk<R>(-v[1][co].re, -v[1][co].im) : v[1][co];
        l1 = fwd ? v[0][co] : cmk<R>(-v[0][co].re, -v[0][co].im);
      } else if (mu == 2) {
        l0 = fwd ? mul_mi(v[0][co]) : mul_i(v[0][co]);
        l1 = fwd ? mul_i(v[1][co]) : mul_mi(v[1][co]);
      } else {
        l0 = fwd ? cmk<R>(-v[0][co].re, -v[0][co].im) : v[0][co];
        l1 = fwd ? cmk<R>(-v[1][co].re, -v[1][co].im) : v[1][co];
      }
      acc[2 * 3 + co] = acc[2 * 3 + co] + l0;
      acc[3 * 3 + co] = acc[3 * 3 + co] + l1;
    }
  }
}

struct HopDev {
  const void* in;
  void* out;
  const void* pre;
  const void* post;
  const void* links;
  const int* nbr;
  const void* mix;  // [2][Ls][Ls] real of the compute precision, or null
  double* partials;
  double hop_coef, pre_coef, post_coef;
  int parity_out;
  int nslices;
  unsigned Vh;
};

// Hop without a fifth-dimension mix: one thread per (site, slice).
template <typename S>
__global__ void __launch_bounds__(128) hop_plain_kernel(HopDev a) {
  using R = RealOf<S>;
  using E = typename S::elem;
  const unsigned site = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned s = blockIdx.y;
  double nrm = 0.0;
  if (site < a.Vh) {
    cpx<R> acc[12];
    hop_site<S>((const E*)a.in, (const E*)a.links, a.nbr, a.parity_out, site, s, a.Vh, acc);
    const size_t base = size_t(s) * 12 * a.Vh + site;
    const R hc = (R)a.hop_coef, pc = (R)a.pre_coef, qc = (R)a.post_coef;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      cpx<R> o = hc * acc[k];
      if (a.pre) o = o + pc * ld<S>((const E*)a.pre, base + size_t(k) * a.Vh);
      if (a.post) o = o + qc * ld<S>((const E*)a.post, base + size_t(k) * a.Vh);
      st<S>((E*)a.out, base + size_t(k) * a.Vh, o);
      nrm += (double)norm2(o);
    }
  }
  if (a.partials) block_sum_to(nrm, &a.partials[blockIdx.y * gridDim.x + blockIdx.x]);
}

// Hop followed by a dense fifth-dimension mix.  Phase 1: thread (site, s) computes
// h' = hop_coef * H in + pre_coef * pre and stores it in LDS as [s][comp][site].
// Phase 2: thread (site, comp) holds all Ls values of one component in registers,
// applies the per-chirality Ls x Ls matrix, adds post_coef * post and writes out.
template <typename S, int NS, int LSMAX>
__global__ void __launch_bounds__(NS* LSMAX) hop_mix_kernel(HopDev a) {
  using R = RealOf<S>;
  using E = typename S::elem;
  extern __shared__ char smem_raw[];
  cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
  const int Ls = a.nslices;
  const unsigned site0 = blockIdx.x * NS;
  {
    const int sl = threadIdx.x % NS, s = threadIdx.x / NS;
    const unsigned site = site0 + sl;
    if (s < Ls) {
      cpx<R> acc[12];
      if (site < a.Vh) {
        hop_site<S>((const E*)a.in, (const E*)a.links, a.nbr, a.parity_out, site, s, a.Vh, acc);
        const R hc = (R)a.hop_coef, pc = (R)a.pre_coef;
        const size_t base = size_t(s) * 12 * a.Vh + site;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          cpx<R> o = hc * acc[k];
          if (a.pre) o = o + pc * ld<S>((const E*)a.pre, base + size_t(k) * a.Vh);
          acc[k] = o;
        }
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cmk<R>(0, 0);
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) lds[(s * 12 + k) * NS + sl] = acc[k];
    }
  }
  __syncthreads();
  double nrm = 0.0;
  const R* M = (const R*)a.mix;
  const R qc = (R)a.post_coef;
  for (int t = threadIdx.x; t < NS * 12; t += blockDim.x) {
    const int sl = t % NS, comp = t / NS, ch = comp / 6;
    const unsigned site = site0 + sl;
    if (site >= a.Vh) continue;
    cpx<R> v[LSMAX];
#pragma unroll
    for (int j = 0; j < LSMAX; ++j)
      if (j < Ls) v[j] = lds[(j * 12 + comp) * NS + sl];
    const R* Mc = M + size_t(ch) * Ls * Ls;
#pragma unroll
    for (int i = 0; i < LSMAX; ++i) {
      if (i < Ls) {
      cpx<R> o = cmk<R>(0, 0);
#pragma unroll
      for (int j = 0; j < LSMAX; ++j)
        if (j < Ls) {
          const R mij = Mc[i * Ls + j];
          o.re = fma(mij, v[j].re, o.re);
          o.im = fma(mij, v[j].im, o.im);
        }
      const size_t idx = (size_t(i) * 12 + comp) * a.Vh + site;
      if (a.post) o = o + qc * ld<S>((const E*)a.post, idx);
      st<S>((E*)a.out, idx, o);
      nrm += (double)norm2(o);
      }
    }
  }
  if (a.partials) block_sum_to(nrm, &a.partials[blockIdx.x]);
}

// Site-local mix: out[s] = sum_s' M[ch][s][s'] in[s'] (+ post_coef * post[s]).
template <typename S, int LSMAX>
__global__ void __launch_bounds__(256) smix_kernel(typename S::elem* __restrict__ out,
                                                   const typename S::elem* __restrict__ in,
                                                   const typename S::elem* __restrict__ post,
                                                   double post_coef, const RealOf<S>* __restrict__ M,
                                                   int Ls, unsigned Vh, double* partials) {
  using R = RealOf<S>;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  double nrm = 0.0;
  if (t < 12u * Vh) {
    const unsigned comp = t / Vh, site = t % Vh, ch = comp / 6;
    cpx<R> v[LSMAX];
#pragma unroll
    for (int j = 0; j < LSMAX; ++j)
      if (j < Ls) v[j] = ld<S>(in, (size_t(j) * 12 + comp) * Vh + site);
    const R* Mc = M + size_t(ch) * Ls * Ls;
#pragma unroll
    for (int i = 0; i < LSMAX; ++i) {
      if (i < Ls) {
      cpx<R> o = cmk<R>(0, 0);
#pragma unroll
      for (int j = 0; j < LSMAX; ++j)
        if (j < Ls) {
          const R mij = Mc[i * Ls + j];
          o.re = fma(mij, v[j].re, o.re);
          o.im = fma(mij, v[j].im, o.im);
        }
      const size_t idx = (size_t(i) * 12 + comp) * Vh + site;
      if (post) o = o + (R)post_coef * ld<S>(post, idx);
      st<S>(out, idx, o);
      nrm += (double)norm2(o);
      }
    }
  }
  if (partials) block_sum_to(nrm, &partials[blockIdx.x]);
}

// CGLS update 1: x += a p ; r -= a q ; |r|^2 ; w = (g5 I^-T G^-1) r
template <typename S, int LSMAX>
__global__ void __launch_bounds__(256) cg_update1_kernel(typename S::elem* __restrict__ x,
                                                         typename S::elem* __restrict__ r,
                                                         typename S::elem* __restrict__ w,
                                                         const typename S::elem* __restrict__ p,
                                                         const typename S::elem* __restrict__ q,
                                                         const DevScalars* __restrict__ sc,
                                                         const RealOf<S>* __restrict__ M, int Ls,
                                                         unsigned Vh, double* partials) {
  using R = RealOf<S>;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  double nrm = 0.0;
  if (t < 12u * Vh) {
    const R a = (R)sc->a;
    const unsigned comp = t / Vh, site = t % Vh, ch = comp / 6;
    cpx<R> rv[LSMAX];
#pragma unroll
    for (int j = 0; j < LSMAX; ++j)
      if (j < Ls) {
        const size_t idx = (size_t(j) * 12 + comp) * Vh + site;
        cpx<R> xv = ld<S>(x, idx), pv = ld<S>(p, idx), qv = ld<S>(q, idx), rr = ld<S>(r, idx);
        xv = xv + a * pv;
        rr = rr - a * qv;
        st<S>(x, idx, xv);
        st<S>(r, idx, rr);
        rv[j] = as_stored<S>(rr);  // premix the value as stored
        nrm += (double)norm2(rv[j]);
      }
    const R* Mc = M + size_t(ch) * Ls * Ls;
#pragma unroll
    for (int i = 0; i < LSMAX; ++i) {
      if (i < Ls) {
      cpx<R> o = cmk<R>(0, 0);
#pragma unroll
      for (int j = 0; j < LSMAX; ++j)
        if (j < Ls) {
          const R mij = Mc[i * Ls + j];
          o.re = fma(mij, rv[j].re, o.re);
          o.im = fma(mij, rv[j].im, o.im);
        }
      st<S>(w, (size_t(i) * 12 + comp) * Vh + site, o);
      }
    }
  }
  if (partials) block_sum_to(nrm, &partials[blockIdx.x]);
}

// CGLS update 2: p = z + beta p ; u = (B G) p
template <typename S, int LSMAX>
__global__ void __launch_bounds__(256) cg_update2_kernel(typename S::elem* __restrict__ p,
                                                         typename S::elem* __restrict__ u,
                                                         const typename S::elem* __restrict__ z,
                                                         const DevScalars* __restrict__ sc,
                                                         const RealOf<S>* __restrict__ M, int Ls,
                                                         unsigned Vh) {
  using R = RealOf<S>;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12u * Vh) return;
  const R beta = (R)sc->beta;
  const unsigned comp = t / Vh, site = t % Vh, ch = comp / 6;
  cpx<R> pv[LSMAX];
#pragma unroll
  for (int j = 0; j < LSMAX; ++j)
    if (j < Ls) {
      const size_t idx = (size_t(j) * 12 + comp) * Vh + site;
      cpx<R> v = ld<S>(z, idx) + beta * ld<S>(p, idx);
      st<S>(p, idx, v);
      pv[j] = as_stored<S>(v);
    }
  const R* Mc = M + size_t(ch) * Ls * Ls;
#pragma unroll
  for (int i = 0; i < LSMAX; ++i) {
    if (i < Ls) {
    cpx<R> o = cmk<R>(0, 0);
#pragma unroll
    for (int j = 0; j < LSMAX; ++j)
      if (j < Ls) {
        const R mij = Mc[i * Ls + j];
        o.re = fma(mij, pv[j].re, o.re);
        o.im = fma(mij, pv[j].im, o.im);
      }
    st<S>(u, (size_t(i) * 12 + comp) * Vh + site, o);
    }
  }
}

__device__ double sum_partials_block(const double* part, int n) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  __shared__ double res;
  block_sum_to(v, &res);
  __syncthreads();
  return res;
}

// which: 0 -> qq, a = gamma/qq ; 1 -> zz (bank a), rr (bank b), beta, gamma ;
//        2 -> init: gamma = sum(a), rr = b2 = sum(b) ; 3 -> aux = sum(a) ; 4 -> rr = sum(a)
__global__ void __launch_bounds__(RED_THREADS) cg_finalize_kernel(DevScalars* s, int which,
                                                                   const double* pa, int na,
                                                                   const double* pb, int nb) {
  const double A = sum_partials_block(pa, na);
  const double B = (pb != nullptr) ? sum_partials_block(pb, nb) : 0.0;
  if (threadIdx.x != 0) return;
  if (which == 0) {
    s->qq = A;
    if (!(A > 0.0) || !isfinite(A)) {
      s->flags |= 1;
      s->a = 0.0;
    } else {
      s->a = s->gamma / A;
    }
  } else if (which == 1) {
    s->zz = A;
    s->rr = B;
    if (!isfinite(A) || !(s->gamma > 0.0)) {
      s->flags |= 2;
      s->beta = 0.0;
    } else {
      s->beta = A / s->gamma;
    }
    s->gamma = A;
  } else if (which == 2) {
    s->gamma = A;
    s->rr = B;
    s->b2 = B;
    s->flags = 0;
  } else if (which == 3) {
    s->aux = A;
  } else {
    s->rr = A;
  }
}

__global__ void __launch_bounds__(RED_THREADS) sum_partials_kernel(double* out, const double* pa,
                                                                    int na) {
  const double A = sum_partials_block(pa, na);
  if (threadIdx.x == 0) *out = A;
}

template <typename S>
__global__ void __launch_bounds__(256) norm2_kernel(const typename S::elem* __restrict__ x, size_t n,
                                                    double* partials) {
  double v = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    v += (double)norm2(ld<S>(x, i));
  block_sum_to(v, &partials[blockIdx.x]);
}

template <typename S>
__global__ void __launch_bounds__(256) axpby_kernel(typename S::elem* __restrict__ y, double a,
                                                    const typename S::elem* __restrict__ x, double b,
                                                    size_t n) {
  using R = RealOf<S>;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    cpx<R> o = (R)a * ld<S>(x, i);
    if (b != 0.0) o = o + (R)b * ld<S>(y, i);
    st<S>(y, i, o);
  }
}

template <typename SO, typename SI>
__global__ void __launch_bounds__(256) convert_kernel(typename SO::elem* __restrict__ out,
                                                      const typename SI::elem* __restrict__ in,
                                                      size_t n, double scale) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    cpx<RealOf<SI>> v = ld<SI>(in, i);
    // scale and round in FP64 / FP32 as the output needs
    cpx<RealOf<SO>> o = cmk<RealOf<SO>>((RealOf<SO>)(scale * (double)v.re),
                                        (RealOf<SO>)(scale * (double)v.im));
    st<SO>(out, i, o);
  }
}

template <typename S>
__global__ void __launch_bounds__(256) zero_kernel(typename S::elem* __restrict__ p, size_t n) {
  using R = RealOf<S>;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    st<S>(p, i, cmk<R>(0, 0));
}

// canonical complex128 [n][V][12] -> SoA [n][12][Vh] of one parity
template <typename S>
__global__ void __launch_bounds__(256) pack5_kernel(typename S::elem* __restrict__ dst,
                                                    const double2* __restrict__ src,
                                                    const int* __restrict__ cb2lex, int parity,
                                                    int nslices, unsigned Vh, unsigned V) {
  using R = RealOf<S>;
  const size_t n = size_t(nslices) * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    const size_t sc = t / Vh;
    const unsigned comp = sc % 12, s = sc / 12;
    const unsigned lex = (unsigned)cb2lex[parity * Vh + cb];
    const double2 v = src[(size_t(s) * V + lex) * 12 + comp];
    st<S>(dst, t, cmk<R>((R)v.x, (R)v.y));
  }
}

template <typename S>
__global__ void __launch_bounds__(256) unpack5_kernel(double2* __restrict__ dst,
                                                      const typename S::elem* __restrict__ src,
                                                      const int* __restrict__ cb2lex, int parity,
                                                      int nslices, unsigned Vh, unsigned V) {
  const size_t n = size_t(nslices) * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    const size_t sc = t / Vh;
    const unsigned comp = sc % 12, s = sc / 12;
    const unsigned lex = (unsigned)cb2lex[parity * Vh + cb];
    const auto v = ld<S>(src, t);
    dst[(size_t(s) * V + lex) * 12 + comp] = make_double2((double)v.re, (double)v.im);
  }
}

// canonical links [4][V][9] complex128 -> [p][mu][9][Vh], time phase folded
template <typename S>
__global__ void __launch_bounds__(256) pack_links_kernel(typename S::elem* __restrict__ dst,
                                                         const double2* __restrict__ src, int Lx,
                                                         int Ly, int Lz, int Lt, int apbc,
                                                         unsigned V) {
  using R = RealOf<S>;
  const unsigned Vh = V / 2;
  const size_t n = size_t(4) * V;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned lex = t % V, mu = t / V;
    unsigned r = lex;
    const unsigned x = r % Lx;
    r /= Lx;
    const unsigned y = r % Ly;
    r /= Ly;
    const unsigned z = r % Lz;
    const unsigned tt = r / Lz;
    const unsigned par = (x + y + z + tt) & 1u, cb = lex >> 1;
    const double sign = (apbc && mu == 3 && tt == (unsigned)(Lt - 1)) ? -1.0 : 1.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 v = src[(size_t(mu) * V + lex) * 9 + k];
      st<S>(dst, (size_t(par * 4 + mu) * 9 + k) * Vh + cb,
            cmk<R>((R)(sign * v.x), (R)(sign * v.y)));
    }
  }
}

// Source slices of rho = D_1(1) P (eta, 0, ...): only s = 0 and s = Ls-1 are non-zero,
//   chi_0 = (b_0 P- - c_0 P+) eta,  chi_L = (b_L P+ - c_L P-) eta,
//   rho_s = D_w chi_s + eta = (4 + M5) chi_s + eta - 1/2 H chi_s.
// This kernel writes chi (both parities, all slices) and aux = (4 + M5) chi + eta on
// the two wall slices; the hop adds -1/2 H chi afterwards.
__global__ void __launch_bounds__(256) source_kernel(double2* __restrict__ chi_b, double2* __restrict__ chi_r,
                                                     double2* __restrict__ aux_b, double2* __restrict__ aux_r,
                                                     const double2* __restrict__ eta,
                                                     const int* __restrict__ cb2lex, int Ls,
                                                     unsigned Vh, double M5, double b0, double c0,
                                                     double bL, double cL) {
  const size_t n = size_t(2) * Ls * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    size_t r = t / Vh;
    const unsigned comp = r % 12;
    r /= 12;
    const unsigned s = r % Ls;
    const unsigned par = r / Ls;
    const size_t idx = (size_t(s) * 12 + comp) * Vh + cb;
    double2* chi = par ? chi_r : chi_b;
    double2* aux = par ? aux_r : aux_b;
    const bool upper = comp < 6;  // spins 0,1: P+
    bool wall = false;
    double2 e = make_double2(0.0, 0.0);
    if (s == 0 || s == (unsigned)(Ls - 1)) {
      e = eta[size_t(cb2lex[par * Vh + cb]) * 12 + comp];
    }
    double f = 0.0;
    if (s == 0) {
      f = upper ? -c0 : b0;
      wall = true;
    } else if (s == (unsigned)(Ls - 1)) {
      f = upper ? bL : -cL;
      wall = true;
    }
    const double2 cv = make_double2(f * e.x, f * e.y);
    chi[idx] = cv;
    // rho_0 and rho_{Ls-1} each carry + eta
    const double ne = wall ? 1.0 : 0.0;
    aux[idx] = make_double2((4.0 + M5) * cv.x + ne * e.x, (4.0 + M5) * cv.y + ne * e.y);
  }
}

// y_1 = P- psi_0 + P+ psi_{Ls-1} (canonical output, all sites)
__global__ void __launch_bounds__(256) extract_kernel(double2* __restrict__ y1,
                                                      const double2* __restrict__ psi_b,
                                                      const double2* __restrict__ psi_r,
                                                      const int* __restrict__ cb2lex, int Ls,
                                                      unsigned Vh) {
  const size_t n = size_t(2) * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    const unsigned comp = (t / Vh) % 12;
    const unsigned par = t / (size_t(12) * Vh);
    const double2* psi = par ? psi_r : psi_b;
    const unsigned s = comp < 6 ? (unsigned)(Ls - 1) : 0u;
    y1[size_t(cb2lex[par * Vh + cb]) * 12 + comp] = psi[(size_t(s) * 12 + comp) * Vh + cb];
  }
}

__global__ void __launch_bounds__(256) check_finite_kernel(const double* __restrict__ v, size_t n,
                                                           int* flag) {
  int bad = 0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    if (!isfinite(v[i])) bad = 1;
  if (bad) atomicOr(flag, 1);
}

inline int grid_for(size_t n, int block, int cap = 65536) {
  size_t g = (n + block - 1) / block;
  if (g > (size_t)cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

inline int lsmax_for(int Ls) { return Ls <= 8 ? 8 : (Ls <= 16 ? 16 : 32); }

const void* mix_ptr(dwa_ctx* ctx, int prec, int kind) {
  const size_t off = size_t(kind) * 2 * ctx->Ls * ctx->Ls;
  if (prec == DWA_F64) return ctx->d_mix64 + off;
  return ctx->d_mix32 + off;
}

template <typename S>
int launch_hop_t(dwa_ctx* ctx, const HopOp& op, int* nblocks_out) {
  HopDev a;
  a.in = op.in;
  a.out = op.out;
  a.pre = op.pre;
  a.post = op.post;
  a.links = ctx->prec[S::prec].links;
  a.nbr = ctx->d_nbr;
  a.mix = op.mix == MIX_IDENTITY ? nullptr : mix_ptr(ctx, S::prec, op.mix);
  a.partials = op.partials;
  a.hop_coef = op.hop_coef;
  a.pre_coef = op.pre_coef;
  a.post_coef = op.post_coef;
  a.parity_out = op.parity_out;
  a.nslices = op.nslices;
  a.Vh = (unsigned)ctx->Vh;
  if (op.mix == MIX_IDENTITY) {
    dim3 grid((unsigned)((ctx->Vh + 127) / 128), (unsigned)op.nslices);
    hipLaunchKernelGGL(hop_plain_kernel<S>, grid, dim3(128), 0, ctx->stream, a);
    if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y);
  } else {
    const int Ls = op.nslices;
    const int lm = lsmax_for(Ls);
    const int NS = lm == 32 ? 8 : 16;  // keeps the LDS tile at <= 48 KB in FP64
    const unsigned grid = (unsigned)((ctx->Vh + NS - 1) / NS);
    const size_t shm = size_t(NS) * Ls * 12 * sizeof(cpx<RealOf<S>>);
    const dim3 block(NS * Ls);
    if (lm == 8)
      hipLaunchKernelGGL((hop_mix_kernel<S, 16, 8>), dim3(grid), block, shm, ctx->stream, a);
    else if (lm == 16)
      hipLaunchKernelGGL((hop_mix_kernel<S, 16, 16>), dim3(grid), block, shm, ctx->stream, a);
    else
      hipLaunchKernelGGL((hop_mix_kernel<S, 8, 32>), dim3(grid), block, shm, ctx->stream, a);
    if (nblocks_out) *nblocks_out = (int)grid;
  }
  return hip_fail(hipGetLastError(), "hop kernel launch");
}

template <typename S>
int launch_smix_t(dwa_ctx* ctx, int mix, void* out, const void* in, const void* post,
                  double post_coef, int nslices, double* partials, int* nblocks_out) {
  using E = typename S::elem;
  using R = RealOf<S>;
  const unsigned Vh = (unsigned)ctx->Vh;
  const int grid = (int)((12u * Vh + 255) / 256);
  const R* M = (const R*)mix_ptr(ctx, S::prec, mix);
  const int lm = lsmax_for(nslices);
  if (lm == 8)
    hipLaunchKernelGGL((smix_kernel<S, 8>), dim3(grid), dim3(256), 0, ctx->stream, (E*)out,
                       (const E*)in, (const E*)post, post_coef, M, nslices, Vh, partials);
  else if (lm == 16)
    hipLaunchKernelGGL((smix_kernel<S, 16>), dim3(grid), dim3(256), 0, ctx->stream, (E*)out,
                       (const E*)in, (const E*)post, post_coef, M, nslices, Vh, partials);
  else
    hipLaunchKernelGGL((smix_kernel<S, 32>), dim3(grid), dim3(256), 0, ctx->stream, (E*)out,
                       (const E*)in, (const E*)post, post_coef, M, nslices, Vh, partials);
  if (nblocks_out) *nblocks_out = grid;
  return hip_fail(hipGetLastError(), "smix kernel launch");
}

template <typename S>
int launch_update1_t(dwa_ctx* ctx, void* x, void* r, void* w, const void* p, const void* q,
                     const DevScalars* s, double* partials, int* nblocks) {
  using E = typename S::elem;
  using R = RealOf<S>;
  const unsigned Vh = (unsigned)ctx->Vh;
  const int grid = (int)((12u * Vh + 255) / 256);
  const R* M = (const R*)mix_ptr(ctx, S::prec, MIX_G5_IINVT_GINV);
  const int lm = lsmax_for(ctx->Ls);
#define DWA_U1(LM)                                                                            \
  hipLaunchKernelGGL((cg_update1_kernel<S, LM>), dim3(grid), dim3(256), 0, ctx->stream, (E*)x, \
                     (E*)r, (E*)w, (const E*)p, (const E*)q, s, M, ctx->Ls, Vh, partials)
  if (lm == 8)
    DWA_U1(8);
  else if (lm == 16)
    DWA_U1(16);
  else
    DWA_U1(32);
#undef DWA_U1
  if (nblocks) *nblocks = grid;
  return hip_fail(hipGetLastError(), "cg update1 launch");
}

template <typename S>
int launch_update2_t(dwa_ctx* ctx, void* p, void* u, const void* z, const DevScalars* s) {
  using E = typename S::elem;
  using R = RealOf<S>;
  const unsigned Vh = (unsigned)ctx->Vh;
  const int grid = (int)((12u * Vh + 255) / 256);
  const R* M = (const R*)mix_ptr(ctx, S::prec, MIX_BG);
  const int lm = lsmax_for(ctx->Ls);
#define DWA_U2(LM)                                                                            \
  hipLaunchKernelGGL((cg_update2_kernel<S, LM>), dim3(grid), dim3(256), 0, ctx->stream, (E*)p, \
                     (E*)u, (const E*)z, s, M, ctx->Ls, Vh)
  if (lm == 8)
    DWA_U2(8);
  else if (lm == 16)
    DWA_U2(16);
  else
    DWA_U2(32);
#undef DWA_U2
  return hip_fail(hipGetLastError(), "cg update2 launch");
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatch on precision

#define DWA_DISPATCH(prec, CALL)                    \
  switch (prec) {                                   \
    case DWA_F64: { using S_ = F64; return CALL; }  \
    case DWA_F32: { using S_ = F32; return CALL; }  \
    case DWA_BF16: { using S_ = BF16; return CALL; } \
    default: set_error("bad precision"); return DWA_EINVAL; \
  }

int launch_hop(dwa_ctx* ctx, int prec, const HopOp& op, int* nblocks_out) {
  DWA_DISPATCH(prec, launch_hop_t<S_>(ctx, op, nblocks_out));
}

int launch_smix(dwa_ctx* ctx, int prec, int mix, void* out, const void* in, const void* post,
                double post_coef, int nslices, double* partials, int* nblocks_out) {
  DWA_DISPATCH(prec, launch_smix_t<S_>(ctx, mix, out, in, post, post_coef, nslices, partials,
                                       nblocks_out));
}

int launch_cg_update1(dwa_ctx* ctx, int prec, void* x, void* r, void* w, const void* p,
                      const void* q, const DevScalars* s, double* partials, int* nblocks) {
  DWA_DISPATCH(prec, launch_update1_t<S_>(ctx, x, r, w, p, q, s, partials, nblocks));
}

int launch_cg_update2(dwa_ctx* ctx, int prec, void* p, void* u, const void* z,
                      const DevScalars* s) {
  DWA_DISPATCH(prec, launch_update2_t<S_>(ctx, p, u, z, s));
}

int launch_cg_finalize(dwa_ctx* ctx, int which, DevScalars* s, const double* pa, int na,
                       const double* pb, int nb) {
  hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(RED_THREADS), 0, ctx->stream, s, which, pa,
                     na, pb, nb);
  return hip_fail(hipGetLastError(), "finalize launch");
}

namespace {
template <typename S>
int norm2_t(dwa_ctx* ctx, const void* x, size_t n, double* partials, int* nblocks) {
  const int grid = grid_for(n, 256, 2048);
  hipLaunchKernelGGL(norm2_kernel<S>, dim3(grid), dim3(256), 0, ctx->stream,
                     (const typename S::elem*)x, n, partials);
  *nblocks = grid;
  return hip_fail(hipGetLastError(), "norm2 launch");
}
template <typename S>
int axpby_t(dwa_ctx* ctx, void* y, double a, const void* x, double b, size_t n) {
  hipLaunchKernelGGL(axpby_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename S::elem*)y, a, (const typename S::elem*)x, b, n);
  return hip_fail(hipGetLastError(), "axpby launch");
}
template <typename S>
int zero_t(dwa_ctx* ctx, void* p, size_t n) {
  hipLaunchKernelGGL(zero_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename S::elem*)p, n);
  return hip_fail(hipGetLastError(), "zero launch");
}
template <typename S>
int pack5_t(dwa_ctx* ctx, void* dst, const void* src, int parity, int nslices) {
  const size_t n = size_t(nslices) * 12 * ctx->Vh;
  hipLaunchKernelGGL(pack5_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename S::elem*)dst, (const double2*)src, ctx->d_cb2lex, parity, nslices,
                     (unsigned)ctx->Vh, (unsigned)ctx->V);
  return hip_fail(hipGetLastError(), "pack5 launch");
}
template <typename S>
int unpack5_t(dwa_ctx* ctx, void* dst, const void* src, int parity, int nslices) {
  const size_t n = size_t(nslices) * 12 * ctx->Vh;
  hipLaunchKernelGGL(unpack5_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)dst, (const typename S::elem*)src, ctx->d_cb2lex, parity, nslices,
                     (unsigned)ctx->Vh, (unsigned)ctx->V);
  return hip_fail(hipGetLastError(), "unpack5 launch");
}
template <typename S>
int pack_links_t(dwa_ctx* ctx, void* dst, const void* src) {
  const size_t n = size_t(4) * ctx->V;
  hipLaunchKernelGGL(pack_links_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename S::elem*)dst, (const double2*)src, ctx->dims[0], ctx->dims[1],
                     ctx->dims[2], ctx->dims[3], ctx->antiperiodic_t, (unsigned)ctx->V);
  return hip_fail(hipGetLastError(), "pack links launch");
}
template <typename SO, typename SI>
int convert_t2(dwa_ctx* ctx, void* out, const void* in, size_t n, double scale) {
  hipLaunchKernelGGL((convert_kernel<SO, SI>), dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename SO::elem*)out, (const typename SI::elem*)in, n, scale);
  return hip_fail(hipGetLastError(), "convert launch");
}
template <typename SO>
int convert_t1(dwa_ctx* ctx, void* out, int prec_in, const void* in, size_t n, double scale) {
  DWA_DISPATCH(prec_in, (convert_t2<SO, S_>(ctx, out, in, n, scale)));
}
}  // namespace

int launch_norm2(dwa_ctx* ctx, int prec, const void* x, size_t n, double* partials, int* nblocks) {
  DWA_DISPATCH(prec, norm2_t<S_>(ctx, x, n, partials, nblocks));
}
int launch_axpby(dwa_ctx* ctx, int prec, void* y, double a, const void* x, double b, size_t n) {
  DWA_DISPATCH(prec, axpby_t<S_>(ctx, y, a, x, b, n));
}
int launch_zero(dwa_ctx* ctx, int prec, void* p, size_t n) {
  DWA_DISPATCH(prec, zero_t<S_>(ctx, p, n));
}
int launch_pack5(dwa_ctx* ctx, int prec, void* dst, const void* src, int parity, int nslices) {
  DWA_DISPATCH(prec, pack5_t<S_>(ctx, dst, src, parity, nslices));
}
int launch_unpack5(dwa_ctx* ctx, int prec, void* dst, const void* src, int parity, int nslices) {
  DWA_DISPATCH(prec, unpack5_t<S_>(ctx, dst, src, parity, nslices));
}
int launch_pack_links(dwa_ctx* ctx, int prec, void* dst, const void* src) {
  DWA_DISPATCH(prec, pack_links_t<S_>(ctx, dst, src));
}
int launch_convert(dwa_ctx* ctx, int prec_out, void* out, int prec_in, const void* in, size_t n,
                   double scale) {
  DWA_DISPATCH(prec_out, convert_t1<S_>(ctx, out, prec_in, in, n, scale));
}

int launch_sum_partials(dwa_ctx* ctx, const double* partials, int n, double* out) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RED_THREADS), 0, ctx->stream, out,
                     partials, n);
  return hip_fail(hipGetLastError(), "sum partials launch");
}

int launch_source(dwa_ctx* ctx, void* chi_b, void* chi_r, void* aux_b, void* aux_r,
                  const void* eta) {
  const int Ls = ctx->Ls;
  const size_t n = size_t(2) * Ls * 12 * ctx->Vh;
  hipLaunchKernelGGL(source_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)chi_b, (double2*)chi_r, (double2*)aux_b, (double2*)aux_r,
                     (const double2*)eta, ctx->d_cb2lex, Ls, (unsigned)ctx->Vh, ctx->M5, ctx->b[0],
                     ctx->c[0], ctx->b[Ls - 1], ctx->c[Ls - 1]);
  return hip_fail(hipGetLastError(), "source launch");
}

int launch_extract(dwa_ctx* ctx, void* y1, const void* psi_b, const void* psi_r) {
  const size_t n = size_t(2) * 12 * ctx->Vh;
  hipLaunchKernelGGL(extract_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)y1, (const double2*)psi_b, (const double2*)psi_r, ctx->d_cb2lex,
                     ctx->Ls, (unsigned)ctx->Vh);
  return hip_fail(hipGetLastError(), "extract launch");
}

int launch_check_finite(dwa_ctx* ctx, const void* canon, size_t ncomplex, int* d_flag) {
  const size_t n = 2 * ncomplex;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, ctx->stream,
                     (const double*)canon, n, d_flag);
  return hip_fail(hipGetLastError(), "check finite launch");
}

}  // namespace dwa
