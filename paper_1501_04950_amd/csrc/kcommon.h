// Device code of libdwa shared by the per-precision translation units
// (kernels_f64.hip, kernels_f32.hip, kernels_bf16.hip): kernel templates and their
// launchers.  Each unit instantiates the launchers for one storage precision.
//
// Field layout (one parity, "SoA"): element (s, comp, cb) of a 5D half field sits at
// (s * 12 + comp) * Vh + cb, comp = spin * 3 + colour, so a wavefront of consecutive
// checkerboard sites reads or writes one contiguous run per (s, comp).  Links of one
// precision are [parity][mu][row*3+col][cb] with the antiperiodic time phase folded in.
// nbr[p][dir][cb] is the checkerboard index (in the other parity) of the neighbour
// x + mu (dir = mu) or x - mu (dir = 4 + mu) of the output site cb of parity p.
#pragma once

#include <hip/hip_runtime.h>

#include "dwa_internal.h"
#include "kreduce.h"

namespace dwa {

template <typename S>
using RealOf = typename S::real;

// the value a complex number has after a store/load round trip in storage S
template <typename S>
__device__ __forceinline__ cpx<RealOf<S>> as_stored(cpx<RealOf<S>> v) {
  if constexpr (S::prec == DWA_BF16) {
    const uint32_t b = pack_bf16x2(v.re, v.im);
    return cmk<float>(__uint_as_float(b << 16), __uint_as_float(b & 0xffff0000u));
  } else {
    return v;
  }
}

// ---------------------------------------------------------------------------
// Raw buffer access to one half field.  The descriptor (base, size in bytes) sits in
// scalar registers; a load or store takes a 32-bit lane offset plus a wave-uniform
// scalar offset, so the twelve colour-spin components of a gather share one vector
// address and cost no vector arithmetic.  Fields are below 4 GiB (checked when a
// context is created); reads past the size return zero.
typedef unsigned dwa_v2u __attribute__((ext_vector_type(2)));
typedef unsigned dwa_v4u __attribute__((ext_vector_type(4)));
typedef float dwa_v2f __attribute__((ext_vector_type(2)));
typedef double dwa_v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
  // 0x00020000: the descriptor word 3 of gfx9 raw (untyped, stride 0) buffers
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename S>
__device__ __forceinline__ cpx<typename S::real> ldbuf(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                       unsigned soff) {
  if constexpr (S::prec == DWA_F64) {
    const dwa_v2d d = __builtin_bit_cast(dwa_v2d, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    return {d.x, d.y};
  } else if constexpr (S::prec == DWA_F32) {
    const dwa_v2f f = __builtin_bit_cast(dwa_v2f, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    return {f.x, f.y};
  } else {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
  }
}

// AUX: the cache-policy operand of the store (0, or kStoreNT for a non-temporal store)
constexpr int kStoreNT = 2;
template <typename S, int AUX = 0>
__device__ __forceinline__ void stbuf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                      cpx<typename S::real> v) {
  if constexpr (S::prec == DWA_F64) {
    // A store of more than 64 bits must not have its data registers rewritten by the
    // very next VALU instruction.  The compiler inserts that wait state only when the
    // store has no register scalar offset, yet gfx950 needs it either way (with an SGPR
    // soffset the imaginary half of the last store of a loop was seen overwritten by
    // the norm that followed it).  So the whole offset goes into the lane offset.
    const dwa_v2d d = {v.re, v.im};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(dwa_v4u, d), r, voff + soff, 0, AUX);
  } else if constexpr (S::prec == DWA_F32) {
    const dwa_v2f f = {v.re, v.im};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(dwa_v2u, f), r, voff, soff, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(pack_bf16x2(v.re, v.im), r, voff, soff, AUX);
  }
}

// Complex numbers in LDS as naturally aligned two-element vectors, so that an access
// is one ds_read/ds_write_b64 (b128 for doubles) whose 16-bit offset field reaches the
// whole tile.
template <typename R> struct LdsT;
template <> struct LdsT<float> { using type = dwa_v2f; };
template <> struct LdsT<double> { using type = dwa_v2d; };
template <typename R>
using lcpx = typename LdsT<R>::type;
template <typename R>
__device__ __forceinline__ lcpx<R> to_lds(cpx<R> v) {
  return lcpx<R>{v.re, v.im};
}
template <typename R>
__device__ __forceinline__ cpx<R> from_lds(lcpx<R> v) {
  return cmk<R>(v.x, v.y);
}

// Scalar-loadable view of a read-only table: the constant address space tells the
// compiler no store in the kernel can alias it, so wave-uniform reads become s_load.
template <typename R>
using cptr = const __attribute__((address_space(4))) R*;

template <typename R>
__device__ __forceinline__ cptr<R> as_const(const R* p) {
  return (cptr<R>)(p);
}

// Apply one row of a per-chirality fifth-dimension matrix: sum_j M[i][j] v[j]; the row
// is wave-uniform and read through scalar loads.
template <typename R, int LSM>
__device__ __forceinline__ cpx<R> mix_row_c(cptr<R> Mrow, const cpx<R>* v, int Ls) {
  cpx<R> o = cmk<R>(0, 0);
#pragma unroll
  for (int j = 0; j < LSM; ++j)
    if (j < Ls) {
      const R mij = Mrow[j];
      o.re = fma(mij, v[j].re, o.re);
      o.im = fma(mij, v[j].im, o.im);
    }
  return o;
}


// ---------------------------------------------------------------------------
// Site-local fifth-dimension operators as O(Ls) sweeps.  Each matrix kind is a fixed
// product of at most three factors per chirality (diagonal, cyclic bidiagonal, cyclic
// bidiagonal solve); the factor order is fixed here at compile time and the host
// (build_smatrices) writes the coefficients of each factor in the same order.  The
// coefficient rows are wave-uniform and come in through scalar loads.  v holds the Ls
// values of one colour-spin component.

template <typename R, int LSM>
__device__ __forceinline__ void stage_scale(cpx<R>* v, cptr<R> A, int Ls) {
#pragma unroll
  for (int s = 0; s < LSM; ++s)
    if (s < Ls) v[s] = A[s] * v[s];
}

// y_s = A_s x_s + B_s x_{s-1} (lower; y_0 takes B_0 x_{Ls-1}) or x_{s+1} (upper;
// y_{Ls-1} takes B_{Ls-1} x_0)
template <typename R, int LSM, bool LOWER>
__device__ __forceinline__ void stage_bidiag(cpx<R>* v, cptr<R> A, cptr<R> B, int Ls) {
  if constexpr (LOWER) {
    cpx<R> xl = v[0];
#pragma unroll
    for (int s = 0; s < LSM; ++s)
      if (s < Ls) xl = v[s];
#pragma unroll
    for (int s = LSM - 1; s >= 1; --s)
      if (s < Ls) {
        cpx<R> o = A[s] * v[s];
        o.re = fma(B[s], v[s - 1].re, o.re);
        o.im = fma(B[s], v[s - 1].im, o.im);
        v[s] = o;
      }
    cpx<R> o = A[0] * v[0];
    o.re = fma(B[0], xl.re, o.re);
    o.im = fma(B[0], xl.im, o.im);
    v[0] = o;
  } else {
    const cpx<R> x0 = v[0];
#pragma unroll
    for (int s = 0; s < LSM - 1; ++s)
      if (s + 1 < Ls) {
        cpx<R> o = A[s] * v[s];
        o.re = fma(B[s], v[s + 1].re, o.re);
        o.im = fma(B[s], v[s + 1].im, o.im);
        v[s] = o;
      }
#pragma unroll
    for (int s = 0; s < LSM; ++s)
      if (s == Ls - 1) {
        cpx<R> o = A[s] * v[s];
        o.re = fma(B[s], x0.re, o.re);
        o.im = fma(B[s], x0.im, o.im);
        v[s] = o;
      }
  }
}

// Solve with a cyclic bidiagonal matrix (A = 1/d, B = e/d, C = f, W = 1/(1 - f_end)):
// a sweep for the particular part, the closure value, and a correction pass.
template <typename R, int LSM, bool LOWER>
__device__ __forceinline__ void stage_solve(cpx<R>* v, cptr<R> A, cptr<R> B, cptr<R> C,
                                            int Ls) {
  const R W = A[3 * kLsPad];
  if constexpr (LOWER) {
    v[0] = A[0] * v[0];
#pragma unroll
    for (int s = 1; s < LSM; ++s)
      if (s < Ls) {
        cpx<R> o = A[s] * v[s];
        o.re = fma(-B[s], v[s - 1].re, o.re);
        o.im = fma(-B[s], v[s - 1].im, o.im);
        v[s] = o;
      }
    cpx<R> Y = cmk<R>(0, 0);
#pragma unroll
    for (int s = 0; s < LSM; ++s)
      if (s == Ls - 1) Y = W * v[s];
#pragma unroll
    for (int s = 0; s < LSM; ++s) {
      if (s < Ls - 1) {
        v[s].re = fma(C[s], Y.re, v[s].re);
        v[s].im = fma(C[s], Y.im, v[s].im);
      } else if (s == Ls - 1) {
        v[s] = Y;
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < LSM; ++s)
      if (s == Ls - 1) v[s] = A[s] * v[s];
#pragma unroll
    for (int s = LSM - 2; s >= 0; --s)
      if (s < Ls - 1) {
        cpx<R> o = A[s] * v[s];
        o.re = fma(-B[s], v[s + 1].re, o.re);
        o.im = fma(-B[s], v[s + 1].im, o.im);
        v[s] = o;
      }
    const cpx<R> Y = W * v[0];
    v[0] = Y;
#pragma unroll
    for (int s = 1; s < LSM; ++s)
      if (s < Ls) {
        v[s].re = fma(C[s], Y.re, v[s].re);
        v[s].im = fma(C[s], Y.im, v[s].im);
      }
  }
}

// Tables of one matrix kind in the compute precision R:
//   coef  [2][kMaxStages][4][kLsPad]   (chirality, stage, row A/B/C/W, slice)
//   dense [2][Ls][Ls]
struct MixTables {
  const void* coef;
  const void* dense;
};

// Apply matrix KIND of chirality CH (0 = P+, 1 = P-) to v.  For P+ the factors B and I_1
// are lower cyclic bidiagonal and their transposes upper; for P- the other way round.
template <typename R, int LSM, int KIND, int CH, bool DENSE>
__device__ __forceinline__ void apply_mix(cpx<R>* v, int Ls, const MixTables& T) {
  if constexpr (DENSE) {
    cptr<R> M = as_const((const R*)T.dense + (size_t)CH * Ls * Ls);
    cpx<R> y[LSM];
#pragma unroll
    for (int i = 0; i < LSM; ++i)
      if (i < Ls) y[i] = mix_row_c<R, LSM>(M + i * Ls, v, Ls);
#pragma unroll
    for (int i = 0; i < LSM; ++i)
      if (i < Ls) v[i] = y[i];
  } else {
    constexpr bool LOW = CH == 0;
    cptr<R> c0 = as_const((const R*)T.coef + (size_t)CH * kMaxStages * 4 * kLsPad);
    cptr<R> c1 = c0 + 4 * kLsPad;
    if constexpr (KIND == MIX_BG) {  // B G
      stage_scale<R, LSM>(v, c0, Ls);
      stage_bidiag<R, LSM, LOW>(v, c1, c1 + kLsPad, Ls);
    } else if constexpr (KIND == MIX_N) {  // B I_1^-1
      stage_solve<R, LSM, LOW>(v, c0, c0 + kLsPad, c0 + 2 * kLsPad, Ls);
      stage_bidiag<R, LSM, LOW>(v, c1, c1 + kLsPad, Ls);
    } else if constexpr (KIND == MIX_GINV_IINV) {  // G^-1 I_1^-1
      stage_solve<R, LSM, LOW>(v, c0, c0 + kLsPad, c0 + 2 * kLsPad, Ls);
      stage_scale<R, LSM>(v, c1, Ls);
    } else if constexpr (KIND == MIX_G5_IINVT_GINV) {  // g5 I_1^-T G^-1
      stage_scale<R, LSM>(v, c0, Ls);
      stage_solve<R, LSM, !LOW>(v, c1, c1 + kLsPad, c1 + 2 * kLsPad, Ls);
    } else if constexpr (KIND == MIX_NT) {  // I_1^-T B^T
      stage_bidiag<R, LSM, !LOW>(v, c0, c0 + kLsPad, Ls);
      stage_solve<R, LSM, !LOW>(v, c1, c1 + kLsPad, c1 + 2 * kLsPad, Ls);
    } else if constexpr (KIND == MIX_G_BT_G5) {  // G B^T g5
      stage_bidiag<R, LSM, !LOW>(v, c0, c0 + kLsPad, Ls);
      stage_scale<R, LSM>(v, c1, Ls);
    }
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
  unsigned nbs[8];
#pragma unroll
  for (int dir = 0; dir < 8; ++dir) nbs[dir] = (unsigned)nbr[(p * 8 + dir) * Vh + site];
  // the direction loop stays rolled: unrolled, the scheduler hoists all eight gathers
  // (8 x 12 spinor + 8 x 9 link complex numbers) and the kernel spills in FP64
#pragma unroll 1
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    const unsigned nb = nbs[dir];
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
  MixTables mix;      // tables of the output fifth-dimension matrix
  const int* blkmap;  // block -> chunk of NS sites, or null for the identity
  double* partials;
  double hop_coef, pre_coef, post_coef;
  int parity_out;
  int nslices;
  unsigned Vh;
  unsigned nrhs;                 // fields in a batch (1 for a single field)
  unsigned nf;                   // fields per block (the block's links serve all of them)
  unsigned long long rhs_stride; // elements from one field of the batch to the next
};

// The fields of batch entry rhs (pointers moved by rhs * rhs_stride elements).
template <typename S>
__device__ __forceinline__ HopDev hop_for_rhs(const HopDev& a0, unsigned rhs) {
  using E = typename S::elem;
  HopDev a = a0;
  const size_t roff = size_t(rhs) * a0.rhs_stride;
  a.in = (const E*)a0.in + roff;
  a.out = (E*)a0.out + roff;
  if (a0.pre) a.pre = (const E*)a0.pre + roff;
  if (a0.post) a.post = (const E*)a0.post + roff;
  return a;
}

// Hop without a fifth-dimension mix: one thread per (site, slice).
template <typename S>
__global__ void __launch_bounds__(128) hop_plain_kernel(HopDev a0) {
  using R = RealOf<S>;
  using E = typename S::elem;
  const HopDev a = hop_for_rhs<S>(a0, blockIdx.z);
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
  if (a.partials)
    block_sum_to(nrm, &a.partials[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x]);
}

// Blocks are dealt to the 8 XCDs round robin; remap so that each XCD works on one
// contiguous range of checkerboard sites and its L2 sees the neighbours' reuse.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nblocks) {
  if (nblocks % 8u) return b;
  return (b % 8u) * (nblocks / 8u) + b / 8u;
}


// One site of H psi with the neighbour offsets and links of the block in LDS.  in is
// the input field's buffer descriptor, sboff the byte offset of this thread's slice,
// cstride = Vh * sizeof(elem) the byte stride between colour-spin components, and
// lnbr[dir * NS + sl] the neighbour's byte offset nb * sizeof(elem).  Every gather is
// (one lane offset per direction) + (scalar offset of the component).
template <typename S>
__device__ __forceinline__ void hop_site_lds(__amdgpu_buffer_rsrc_t in, unsigned sboff,
                                             unsigned cstride, const unsigned* lnbr,
                                             const lcpx<RealOf<S>>* llink, int sl, int NS,
                                             cpx<RealOf<S>> acc[12]) {
  using R = RealOf<S>;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = cmk<R>(0, 0);
  // fully unrolled: with the links in LDS only the spinor gathers are global loads,
  // and compile-time directions remove every branch on mu and on the hop sign
#pragma unroll
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    const unsigned off = sboff + lnbr[dir * NS + sl];
    cpx<R> ps[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int co = 0; co < 3; ++co) ps[sp][co] = ldbuf<S>(in, off, unsigned(sp * 3 + co) * cstride);
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
    cpx<R> u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = from_lds<R>(llink[(dir * 9 + k) * NS + sl]);
    cpx<R> v[2][3];
#pragma unroll
    for (int hs = 0; hs < 2; ++hs)
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) {
        cpx<R> t = cmk<R>(0, 0);
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          if (fwd) cmac(t, u[aa * 3 + bb], h[hs][bb]);
          else cmac_conj(t, u[bb * 3 + aa], h[hs][bb]);
        }
        v[hs][aa] = t;
      }
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

// LDS footprint of hop_mix_kernel in bytes.
template <typename R>
__host__ __device__ constexpr size_t hop_mix_lds_bytes(int NS, int Ls, int nf = 1) {
  return (nf > 1 ? size_t(Ls) * 12 * (NS + 1) * sizeof(cpx<R>) + size_t(72) * NS * sizeof(cpx<R>)
                 : (size_t(Ls) * 12 * (NS + 1) * sizeof(cpx<R>) > size_t(72) * NS * sizeof(cpx<R>)
                        ? size_t(Ls) * 12 * (NS + 1) * sizeof(cpx<R>)
                        : size_t(72) * NS * sizeof(cpx<R>))) +
         size_t(8) * NS * sizeof(unsigned);
}

// Cache policy of the fused hop's output stores.  FP64 and FP32 store non-temporally: at
// 16^3 x 32, L_s = 16 the input field, the links and the output of an FP64 hop (201 + 75
// + 201 MB) exceed the 256 MB Infinity Cache, and without the hint the output evicts the
// input lines that the gathers of the neighbouring sites read again.  Measured there:
// FP64 D_bb 478 -> 464 us (solve 466 -> 462 ms), FP32 D_bb 257 -> 248 us (FP32-inner solve
// 264.6 -> 258.2 ms); the BF16 solve, whose fields fit, got slower (138.3 -> 140.3 ms).
template <typename S>
__host__ __device__ constexpr int hop_store_aux() {
  return S::prec == DWA_BF16 ? 0 : kStoreNT;
}

// Phase 2 of hop_mix_kernel for one (site, component) of chirality CH: read the Ls
// values from the tile, apply the fifth-dimension matrix, add the post term, store.
template <typename S, int NS, int LSM, int MODE, int KIND, int CH, bool DENSE>
__device__ __forceinline__ double hop_mix_out(const HopDev& a, const lcpx<RealOf<S>>* tile,
                                              unsigned site0, int Ls, int lt) {
  using R = RealOf<S>;
  using E = typename S::elem;
  constexpr int NSP = NS + 1;
  const int sl = lt % NS, comp = CH * 6 + lt / NS;
  const unsigned site = site0 + sl;
  // the x term first, so its loads are in flight during the LDS reads and the mix
  cpx<R> pv[MODE == 1 ? LSM : 1];
  if constexpr (MODE == 1) {
    const unsigned sstride = 12u * a.Vh * unsigned(sizeof(E));
    const __amdgpu_buffer_rsrc_t rpost = make_rsrc(a.post, unsigned(Ls) * sstride);
    const unsigned off = (unsigned(comp) * a.Vh + site) * unsigned(sizeof(E));
    const bool ok = site < a.Vh;
#pragma unroll
    for (int i = 0; i < LSM; ++i)
      if (i < Ls) pv[i] = ok ? ldbuf<S>(rpost, off, unsigned(i) * sstride) : cmk<R>(0, 0);
  }
  cpx<R> v[LSM];
#pragma unroll
  for (int j = 0; j < LSM; ++j)
    if (j < Ls) v[j] = from_lds<R>(tile[(j * 12 + comp) * NSP + sl]);
  apply_mix<R, LSM, KIND, CH, DENSE>(v, Ls, a.mix);
  double nrm = 0.0;
  if (site < a.Vh) {
    const R qc = (R)a.post_coef;
    const unsigned sstride = 12u * a.Vh * unsigned(sizeof(E));  // bytes per slice
    const unsigned fbytes = unsigned(Ls) * sstride;
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(a.out, fbytes);
    const unsigned off = (unsigned(comp) * a.Vh + site) * unsigned(sizeof(E));
#pragma unroll
    for (int i = 0; i < LSM; ++i)
      if (i < Ls) {
        cpx<R> o = v[i];
        if constexpr (MODE == 1) o = o + qc * pv[i];
        stbuf<S, hop_store_aux<S>()>(rout, off, unsigned(i) * sstride, o);
        if constexpr (MODE == 1) nrm += (double)norm2(o);
      }
  }
  return nrm;
}

// Hop followed by a dense fifth-dimension mix, one block per NS checkerboard sites and
// all Ls slices.
//   Phase 0: the block stages the 8 neighbour indices and 72 link entries of its sites
//            in LDS (each link is read from HBM once per block, not once per slice).
//   Phase 1: thread (site, s) computes h' = hop_coef * H in (+ pre_coef * pre) and
//            writes it to an LDS tile [s][comp][site] (padded rows; it reuses the link
//            area once every thread is past the hop).
//   Phase 2: thread (site, colour-spin component) holds the Ls values of that component
//            of each chirality in turn in registers and applies the Ls x Ls matrix; the
//            chirality loop is uniform, so matrix rows come in through scalar loads.  With
//            enough threads the output rows are split into groups of whole wavefronts.
// The block order comes from a host-built table that walks each XCD's share of the
// lattice slab by slab, keeping the neighbours' reuse distance inside one XCD's L2.
// LS > 0: Ls is the compile-time LS; LS == 0: runtime Ls <= 32.  The block is NS * Ls
// threads rounded up to whole wavefronts (the bound below matches the launcher).
// MODE selects the epilogue at compile time so that each use is its own kernel:
//   0: out = M H in                 (first hop of D_bb / D_bb^dag)
//   1: out = M (hop_coef H in) + post_coef post   (second hop, with the x term; the
//      only epilogue that also writes per-block partial sums of |out|^2)
//   2: out = M (hop_coef H in + pre_coef pre)     (Schur prep and reconstruction)
template <typename S, int NS, int LS, int MODE, int KIND, bool DENSE, bool MULTI>
__global__ void __launch_bounds__((NS * (LS > 0 ? LS : 32) + 63) / 64 * 64) hop_mix_kernel(HopDev a0) {
  using R = RealOf<S>;
  using E = typename S::elem;
  // chunk of sites from the XCD-aware block order; fields blockIdx.y * nf ... of a batch.
  // MULTI (a0.nf > 1 fields per block) is a kernel of its own: with the field count
  // known to be one, the single-field kernel keeps its register budget.
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const unsigned nf = MULTI ? a0.nf : 1u;
  const HopDev a1 = hop_for_rhs<S>(a0, MULTI ? 0u : blockIdx.y);  // the field of a one-field block
  constexpr int LSM = LS > 0 ? LS : 32;
  constexpr int NSP = NS + 1;
  extern __shared__ __align__(16) char smem_raw[];
  const int Ls = LS > 0 ? LS : a0.nslices;
  // LDS: the output tile [Ls][12][NS+1]; the links [72][NS] share its space when the
  // block does one field and follow it when the block does several (they are re-used
  // by every field); then the neighbour offsets [8][NS].
  const size_t tile_b = size_t(Ls) * 12 * NSP * sizeof(cpx<R>), link_b = size_t(72) * NS * sizeof(cpx<R>);
  lcpx<R>* tile = reinterpret_cast<lcpx<R>*>(smem_raw);
  lcpx<R>* llink = reinterpret_cast<lcpx<R>*>(smem_raw + (MULTI ? tile_b : 0));
  unsigned* lnbr = reinterpret_cast<unsigned*>(smem_raw + (MULTI ? tile_b + link_b : (tile_b > link_b ? tile_b : link_b)));
  const unsigned site0 = (a0.blkmap ? (unsigned)a0.blkmap[blk] : blk) * NS;
  const int p = a0.parity_out;
  const unsigned Vh = a0.Vh;
  const unsigned cstride = Vh * unsigned(sizeof(E));  // bytes between components

  // phase 0: neighbour byte offsets, then links.  Thread (sl, j) stages rows j,
  // j + nthreads / NS, ... of site sl (NS is a power of two).
  const int sl1 = threadIdx.x % NS, j1 = threadIdx.x / NS;
  const int nj = blockDim.x / NS;
  const unsigned site1 = site0 + sl1;
  for (int dir = j1; dir < 8; dir += nj)
    lnbr[dir * NS + sl1] = site1 < Vh ? (unsigned)a0.nbr[(p * 8 + dir) * Vh + site1] * unsigned(sizeof(E)) : 0u;
  __syncthreads();
  {
    const E* L = (const E*)a0.links;
    for (int r = j1; r < 72; r += nj) {
      const int dir = r / 9, k = r - 9 * dir, mu = dir & 3;
      cpx<R> v = cmk<R>(0, 0);
      if (site1 < Vh) {
        const bool fwd = dir < 4;
        const unsigned lsite = fwd ? site1 : lnbr[dir * NS + sl1] / unsigned(sizeof(E));
        const int lpar = fwd ? p : 1 - p;
        v = ld<S>(L, ((lpar * 4 + mu) * 9 + k) * Vh + lsite);
      }
      llink[r * NS + sl1] = to_lds<R>(v);
    }
  }
  __syncthreads();

  const int s1 = j1;
  const bool act1 = s1 < Ls && site1 < Vh;
  constexpr int PH = ((NS * 6 + 63) / 64) * 64;
  // one field: hop into the tile, then the fifth-dimension mix and the stores
  auto field = [&](const HopDev& a, unsigned rhs) {
    // phase 1: hop, thread (site sl1, slice s1)
    cpx<R> acc[12];
    if (act1) {
      const unsigned sboff = unsigned(s1) * 12u * cstride;
      hop_site_lds<S>(make_rsrc(a.in, unsigned(Ls) * 12u * cstride), sboff, cstride, lnbr, llink, sl1, NS, acc);
      if (MODE != 0) {
        const R hc = (R)a.hop_coef, pc = (R)a.pre_coef;
        const unsigned off = sboff + site1 * unsigned(sizeof(E));
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          cpx<R> o = hc * acc[k];
          if (MODE == 2) o = o + pc * ldbuf<S>(make_rsrc(a.pre, unsigned(Ls) * 12u * cstride), off, unsigned(k) * cstride);
          acc[k] = o;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = cmk<R>(0, 0);
    }
    // every thread is done with the links (one field: they share the tile's space) and
    // with the previous field's tile
    __syncthreads();
    if (s1 < Ls) {
#pragma unroll
      for (int k = 0; k < 12; ++k) tile[(s1 * 12 + k) * NSP + sl1] = to_lds<R>(acc[k]);
    }
    __syncthreads();

    // phase 2: fifth-dimension mix.  Work items are (chirality, site, component of that
    // chirality); PH is a whole number of wavefronts and the block is launched in whole
    // wavefronts, so the chirality is the same on every lane of a wave and the branch on
    // it is uniform.
    double nrm = 0.0;
    for (int t = threadIdx.x; t < 2 * PH; t += blockDim.x) {
      const int ch = __builtin_amdgcn_readfirstlane(t / PH), lt = t % PH;
      if (lt >= NS * 6) continue;
      if (ch == 0)
        nrm += hop_mix_out<S, NS, LSM, MODE, KIND, 0, DENSE>(a, tile, site0, Ls, lt);
      else
        nrm += hop_mix_out<S, NS, LSM, MODE, KIND, 1, DENSE>(a, tile, site0, Ls, lt);
    }
    if (MODE == 1 && a.partials) block_sum_to(nrm, &a.partials[rhs * gridDim.x + blk]);
  };
  if constexpr (MULTI) {
    for (unsigned f = 0; f < nf; ++f) {
      const unsigned rhs = blockIdx.y * nf + f;
      if (rhs >= a0.nrhs) break;  // the same for the whole block
      field(hop_for_rhs<S>(a0, rhs), rhs);
    }
  } else {
    field(a1, blockIdx.y);
  }
}

// Site-local kernels run one thread per (site, colour-spin component of one chirality)
// and loop over the two chiralities, so the matrix rows are wave-uniform.
#define DWA_SITE_THREAD                                                       \
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;                   \
  const bool live = t < 6u * Vh;                                              \
  const unsigned c6 = live ? t / Vh : 0u, site = live ? t % Vh : 0u

// Site-local mix: out[s] = sum_s' M[ch][s][s'] in[s'] (+ post_coef * post[s]).
template <typename S, int LS, int KIND, bool DENSE>
__global__ void __launch_bounds__(256) smix_kernel(typename S::elem* __restrict__ out,
                                                   const typename S::elem* __restrict__ in,
                                                   const typename S::elem* __restrict__ post,
                                                   double post_coef, MixTables P, int Ls_rt,
                                                   unsigned Vh, double* partials) {
  using R = RealOf<S>;
  constexpr int LSM = LS > 0 ? LS : 32;
  const int Ls = LS > 0 ? LS : Ls_rt;
  DWA_SITE_THREAD;
  {  // batch entry blockIdx.y
    const size_t roff = size_t(blockIdx.y) * (size_t(Ls) * 12 * Vh);
    out += roff;
    in += roff;
    if (post) post += roff;
  }
  double nrm = 0.0;
  if (live) {
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const unsigned comp = ch * 6 + c6;
      cpx<R> v[LSM];
#pragma unroll
      for (int j = 0; j < LSM; ++j)
        if (j < Ls) v[j] = ld<S>(in, (size_t(j) * 12 + comp) * Vh + site);
      if (ch == 0) apply_mix<R, LSM, KIND, 0, DENSE>(v, Ls, P);
      else apply_mix<R, LSM, KIND, 1, DENSE>(v, Ls, P);
#pragma unroll
      for (int i = 0; i < LSM; ++i)
        if (i < Ls) {
          cpx<R> o = v[i];
          const size_t idx = (size_t(i) * 12 + comp) * Vh + site;
          if (post) o = o + (R)post_coef * ld<S>(post, idx);
          st<S>(out, idx, o);
          nrm += (double)norm2(o);
        }
    }
  }
  if (partials) block_sum_to(nrm, &partials[blockIdx.y * gridDim.x + blockIdx.x]);
}

// Streaming (non-temporal) access for data touched once per CG iteration: the solution
// accumulator (read and written by update 1 only) and the last read of q and z.  On
// MI355X the hint keeps such traffic from displacing, in L2 and the 256 MB Infinity
// Cache, the fields that the next kernels re-read (p, r, and the hop inputs and
// outputs, 50 MB each at BF16 on 16^3 x 32, L_s = 16).  Measured there: the BF16-inner
// solve 167.6 -> 156.1 ms.
template <typename S>
__device__ __forceinline__ cpx<typename S::real> ld_stream(const typename S::elem* p, size_t i) {
  if constexpr (S::prec == DWA_F64) {
    const dwa_v2d v = __builtin_nontemporal_load(reinterpret_cast<const dwa_v2d*>(p) + i);
    return {v.x, v.y};
  } else if constexpr (S::prec == DWA_F32) {
    const dwa_v2f v = __builtin_nontemporal_load(reinterpret_cast<const dwa_v2f*>(p) + i);
    return {v.x, v.y};
  } else {
    const unsigned v = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p) + i);
    return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
  }
}
template <typename S>
__device__ __forceinline__ void st_stream(typename S::elem* p, size_t i, cpx<typename S::real> v) {
  if constexpr (S::prec == DWA_F64) {
    __builtin_nontemporal_store(dwa_v2d{v.re, v.im}, reinterpret_cast<dwa_v2d*>(p) + i);
  } else if constexpr (S::prec == DWA_F32) {
    __builtin_nontemporal_store(dwa_v2f{v.re, v.im}, reinterpret_cast<dwa_v2f*>(p) + i);
  } else {
    __builtin_nontemporal_store(pack_bf16x2(v.re, v.im), reinterpret_cast<unsigned*>(p) + i);
  }
}

// CGLS update 1: x += a p ; r -= a q ; |r|^2 ; w = (g5 I^-T G^-1) r.
// With qparts (the nq block partials of |q|^2 per field), every block sums them itself
// in the finalize kernel's order and takes a = gamma / |q|^2, and block 0 stores qq, a
// and the breakdown flag for the host: the finalize launch between the second hop and
// this update is saved.  Otherwise a comes from the scalars.  With zparts as well (the
// nz partials of |z|^2 of the current z = A^dag r), gamma = |z|^2 is summed here too
// and block 0 stores it (update 2 of this step divides by it).
template <typename S, int LS, bool DENSE, int PK>
__global__ void __launch_bounds__(256) cg_update1_kernel(typename XAcc<S>::type::elem* __restrict__ x,
                                                         typename S::elem* __restrict__ r,
                                                         typename S::elem* __restrict__ w,
                                                         const typename S::elem* __restrict__ p,
                                                         const typename S::elem* __restrict__ q,
                                                         DevScalars* __restrict__ sc,
                                                         MixTables P, int Ls_rt, unsigned Vh,
                                                         double* partials,
                                                         const double* __restrict__ qparts, int nq,
                                                         const double* __restrict__ zparts, int nz) {
  using R = RealOf<S>;
  constexpr int LSM = LS > 0 ? LS : 32;
  const int Ls = LS > 0 ? LS : Ls_rt;
  DWA_SITE_THREAD;
  {  // batch entry blockIdx.y
    const size_t roff = size_t(blockIdx.y) * (size_t(Ls) * 12 * Vh);
    x += roff;
    r += roff;
    w += roff;
    p += roff;
    q += roff;
    sc += blockIdx.y;
  }
  double ad;
  if (qparts) {
    const double qq = sum_partials_block(qparts + size_t(blockIdx.y) * nq, nq);
    const double gamma = zparts ? sum_partials_block(zparts + size_t(blockIdx.y) * nz, nz) : sc->gamma;
    const bool bad = !(qq > 0.0) || !isfinite(qq);
    ad = (!sc->active || bad) ? 0.0 : gamma / qq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->qq = qq;
      sc->a = ad;
      if (zparts) sc->gamma = gamma;
      if (sc->active && bad) sc->flags |= 1;
    }
  } else {
    ad = sc->a;
  }
  double nrm = 0.0;
  if (live) {
    const R a = (R)ad;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const unsigned comp = ch * 6 + c6;
      cpx<R> rv[LSM];
#pragma unroll
      for (int j = 0; j < LSM; ++j)
        if (j < Ls) {
          const size_t idx = (size_t(j) * 12 + comp) * Vh + site;
          using SX = typename XAcc<S>::type;
          cpx<R> xv = ld_stream<SX>(x, idx), pv = ld<S>(p, idx), qv = ld_stream<S>(q, idx), rr = ld<S>(r, idx);
          xv = xv + a * pv;
          rr = rr - a * qv;
          st_stream<SX>(x, idx, xv);
          st<S>(r, idx, rr);
          rv[j] = as_stored<S>(rr);  // premix the value as stored
          nrm += (double)norm2(rv[j]);
        }
      if (ch == 0) apply_mix<R, LSM, PK, 0, DENSE>(rv, Ls, P);
      else apply_mix<R, LSM, PK, 1, DENSE>(rv, Ls, P);
#pragma unroll
      for (int i = 0; i < LSM; ++i)
        if (i < Ls) st<S>(w, (size_t(i) * 12 + comp) * Vh + site, rv[i]);
    }
  }
  if (partials) block_sum_to(nrm, &partials[blockIdx.y * gridDim.x + blockIdx.x]);
}

// CGLS update 2: p = z + beta p ; u = (B G) p.  With zparts (the nz partials of |z|^2
// per field) every block sums them itself, in the finalize kernel's order, and takes
// beta = |z|^2 / gamma; block 0 stores zz, beta and the breakdown flag.  gamma keeps
// the previous |z|^2 until the next update 1 replaces it.  Otherwise beta comes from
// the scalars.
template <typename S, int LS, bool DENSE, int PK>
__global__ void __launch_bounds__(256) cg_update2_kernel(typename S::elem* __restrict__ p,
                                                         typename S::elem* __restrict__ u,
                                                         const typename S::elem* __restrict__ z,
                                                         DevScalars* __restrict__ sc,
                                                         MixTables P, int Ls_rt, unsigned Vh,
                                                         const double* __restrict__ zparts, int nz) {
  using R = RealOf<S>;
  constexpr int LSM = LS > 0 ? LS : 32;
  const int Ls = LS > 0 ? LS : Ls_rt;
  DWA_SITE_THREAD;
  {  // batch entry blockIdx.y
    const size_t roff = size_t(blockIdx.y) * (size_t(Ls) * 12 * Vh);
    p += roff;
    u += roff;
    z += roff;
    sc += blockIdx.y;
  }
  double bd;
  if (zparts) {
    const double zz = sum_partials_block(zparts + size_t(blockIdx.y) * nz, nz);
    const bool bad = !isfinite(zz) || !(sc->gamma > 0.0);
    bd = (!sc->active || bad) ? 0.0 : zz / sc->gamma;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->zz = zz;
      sc->beta = bd;
      if (sc->active && bad) sc->flags |= 2;
    }
  } else {
    bd = sc->beta;
  }
  if (!live) return;
  const R beta = (R)bd;
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const unsigned comp = ch * 6 + c6;
    cpx<R> pv[LSM];
#pragma unroll
    for (int j = 0; j < LSM; ++j)
      if (j < Ls) {
        const size_t idx = (size_t(j) * 12 + comp) * Vh + site;
        cpx<R> v = ld_stream<S>(z, idx) + beta * ld<S>(p, idx);
        st<S>(p, idx, v);
        pv[j] = as_stored<S>(v);
      }
    if (ch == 0) apply_mix<R, LSM, PK, 0, DENSE>(pv, Ls, P);
    else apply_mix<R, LSM, PK, 1, DENSE>(pv, Ls, P);
#pragma unroll
    for (int i = 0; i < LSM; ++i)
      if (i < Ls) st<S>(u, (size_t(i) * 12 + comp) * Vh + site, pv[i]);
  }
}

template <typename S>
__global__ void __launch_bounds__(256) norm2_kernel(const typename S::elem* __restrict__ x, size_t n,
                                                    double* partials) {
  x += size_t(blockIdx.y) * n;  // batch entry
  double v = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x)
    v += (double)norm2(ld<S>(x, i));
  block_sum_to(v, &partials[blockIdx.y * gridDim.x + blockIdx.x]);
}

template <typename S>
__global__ void __launch_bounds__(256) axpby_kernel(typename S::elem* __restrict__ y, double a,
                                                    const typename S::elem* __restrict__ x, double b,
                                                    size_t n, const double* __restrict__ ab) {
  using R = RealOf<S>;
  // batch entry blockIdx.y, with its own (a, b) when a table is given
  y += size_t(blockIdx.y) * n;
  x += size_t(blockIdx.y) * n;
  if (ab) {
    a = ab[2 * blockIdx.y];
    b = ab[2 * blockIdx.y + 1];
  }
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
                                                      size_t n, double scale,
                                                      const double* __restrict__ scales) {
  // batch entry blockIdx.y, with its own scale when a table is given
  out += size_t(blockIdx.y) * n;
  in += size_t(blockIdx.y) * n;
  if (scales) scale = scales[blockIdx.y];
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
  p += size_t(blockIdx.y) * n;  // batch entry
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


// ---------------------------------------------------------------------------
// launchers of one storage precision S (explicitly instantiated once per precision)

inline int grid_for(size_t n, int block, int cap = 65536) {
  size_t g = (n + block - 1) / block;
  if (g > (size_t)cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename S>
MixTables mix_tables(dwa_ctx* ctx, int kind) {
  MixTables T;
  const size_t coff = size_t(kind) * 2 * kMaxStages * 4 * kLsPad;
  const size_t doff = size_t(kind) * 2 * ctx->Ls * ctx->Ls;
  if (S::prec == DWA_F64) {
    T.coef = ctx->d_sweep64 + coff;
    T.dense = ctx->d_mix64 + doff;
  } else {
    T.coef = ctx->d_sweep32 + coff;
    T.dense = ctx->d_mix32 + doff;
  }
  return T;
}

// Ls values with their own compiled site-local kernels; any other Ls <= 32 runs the
// generic one, which is also the only one compiled with the dense fallback.
#define DWA_LS_DISPATCH(Ls, dense, M) \
  if (dense) {                        \
    M(0, true);                       \
  } else {                            \
    switch (Ls) {                     \
      case 4: M(4, false); break;     \
      case 8: M(8, false); break;     \
      case 12: M(12, false); break;   \
      case 16: M(16, false); break;   \
      default: M(0, false); break;    \
    }                                 \
  }

// The fused hop for one tile size (sites per block).  Defined in khop.h and compiled in
// one translation unit per precision and tile, so that the tile variants build in
// parallel; mode is the epilogue (0, 1, 2) and mix the output matrix kind.
template <typename S, int NS>
int launch_hop_tile(dwa_ctx* ctx, const HopDev& a, int mode, int mix, dim3 grid, dim3 block,
                    size_t shm);

template <typename S>
int launch_hop_p(dwa_ctx* ctx, const HopOp& op, int* nblocks_out) {
  HopDev a;
  a.in = op.in;
  a.out = op.out;
  a.pre = op.pre;
  a.post = op.post;
  a.links = ctx->prec[S::prec].links;
  a.nbr = ctx->d_nbr;
  a.mix = mix_tables<S>(ctx, op.mix);
  a.partials = op.partials;
  const int NS = hop_sites_per_block(ctx, S::prec);
  a.blkmap = ctx->d_blkmap[ctx->tune[S::prec].order][tile_index(NS)];
  a.hop_coef = op.hop_coef;
  a.pre_coef = op.pre_coef;
  a.post_coef = op.post_coef;
  a.parity_out = op.parity_out;
  a.nslices = op.nslices;
  a.Vh = (unsigned)ctx->Vh;
  const unsigned nr = op.nrhs > 0 ? (unsigned)op.nrhs : 1u;
  a.nrhs = nr;
  a.rhs_stride = field_elems(ctx);
  // fields per block of the fused hop (a batch's blocks stage their links once for nf
  // fields)
  const unsigned nf_t = ctx->tune[S::prec].nf > 1 ? (unsigned)ctx->tune[S::prec].nf : 1u;
  const unsigned nf = nr > 1 ? (nf_t < nr ? nf_t : nr) : 1u;
  a.nf = nf;
  if (op.mix == MIX_IDENTITY) {
    dim3 grid((unsigned)((ctx->Vh + 127) / 128), (unsigned)op.nslices, nr);
    hipLaunchKernelGGL(hop_plain_kernel<S>, grid, dim3(128), 0, ctx->stream, a);
    if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y);
    return hip_fail(hipGetLastError(), "hop kernel launch");
  }
  const int Ls = op.nslices;
  if (Ls != ctx->Ls) {
    set_error("fused hop runs on the context's Ls slices");
    return DWA_EINVAL;
  }
  const unsigned chunks = (unsigned)((ctx->Vh + NS - 1) / NS);
  const dim3 grid(chunks, (nr + nf - 1) / nf);
  size_t shm = hop_mix_lds_bytes<RealOf<S>>(NS, Ls, int(nf));
  if (shm < ctx->hop_min_lds) shm = ctx->hop_min_lds;
  // whole wavefronts: phase 2 hands each wave one chirality, which needs the work
  // items of a wave to come from one 64-aligned range (the extra threads of the last
  // wave idle in phase 1)
  const dim3 block((NS * Ls + 63) / 64 * 64);
  const int mode = op.pre ? 2 : (op.post ? 1 : 0);
  if (op.pre && op.post) {
    set_error("hop with both pre and post terms is not supported");
    return DWA_EINVAL;
  }
  if (mode == 0 && op.hop_coef != 1.0) {
    set_error("plain fused hop takes hop_coef = 1");
    return DWA_EINVAL;
  }
  if (op.partials && mode != 1) {
    set_error("fused hop: output norms are computed only with a post term");
    return DWA_EINVAL;
  }
  if (shm > ctx->max_lds) {
    set_error("fused hop: the tile's LDS exceeds the device limit (choose a smaller tile)");
    return DWA_EINVAL;
  }
  int rc = DWA_EINVAL;
  switch (NS) {
    case 8: rc = launch_hop_tile<S, 8>(ctx, a, mode, op.mix, grid, block, shm); break;
    case 16: rc = launch_hop_tile<S, 16>(ctx, a, mode, op.mix, grid, block, shm); break;
    case 32: rc = launch_hop_tile<S, 32>(ctx, a, mode, op.mix, grid, block, shm); break;
    default: set_error("fused hop: no kernels for this tile size");
  }
  if (rc != DWA_OK) return rc;
  if (nblocks_out) *nblocks_out = (int)chunks;  // per field of the batch
  return hip_fail(hipGetLastError(), "hop kernel launch");
}

template <typename S, int KIND>
void launch_smix_k(dwa_ctx* ctx, void* out, const void* in, const void* post, double post_coef,
                   double* partials, int grid, int nrhs) {
  using E = typename S::elem;
  const MixTables T = mix_tables<S>(ctx, KIND);
  const unsigned Vh = (unsigned)ctx->Vh;
#define DWA_SMIX(LSV, DV)                                                                    \
  hipLaunchKernelGGL((smix_kernel<S, LSV, KIND, DV>), dim3(grid, nrhs), dim3(256), 0, ctx->stream, \
                     (E*)out, (const E*)in, (const E*)post, post_coef, T, ctx->Ls, Vh, partials)
  DWA_LS_DISPATCH(ctx->Ls, use_dense(ctx, S::prec), DWA_SMIX)
#undef DWA_SMIX
}

template <typename S>
int launch_smix_p(dwa_ctx* ctx, int mix, void* out, const void* in, const void* post,
                  double post_coef, int nslices, double* partials, int* nblocks_out, int nrhs) {
  if (nslices != ctx->Ls) {
    set_error("site-local mix runs on the context's Ls slices");
    return DWA_EINVAL;
  }
  const int grid = (int)((6u * (unsigned)ctx->Vh + 255) / 256);
  if (mix == MIX_I_ALPHA || mix == MIX_I_ALPHA_T || mix == MIX_W_I || mix == MIX_W_I_T) {
    // the site-local block I of D_alpha and its forms for eq.(redblack1): dense tables
    // (the kernel's dense path reads the table of the kind given), FP64 only
    if constexpr (S::prec == DWA_F64) {
      const MixTables T = mix_tables<S>(ctx, mix);
      hipLaunchKernelGGL((smix_kernel<S, 0, MIX_I_ALPHA, true>), dim3(grid, nrhs), dim3(256), 0,
                         ctx->stream, (double2*)out, (const double2*)in, (const double2*)post,
                         post_coef, T, ctx->Ls, (unsigned)ctx->Vh, partials);
      if (nblocks_out) *nblocks_out = grid;
      return hip_fail(hipGetLastError(), "smix kernel launch");
    }
    set_error("site-local I_1 G runs in FP64 only");
    return DWA_EINVAL;
  }
  if (mix == MIX_BG) launch_smix_k<S, MIX_BG>(ctx, out, in, post, post_coef, partials, grid, nrhs);
  else if (mix == MIX_N) launch_smix_k<S, MIX_N>(ctx, out, in, post, post_coef, partials, grid, nrhs);
  else if (mix == MIX_G5_IINVT_GINV)
    launch_smix_k<S, MIX_G5_IINVT_GINV>(ctx, out, in, post, post_coef, partials, grid, nrhs);
  else {
    set_error("site-local mix: unsupported matrix kind");
    return DWA_EINVAL;
  }
  if (nblocks_out) *nblocks_out = grid;
  return hip_fail(hipGetLastError(), "smix kernel launch");
}

template <typename S>
int launch_update1_p(dwa_ctx* ctx, void* x, void* r, void* w, const void* p, const void* q,
                     DevScalars* s, double* partials, int* nblocks, bool adj, int nrhs,
                     const double* qparts, int nq, const double* zparts, int nz) {
  using E = typename S::elem;
  using EX = typename XAcc<S>::type::elem;
  const unsigned Vh = (unsigned)ctx->Vh;
  const int grid = (int)((6u * Vh + 255) / 256);
  // w is the premixed input of the operator applied to r next: D_bb^dag (normal CGLS)
  // or, for CGLS on D_bb^dag, D_bb
  const MixTables T = mix_tables<S>(ctx, adj ? MIX_BG : MIX_G5_IINVT_GINV);
#define DWA_U1(LSV, DV)                                                                          \
  if (adj) {                                                                                     \
    hipLaunchKernelGGL((cg_update1_kernel<S, LSV, DV, MIX_BG>), dim3(grid, nrhs), dim3(256), 0,   \
                       ctx->stream, (EX*)x, (E*)r, (E*)w, (const E*)p, (const E*)q, s, T,         \
                       ctx->Ls, Vh, partials, qparts, nq, zparts, nz);                           \
  } else {                                                                                       \
    hipLaunchKernelGGL((cg_update1_kernel<S, LSV, DV, MIX_G5_IINVT_GINV>), dim3(grid, nrhs), dim3(256), \
                       0, ctx->stream, (EX*)x, (E*)r, (E*)w, (const E*)p, (const E*)q, s, T,      \
                       ctx->Ls, Vh, partials, qparts, nq, zparts, nz);                                                   \
  }
  DWA_LS_DISPATCH(ctx->Ls, use_dense(ctx, S::prec), DWA_U1)
#undef DWA_U1
  if (nblocks) *nblocks = grid;
  return hip_fail(hipGetLastError(), "cg update1 launch");
}

template <typename S>
int launch_update2_p(dwa_ctx* ctx, void* p, void* u, const void* z, DevScalars* s, bool adj,
                     int nrhs, const double* zparts, int nz) {
  using E = typename S::elem;
  const unsigned Vh = (unsigned)ctx->Vh;
  const int grid = (int)((6u * Vh + 255) / 256);
  // u is the premixed input of the operator applied to p next: D_bb (normal CGLS) or,
  // for CGLS on D_bb^dag, D_bb^dag
  const MixTables T = mix_tables<S>(ctx, adj ? MIX_G5_IINVT_GINV : MIX_BG);
#define DWA_U2(LSV, DV)                                                                        \
  if (adj) {                                                                                   \
    hipLaunchKernelGGL((cg_update2_kernel<S, LSV, DV, MIX_G5_IINVT_GINV>), dim3(grid, nrhs),     \
                       dim3(256), 0, ctx->stream, (E*)p, (E*)u, (const E*)z, s, T, ctx->Ls, Vh,   \
                       zparts, nz);                                                            \
  } else {                                                                                     \
    hipLaunchKernelGGL((cg_update2_kernel<S, LSV, DV, MIX_BG>), dim3(grid, nrhs), dim3(256), 0, \
                       ctx->stream, (E*)p, (E*)u, (const E*)z, s, T, ctx->Ls, Vh, zparts, nz);  \
  }
  DWA_LS_DISPATCH(ctx->Ls, use_dense(ctx, S::prec), DWA_U2)
#undef DWA_U2
  return hip_fail(hipGetLastError(), "cg update2 launch");
}

template <typename S>
int norm2_p(dwa_ctx* ctx, const void* x, size_t n, double* partials, int* nblocks, int nrhs) {
  const int grid = grid_for(n, 256, 2048);
  hipLaunchKernelGGL(norm2_kernel<S>, dim3(grid, nrhs), dim3(256), 0, ctx->stream,
                     (const typename S::elem*)x, n, partials);
  *nblocks = grid;
  return hip_fail(hipGetLastError(), "norm2 launch");
}
template <typename S>
int axpby_p(dwa_ctx* ctx, void* y, double a, const void* x, double b, size_t n, int nrhs,
            const double* ab) {
  hipLaunchKernelGGL(axpby_kernel<S>, dim3(grid_for(n, 256), nrhs), dim3(256), 0, ctx->stream,
                     (typename S::elem*)y, a, (const typename S::elem*)x, b, n, ab);
  return hip_fail(hipGetLastError(), "axpby launch");
}
template <typename S>
int zero_p(dwa_ctx* ctx, void* p, size_t n, int nrhs) {
  hipLaunchKernelGGL(zero_kernel<S>, dim3(grid_for(n, 256), nrhs), dim3(256), 0, ctx->stream,
                     (typename S::elem*)p, n);
  return hip_fail(hipGetLastError(), "zero launch");
}
template <typename S>
int pack5_p(dwa_ctx* ctx, void* dst, const void* src, int parity, int nslices) {
  const size_t n = size_t(nslices) * 12 * ctx->Vh;
  hipLaunchKernelGGL(pack5_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename S::elem*)dst, (const double2*)src, ctx->d_cb2lex, parity, nslices,
                     (unsigned)ctx->Vh, (unsigned)ctx->V);
  return hip_fail(hipGetLastError(), "pack5 launch");
}
template <typename S>
int unpack5_p(dwa_ctx* ctx, void* dst, const void* src, int parity, int nslices) {
  const size_t n = size_t(nslices) * 12 * ctx->Vh;
  hipLaunchKernelGGL(unpack5_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)dst, (const typename S::elem*)src, ctx->d_cb2lex, parity, nslices,
                     (unsigned)ctx->Vh, (unsigned)ctx->V);
  return hip_fail(hipGetLastError(), "unpack5 launch");
}
template <typename S>
int pack_links_p(dwa_ctx* ctx, void* dst, const void* src) {
  const size_t n = size_t(4) * ctx->V;
  hipLaunchKernelGGL(pack_links_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (typename S::elem*)dst, (const double2*)src, ctx->dims[0], ctx->dims[1],
                     ctx->dims[2], ctx->dims[3], ctx->antiperiodic_t, (unsigned)ctx->V);
  return hip_fail(hipGetLastError(), "pack links launch");
}
template <typename SO, typename SI>
int convert_p(dwa_ctx* ctx, void* out, const void* in, size_t n, double scale, int nrhs,
              const double* scales) {
  hipLaunchKernelGGL((convert_kernel<SO, SI>), dim3(grid_for(n, 256), nrhs), dim3(256), 0,
                     ctx->stream, (typename SO::elem*)out, (const typename SI::elem*)in, n, scale,
                     scales);
  return hip_fail(hipGetLastError(), "convert launch");
}

#define DWA_INSTANTIATE_PRECISION(S)                                                            \
  template int launch_hop_p<S>(dwa_ctx*, const HopOp&, int*);                                  \
  template int launch_smix_p<S>(dwa_ctx*, int, void*, const void*, const void*, double, int,    \
                                double*, int*, int);                                            \
  template int launch_update1_p<S>(dwa_ctx*, void*, void*, void*, const void*, const void*,     \
                                   DevScalars*, double*, int*, bool, int, const double*, int,   \
                                   const double*, int);                                         \
  template int launch_update2_p<S>(dwa_ctx*, void*, void*, const void*, DevScalars*, bool, int, \
                                   const double*, int);                                         \
  template int norm2_p<S>(dwa_ctx*, const void*, size_t, double*, int*, int);                   \
  template int axpby_p<S>(dwa_ctx*, void*, double, const void*, double, size_t, int,            \
                          const double*);                                                       \
  template int zero_p<S>(dwa_ctx*, void*, size_t, int);                                         \
  template int pack5_p<S>(dwa_ctx*, void*, const void*, int, int);                              \
  template int unpack5_p<S>(dwa_ctx*, void*, const void*, int, int);                            \
  template int pack_links_p<S>(dwa_ctx*, void*, const void*);                                   \
  template int convert_p<S, F64>(dwa_ctx*, void*, const void*, size_t, double, int, const double*); \
  template int convert_p<S, F32>(dwa_ctx*, void*, const void*, size_t, double, int, const double*); \
  template int convert_p<S, BF16>(dwa_ctx*, void*, const void*, size_t, double, int, const double*);

}  // namespace dwa
