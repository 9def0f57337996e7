// gfx950 kernels of the gradient (adjoint-state) path of libdwa, FP64.
//
// With psi the 5D solution of D_alpha(m) psi = rho = D_1(1) P b and lambda the
// solution of D_alpha(m)^dag lambda = f (f = E^dag eta', E the extraction of y_1),
// every first-order change of L = Re <eta', y_1> is Re <lambda, d rho - (d D_alpha) psi>.
// Using D_alpha = D_1 G and D_1 = D_w B + C (slice by slice, B and C real and
// chirality diagonal), the U-, b- and c-dependence sits in D_w B:
//   links  : dL = Re <lambda, d D_w phi>,        phi = B_1 P b - B G psi,
//   b_s    : dL/db_s = Re <lambda_s, (D_w (P b - G psi))_s>,
//   c_s    : dL/dc_s = Re <lambda_s, (D_w (T_1 P b - T_m G psi))_s>,
// with (T_m x)_s = P- x_{s+1} + P+ x_{s-1} and the walls closed by -m.  The adjoint
// field arrives as lt = g5 lambda (that is how the red-black adjoint solve delivers
// it), so the kernels multiply by g5 on load.  Fields are SoA half fields
// [s][12][Vh] (comp = spin*3 + colour, comps 0..5 are P+), canonical 4D fields
// [V][4][3], canonical links [mu][V][3][3].
#include <hip/hip_runtime.h>

#include "dwa_internal.h"

namespace dwa {

namespace {

using C = cpx<double>;

__device__ __forceinline__ C ld2(const double2* p, size_t i) {
  const double2 v = p[i];
  return cmk(v.x, v.y);
}
__device__ __forceinline__ C conjc(C a) { return cmk(a.re, -a.im); }
__device__ __forceinline__ C cmul(C a, C b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}

inline int grid_for(size_t n, int block, int cap = 65536) {
  size_t g = (n + block - 1) / block;
  if (g > (size_t)cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

// gamma_mu v in the chiral basis (gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
// gamma_t = [[0, 1], [1, 0]]); v[spin] is one colour component.
__device__ __forceinline__ void gamma_apply(int mu, const C v[4], C o[4]) {
  if (mu == 0) {
    o[0] = mul_mi(v[3]); o[1] = mul_mi(v[2]); o[2] = mul_i(v[1]); o[3] = mul_i(v[0]);
  } else if (mu == 1) {
    o[0] = -1.0 * v[3]; o[1] = v[2]; o[2] = v[1]; o[3] = -1.0 * v[0];
  } else if (mu == 2) {
    o[0] = mul_mi(v[2]); o[1] = mul_i(v[3]); o[2] = mul_i(v[0]); o[3] = mul_mi(v[1]);
  } else {
    o[0] = v[2]; o[1] = v[3]; o[2] = v[0]; o[3] = v[1];
  }
}

// f = E^dag eta': slice 0 holds P- eta', slice Ls-1 holds P+ eta', both parities.
__global__ void __launch_bounds__(256) adj_source_kernel(double2* __restrict__ f_b,
                                                         double2* __restrict__ f_r,
                                                         const double2* __restrict__ eta_p,
                                                         const int* __restrict__ cb2lex, int Ls,
                                                         unsigned Vh) {
  const size_t n = size_t(2) * Ls * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    size_t r = t / Vh;
    const unsigned comp = r % 12;
    r /= 12;
    const unsigned s = r % Ls;
    const unsigned par = r / Ls;
    const bool plus = comp < 6;
    double2 v = make_double2(0.0, 0.0);
    if ((s == 0 && !plus) || (s == unsigned(Ls - 1) && plus))
      v = eta_p[size_t(cb2lex[par * Vh + cb]) * 12 + comp];
    (par ? f_r : f_b)[(size_t(s) * 12 + comp) * Vh + cb] = v;
  }
}

// omega_b = P b - G psi and omega_c = T_1 P b - T_m G psi on one parity.
__global__ void __launch_bounds__(256) omega_kernel(double2* __restrict__ ob, double2* __restrict__ oc,
                                                    const double2* __restrict__ psi,
                                                    const double2* __restrict__ eta,
                                                    const int* __restrict__ cb2lex, int par, int Ls,
                                                    unsigned Vh, double alpha, double m) {
  const size_t n = size_t(Ls) * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    const unsigned comp = (t / Vh) % 12;
    const int s = int(t / (size_t(12) * Vh));
    const bool plus = comp < 6;
    const C e = ld2(eta, size_t(cb2lex[par * Vh + cb]) * 12 + comp);
    // G = diag(P- + alpha P+, alpha, ..., alpha, P+ + alpha P-)
    auto gpsi = [&](int j) {
      const double g = j == 0 ? (plus ? alpha : 1.0) : (j == Ls - 1 ? (plus ? 1.0 : alpha) : alpha);
      return g * ld2(psi, (size_t(j) * 12 + comp) * Vh + cb);
    };
    // P b: P- eta on slice 0, P+ eta on slice Ls-1
    auto pb = [&](int j) {
      return ((j == 0 && !plus) || (j == Ls - 1 && plus)) ? e : cmk(0.0, 0.0);
    };
    const C wb = pb(s) - gpsi(s);
    // T: P+ takes slice s-1, P- slice s+1; across the wall the factor is -m (m = 1 for rho)
    int j = plus ? s - 1 : s + 1;
    double fm = 1.0, f1 = 1.0;
    if (j < 0 || j >= Ls) {
      j = plus ? Ls - 1 : 0;
      fm = -m;
      f1 = -1.0;
    }
    const C wc = f1 * pb(j) - fm * gpsi(j);
    const size_t idx = (size_t(s) * 12 + comp) * Vh + cb;
    ob[idx] = make_double2(wb.re, wb.im);
    oc[idx] = make_double2(wc.re, wc.im);
  }
}

// J psi with J = d G / d alpha = diag(P+, 1, ..., 1, P-)
__global__ void __launch_bounds__(256) jpsi_kernel(double2* __restrict__ out,
                                                   const double2* __restrict__ psi, int Ls,
                                                   unsigned Vh) {
  const size_t n = size_t(Ls) * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned comp = (t / Vh) % 12;
    const int s = int(t / (size_t(12) * Vh));
    const bool plus = comp < 6;
    const bool zero = (s == 0 && !plus) || (s == Ls - 1 && plus);
    out[t] = zero ? make_double2(0.0, 0.0) : psi[t];
  }
}

// Per-slice partial sums of Re <a, b> (a multiplied by g5 when g5 != 0):
// partials[s * gridDim.x + blockIdx.x], slice s = blockIdx.y.
__global__ void __launch_bounds__(256) slice_dot_kernel(const double2* __restrict__ a,
                                                        const double2* __restrict__ b,
                                                        unsigned Vh, int g5, double* partials) {
  const unsigned s = blockIdx.y;
  const size_t n = size_t(12) * Vh;
  const size_t base = size_t(s) * n;
  double v = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    const double2 x = a[base + i], y = b[base + i];
    const double d = x.x * y.x + x.y * y.y;
    v += (g5 && (i / Vh) >= 6) ? -d : d;
  }
  __shared__ double wsum[4];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) partials[size_t(s) * gridDim.x + blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Link force: for the link U_mu(x) (x of parity par, y = x + mu),
//   g = -1/2 sum_s sum_spin [ ((1 - g_mu) lambda_s(x)) (x) conj(phi_s(y))
//                             + phi_s(x) (x) conj((1 + g_mu) lambda_s(y)) ]
// (colour outer products), times the boundary sign of the link, written to the
// canonical gradient array.
__global__ void __launch_bounds__(128) force_kernel(double2* __restrict__ gU,
                                                    const double2* __restrict__ lt_b,
                                                    const double2* __restrict__ lt_r,
                                                    const double2* __restrict__ ph_b,
                                                    const double2* __restrict__ ph_r,
                                                    const int* __restrict__ nbr,
                                                    const int* __restrict__ cb2lex, int Ls,
                                                    unsigned Vh, int Lxyz, int Lt, int antiperiodic) {
  const size_t nthreads = size_t(2) * 4 * Vh;
  const size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  if (t >= nthreads) return;
  const unsigned cb = t % Vh;
  const int mu = int((t / Vh) % 4);
  const int par = int(t / (size_t(4) * Vh));
  const unsigned cbn = (unsigned)nbr[(size_t(par) * 8 + mu) * Vh + cb];
  const double2* lx = par ? lt_r : lt_b;
  const double2* ly = par ? lt_b : lt_r;
  const double2* px = par ? ph_r : ph_b;
  const double2* py = par ? ph_b : ph_r;
  C g[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) g[k] = cmk(0.0, 0.0);
  for (int s = 0; s < Ls; ++s) {
    const size_t b0 = size_t(s) * 12 * Vh;
#pragma unroll
    for (int co = 0; co < 3; ++co) {
      // colour component co of the four spinors (lambda = g5 lt on load)
      C lam_x[4], lam_y[4], gx[4], gy[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const double sg = sp < 2 ? 1.0 : -1.0;
        lam_x[sp] = sg * ld2(lx, b0 + size_t(sp * 3 + co) * Vh + cb);
        lam_y[sp] = sg * ld2(ly, b0 + size_t(sp * 3 + co) * Vh + cbn);
      }
      gamma_apply(mu, lam_x, gx);
      gamma_apply(mu, lam_y, gy);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const C a = lam_x[sp] - gx[sp];  // ((1 - g_mu) lambda(x))_sp, colour co (row)
        const C bb = lam_y[sp] + gy[sp];  // ((1 + g_mu) lambda(y))_sp, colour co (column)
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2) {
          const C phy = ld2(py, b0 + size_t(sp * 3 + c2) * Vh + cbn);  // phi(y), column c2
          const C phx = ld2(px, b0 + size_t(sp * 3 + c2) * Vh + cb);   // phi(x), row c2
          g[co * 3 + c2] = g[co * 3 + c2] + cmul(a, conjc(phy));
          g[c2 * 3 + co] = g[c2 * 3 + co] + cmul(phx, conjc(bb));
        }
      }
    }
  }
  const int lex = cb2lex[par * Vh + cb];
  double sign = -0.5;
  if (antiperiodic && mu == 3 && lex / Lxyz == Lt - 1) sign = 0.5;
  double2* out = gU + (size_t(mu) * (2 * size_t(Vh)) + lex) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) out[k] = make_double2(sign * g[k].re, sign * g[k].im);
}

// Source gradient: the first slice of P^dag D_1(1)^dag lambda.  With u = D_w^dag lambda
// = g5 D_w lt and B_1, C_1 the m = 1 matrices, the P- half of slice 0 and the P+ half
// of slice Ls-1 of B_1^T u + C_1^T lambda are
//   P-: b_0 u_0 - c_{Ls-1} u_{Ls-1} + lambda_0 + lambda_{Ls-1},
//   P+: b_{Ls-1} u_{Ls-1} - c_0 u_0 + lambda_{Ls-1} + lambda_0.
// dw_b / dw_r hold D_w lt on the two wall slices (index 0: s = 0, index 1: s = Ls-1).
__global__ void __launch_bounds__(256) geta_kernel(double2* __restrict__ geta,
                                                   const double2* __restrict__ lt_b,
                                                   const double2* __restrict__ lt_r,
                                                   const double2* __restrict__ dw_b,
                                                   const double2* __restrict__ dw_r,
                                                   const int* __restrict__ cb2lex, int Ls,
                                                   unsigned Vh, double b0, double c0, double bL,
                                                   double cL) {
  const size_t n = size_t(2) * 12 * Vh;
  for (size_t t = blockIdx.x * size_t(blockDim.x) + threadIdx.x; t < n;
       t += size_t(gridDim.x) * blockDim.x) {
    const unsigned cb = t % Vh;
    const unsigned comp = (t / Vh) % 12;
    const unsigned par = t / (size_t(12) * Vh);
    const double2* lt = par ? lt_r : lt_b;
    const double2* dw = par ? dw_r : dw_b;
    const double sg = comp < 6 ? 1.0 : -1.0;  // g5 on this component
    const C l0 = sg * ld2(lt, size_t(comp) * Vh + cb);
    const C lL = sg * ld2(lt, (size_t(Ls - 1) * 12 + comp) * Vh + cb);
    const C u0 = sg * ld2(dw, size_t(comp) * Vh + cb);
    const C uL = sg * ld2(dw, (size_t(12) + comp) * Vh + cb);
    const C g = comp < 6 ? bL * uL - c0 * u0 + lL + l0 : b0 * u0 - cL * uL + l0 + lL;
    geta[size_t(cb2lex[par * Vh + cb]) * 12 + comp] = make_double2(g.re, g.im);
  }
}

}  // namespace

int launch_adj_source(dwa_ctx* ctx, void* f_b, void* f_r, const void* eta_p) {
  const size_t n = size_t(2) * ctx->Ls * 12 * ctx->Vh;
  hipLaunchKernelGGL(adj_source_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)f_b, (double2*)f_r, (const double2*)eta_p, ctx->d_cb2lex, ctx->Ls,
                     (unsigned)ctx->Vh);
  return hip_fail(hipGetLastError(), "adjoint source launch");
}

int launch_omega(dwa_ctx* ctx, void* ob, void* oc, const void* psi, const void* eta, int par) {
  const size_t n = size_t(ctx->Ls) * 12 * ctx->Vh;
  hipLaunchKernelGGL(omega_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream, (double2*)ob,
                     (double2*)oc, (const double2*)psi, (const double2*)eta, ctx->d_cb2lex, par,
                     ctx->Ls, (unsigned)ctx->Vh, ctx->alpha, ctx->m);
  return hip_fail(hipGetLastError(), "omega launch");
}

int launch_jpsi(dwa_ctx* ctx, void* out, const void* psi) {
  const size_t n = size_t(ctx->Ls) * 12 * ctx->Vh;
  hipLaunchKernelGGL(jpsi_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream, (double2*)out,
                     (const double2*)psi, ctx->Ls, (unsigned)ctx->Vh);
  return hip_fail(hipGetLastError(), "jpsi launch");
}

int slice_dot_blocks(size_t per_slice) { return grid_for(per_slice, 256, 256); }

int launch_slice_dot(dwa_ctx* ctx, const void* a, const void* b, int nslices, size_t vh, bool g5,
                     double* partials) {
  const int nb = slice_dot_blocks(12 * vh);
  hipLaunchKernelGGL(slice_dot_kernel, dim3(nb, nslices), dim3(256), 0, ctx->stream,
                     (const double2*)a, (const double2*)b, (unsigned)vh, g5 ? 1 : 0, partials);
  return hip_fail(hipGetLastError(), "slice dot launch");
}

int launch_force(dwa_ctx* ctx, void* gU, const void* lt_b, const void* lt_r, const void* ph_b,
                 const void* ph_r) {
  const size_t n = size_t(2) * 4 * ctx->Vh;
  const int Lxyz = ctx->dims[0] * ctx->dims[1] * ctx->dims[2];
  hipLaunchKernelGGL(force_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, ctx->stream,
                     (double2*)gU, (const double2*)lt_b, (const double2*)lt_r,
                     (const double2*)ph_b, (const double2*)ph_r, ctx->d_nbr, ctx->d_cb2lex,
                     ctx->Ls, (unsigned)ctx->Vh, Lxyz, ctx->dims[3], ctx->antiperiodic_t);
  return hip_fail(hipGetLastError(), "force launch");
}

int launch_geta(dwa_ctx* ctx, void* geta, const void* lt_b, const void* lt_r, const void* dw_b,
                const void* dw_r) {
  const size_t n = size_t(2) * 12 * ctx->Vh;
  const int L = ctx->Ls;
  hipLaunchKernelGGL(geta_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)geta, (const double2*)lt_b, (const double2*)lt_r,
                     (const double2*)dw_b, (const double2*)dw_r, ctx->d_cb2lex, L,
                     (unsigned)ctx->Vh, ctx->b[0], ctx->c[0], ctx->b[L - 1], ctx->c[L - 1]);
  return hip_fail(hipGetLastError(), "source gradient launch");
}

}  // namespace dwa
