// gfx950 kernels of libdwa that do not depend on the field precision (reductions,
// solver scalars, source construction, extraction, input checks) and the dispatch of
// every launcher on the storage precision.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "dwa_internal.h"
#include "kreduce.h"

namespace dwa {

namespace {

constexpr int RED_THREADS = 256;

// Scalars of the CG set-up and of the host checks (the per-iteration step lengths a and
// beta are summed inside the update kernels):
//   which 2 -> init: gamma = sum(a), rr = b2 = sum(b), flags cleared, field active;
//   which 4 -> rr = sum(a).
// Block r finalizes field r of a batch (partials packed per field).
__global__ void __launch_bounds__(RED_THREADS) cg_finalize_kernel(DevScalars* s, int which,
                                                                   const double* pa, int na,
                                                                   const double* pb, int nb) {
  s += blockIdx.x;
  pa += size_t(blockIdx.x) * na;
  if (pb) pb += size_t(blockIdx.x) * nb;
  const double A = sum_partials_block(pa, na);
  const double B = (pb != nullptr) ? sum_partials_block(pb, nb) : 0.0;
  if (threadIdx.x != 0) return;
  if (which == 2) {
    s->gamma = A;
    s->rr = B;
    s->b2 = B;
    s->flags = 0;
    s->active = 1;
  } else {
    s->rr = A;
  }
}

__global__ void __launch_bounds__(RED_THREADS) sum_partials_kernel(double* out, const double* pa,
                                                                    int na) {
  const double A = sum_partials_block(pa, na);
  if (threadIdx.x == 0) *out = A;
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
                                                     double bL, double cL, double ms) {
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
    // rows 1 and Ls of eq.(mobius1) at alpha = 1 and mass ms on P (eta, 0, ..., 0):
    //   rho_1  = (b_1 D_w + 1) P- eta - ms (c_1 D_w - 1) P+ eta,
    //   rho_Ls = (b_Ls D_w + 1) P+ eta - ms (c_Ls D_w - 1) P- eta;
    // chi is the part D_w acts on, the remainder is site-local
    double f = 0.0, g = 0.0;
    if (s == 0) {
      f = upper ? -ms * c0 : b0;
      g = upper ? ms : 1.0;
      wall = true;
    } else if (s == (unsigned)(Ls - 1)) {
      f = upper ? bL : -ms * cL;
      g = upper ? 1.0 : ms;
      wall = true;
    }
    const double2 cv = make_double2(f * e.x, f * e.y);
    chi[idx] = cv;
    const double ne = wall ? g : 0.0;
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

// X += s x_l and x_l = 0 for every field of a batch (blockIdx.y; per-field s when a
// table is given): the low-precision solution accumulator folded into the FP64
// solution at a reliable update or a defect-correction step, in one pass.
template <typename SX>
__global__ void __launch_bounds__(256) fold_acc_kernel(double2* __restrict__ X,
                                                       typename SX::elem* __restrict__ xl, size_t n,
                                                       double scale, const double* __restrict__ scales) {
  X += size_t(blockIdx.y) * n;
  xl += size_t(blockIdx.y) * n;
  if (scales) scale = scales[blockIdx.y];
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    const cpx<typename SX::real> v = ld<SX>(xl, i);
    double2 x = X[i];
    x.x += scale * double(v.re);
    x.y += scale * double(v.im);
    X[i] = x;
    st<SX>(xl, i, cmk<typename SX::real>(0, 0));
  }
}

// RES = PHI - Q (FP64) with the block partial sums of |RES|^2, per field of a batch.
__global__ void __launch_bounds__(256) residual_kernel(double2* __restrict__ res,
                                                       const double2* __restrict__ phi,
                                                       const double2* __restrict__ q, size_t n,
                                                       double* __restrict__ partials) {
  const size_t off = size_t(blockIdx.y) * n;
  res += off;
  phi += off;
  q += off;
  double v = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    const double2 a = phi[i], b = q[i];
    const double2 r = make_double2(a.x - b.x, a.y - b.y);
    res[i] = r;
    v += r.x * r.x + r.y * r.y;
  }
  block_sum_to(v, &partials[blockIdx.y * gridDim.x + blockIdx.x]);
}

inline int grid_for(size_t n, int block, int cap = 65536) {
  size_t g = (n + block - 1) / block;
  if (g > (size_t)cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
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

namespace {
// Diagnostics: DWA_BATCH_SERIAL=hop,smix,up1,up2,vec,fin runs the named batched kernels
// as one launch per field (same arithmetic, no cross-field concurrency).
bool serial(const char* what) {
  const char* e = std::getenv("DWA_BATCH_SERIAL");
  return e && std::strstr(e, what) != nullptr;
}
template <typename T>
T* fshift(T* p, int prec, size_t n, int f) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<std::conditional_t<std::is_const_v<T>, const char, char>*>(p) +
                                  elem_bytes(prec) * n * f)
           : p;
}
}  // namespace

int launch_hop(dwa_ctx* ctx, int prec, const HopOp& op, int* nblocks_out) {
  if (op.nrhs > 1 && (serial("hop,") || serial("hopall") || (op.partials && serial("hopp")) ||
                      (!op.partials && serial("hopn")))) {
    const size_t n = field_elems(ctx);
    for (int f = 0; f < op.nrhs; ++f) {
      HopOp o = op;
      o.nrhs = 1;
      o.in = fshift(op.in, prec, n, f);
      o.out = fshift(op.out, prec, n, f);
      o.pre = fshift(op.pre, prec, n, f);
      o.post = fshift(op.post, prec, n, f);
      int nb = 0;
      if (op.partials) {
        // per-field partial counts are the same for every field: find them first
        HopOp probe = o;
        probe.partials = op.partials;
        if (f == 0) {
          int rc = launch_hop(ctx, prec, probe, &nb);
          if (rc) return rc;
          if (nblocks_out) *nblocks_out = nb;
          continue;
        }
        o.partials = op.partials + size_t(f) * (nblocks_out ? *nblocks_out : 0);
      }
      int rc = launch_hop(ctx, prec, o, &nb);
      if (rc) return rc;
      if (nblocks_out) *nblocks_out = nb;
    }
    return DWA_OK;
  }
  DWA_DISPATCH(prec, launch_hop_p<S_>(ctx, op, nblocks_out));
}
int launch_smix(dwa_ctx* ctx, int prec, int mix, void* out, const void* in, const void* post,
                double post_coef, int nslices, double* partials, int* nblocks_out, int nrhs) {
  if (nrhs > 1 && serial("smix")) {
    const size_t n = field_elems(ctx);
    for (int f = 0; f < nrhs; ++f) {
      int nb = 0;
      int rc = launch_smix(ctx, prec, mix, fshift(out, prec, n, f), fshift(in, prec, n, f),
                           fshift(post, prec, n, f), post_coef, nslices,
                           partials ? partials + size_t(f) * ((6 * ctx->Vh + 255) / 256) : nullptr, &nb, 1);
      if (rc) return rc;
      if (nblocks_out) *nblocks_out = nb;
    }
    return DWA_OK;
  }
  DWA_DISPATCH(prec, launch_smix_p<S_>(ctx, mix, out, in, post, post_coef, nslices, partials,
                                       nblocks_out, nrhs));
}
int launch_cg_update1(dwa_ctx* ctx, int prec, void* x, void* r, void* w, const void* p,
                      const void* q, DevScalars* s, double* partials, int* nblocks, bool adj,
                      int nrhs, const double* qparts, int nq, const double* zparts, int nz) {
  if (nrhs > 1 && serial("up1")) {
    const size_t n = field_elems(ctx);
    for (int f = 0; f < nrhs; ++f) {
      int nb = 0;
      int rc = launch_cg_update1(ctx, prec, fshift(x, xacc_prec(prec), n, f), fshift(r, prec, n, f),
                                 fshift(w, prec, n, f), fshift(p, prec, n, f), fshift(q, prec, n, f), s + f,
                                 partials + size_t(f) * ((6 * ctx->Vh + 255) / 256), &nb, adj, 1,
                                 qparts ? qparts + size_t(f) * nq : nullptr, nq,
                                 zparts ? zparts + size_t(f) * nz : nullptr, nz);
      if (rc) return rc;
      if (nblocks) *nblocks = nb;
    }
    return DWA_OK;
  }
  DWA_DISPATCH(prec, launch_update1_p<S_>(ctx, x, r, w, p, q, s, partials, nblocks, adj, nrhs, qparts, nq,
                                          zparts, nz));
}
int launch_cg_update2(dwa_ctx* ctx, int prec, void* p, void* u, const void* z,
                      DevScalars* s, bool adj, int nrhs, const double* zparts, int nz) {
  if (nrhs > 1 && serial("up2")) {
    const size_t n = field_elems(ctx);
    for (int f = 0; f < nrhs; ++f) {
      int rc = launch_cg_update2(ctx, prec, fshift(p, prec, n, f), fshift(u, prec, n, f),
                                 fshift(z, prec, n, f), s + f, adj, 1,
                                 zparts ? zparts + size_t(f) * nz : nullptr, nz);
      if (rc) return rc;
    }
    return DWA_OK;
  }
  DWA_DISPATCH(prec, launch_update2_p<S_>(ctx, p, u, z, s, adj, nrhs, zparts, nz));
}
int launch_norm2(dwa_ctx* ctx, int prec, const void* x, size_t n, double* partials, int* nblocks,
                 int nrhs) {
  DWA_DISPATCH(prec, norm2_p<S_>(ctx, x, n, partials, nblocks, nrhs));
}
int launch_axpby(dwa_ctx* ctx, int prec, void* y, double a, const void* x, double b, size_t n,
                 int nrhs, const double* ab) {
  DWA_DISPATCH(prec, axpby_p<S_>(ctx, y, a, x, b, n, nrhs, ab));
}
int launch_zero(dwa_ctx* ctx, int prec, void* p, size_t n, int nrhs) {
  DWA_DISPATCH(prec, zero_p<S_>(ctx, p, n, nrhs));
}
int launch_pack5(dwa_ctx* ctx, int prec, void* dst, const void* src, int parity, int nslices) {
  DWA_DISPATCH(prec, pack5_p<S_>(ctx, dst, src, parity, nslices));
}
int launch_unpack5(dwa_ctx* ctx, int prec, void* dst, const void* src, int parity, int nslices) {
  DWA_DISPATCH(prec, unpack5_p<S_>(ctx, dst, src, parity, nslices));
}
int launch_pack_links(dwa_ctx* ctx, int prec, void* dst, const void* src) {
  DWA_DISPATCH(prec, pack_links_p<S_>(ctx, dst, src));
}
namespace {
template <typename SO>
int convert_from(dwa_ctx* ctx, void* out, int prec_in, const void* in, size_t n, double scale,
                 int nrhs, const double* scales) {
  DWA_DISPATCH(prec_in, (convert_p<SO, S_>(ctx, out, in, n, scale, nrhs, scales)));
}
}  // namespace
int launch_convert(dwa_ctx* ctx, int prec_out, void* out, int prec_in, const void* in, size_t n,
                   double scale, int nrhs, const double* scales) {
  DWA_DISPATCH(prec_out, convert_from<S_>(ctx, out, prec_in, in, n, scale, nrhs, scales));
}

int launch_cg_finalize(dwa_ctx* ctx, int which, DevScalars* s, const double* pa, int na,
                       const double* pb, int nb, int nrhs) {
  if (which != 2 && which != 4) {
    set_error("finalize: unknown scalar set");
    return DWA_EINVAL;
  }
  if (nrhs > 1 && serial("fin")) {
    for (int f = 0; f < nrhs; ++f) {
      int rc = launch_cg_finalize(ctx, which, s + f, pa + size_t(f) * na, na,
                                  pb ? pb + size_t(f) * nb : nullptr, nb, 1);
      if (rc) return rc;
    }
    return DWA_OK;
  }
  hipLaunchKernelGGL(cg_finalize_kernel, dim3(nrhs), dim3(RED_THREADS), 0, ctx->stream, s, which,
                     pa, na, pb, nb);
  return hip_fail(hipGetLastError(), "finalize launch");
}

namespace {
__global__ void scale_gamma_kernel(DevScalars* s, double f, const double* fs) {
  // field blockIdx.x of a batch, with its own factor when a table is given
  if (threadIdx.x == 0) s[blockIdx.x].gamma *= fs ? fs[blockIdx.x] : f;
}
}  // namespace

int launch_scale_gamma(dwa_ctx* ctx, DevScalars* s, double f, int nrhs, const double* fs) {
  hipLaunchKernelGGL(scale_gamma_kernel, dim3(nrhs), dim3(64), 0, ctx->stream, s, f, fs);
  return hip_fail(hipGetLastError(), "scale gamma launch");
}

int launch_fold_acc(dwa_ctx* ctx, int xprec, void* X, void* xl, size_t n, double scale, int nrhs,
                    const double* scales) {
  const dim3 grid(grid_for(n, 256, 4096), nrhs);
  if (xprec == DWA_F32)
    hipLaunchKernelGGL(fold_acc_kernel<F32>, grid, dim3(256), 0, ctx->stream, (double2*)X, (float2*)xl, n,
                       scale, scales);
  else if (xprec == DWA_F64)
    hipLaunchKernelGGL(fold_acc_kernel<F64>, grid, dim3(256), 0, ctx->stream, (double2*)X, (double2*)xl, n,
                       scale, scales);
  else {
    set_error("solution accumulator must be FP32 or FP64");
    return DWA_EINVAL;
  }
  return hip_fail(hipGetLastError(), "fold launch");
}

int launch_residual(dwa_ctx* ctx, void* res, const void* phi, const void* q, size_t n, double* partials,
                    int* nblocks, int nrhs) {
  const int g = grid_for(n, 256, 2048);
  hipLaunchKernelGGL(residual_kernel, dim3(g, nrhs), dim3(256), 0, ctx->stream, (double2*)res,
                     (const double2*)phi, (const double2*)q, n, partials);
  if (nblocks) *nblocks = g;
  return hip_fail(hipGetLastError(), "residual launch");
}

int launch_sum_partials(dwa_ctx* ctx, const double* partials, int n, double* out) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RED_THREADS), 0, ctx->stream, out,
                     partials, n);
  return hip_fail(hipGetLastError(), "sum partials launch");
}

int launch_source(dwa_ctx* ctx, void* chi_b, void* chi_r, void* aux_b, void* aux_r,
                  const void* eta, double ms) {
  const int Ls = ctx->Ls;
  const size_t n = size_t(2) * Ls * 12 * ctx->Vh;
  hipLaunchKernelGGL(source_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream,
                     (double2*)chi_b, (double2*)chi_r, (double2*)aux_b, (double2*)aux_r,
                     (const double2*)eta, ctx->d_cb2lex, Ls, (unsigned)ctx->Vh, ctx->M5, ctx->b[0],
                     ctx->c[0], ctx->b[Ls - 1], ctx->c[Ls - 1], ms);
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
