// C-ABI of libdwa: context set-up, operators, CG on the normal equations and the
// propagator pipeline.  Host code; every arithmetic step runs in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "dwa_internal.h"

namespace dwa {

namespace {
thread_local std::string g_last_error;

constexpr int kBanks = 4;
static_assert(sizeof(((dwa_ctx*)nullptr)->w64) / sizeof(void*) == W64_COUNT, "w64 slots");
static_assert(sizeof(((dwa_ctx*)nullptr)->w32) / sizeof(void*) == LOW_COUNT, "w32 slots");
static_assert(sizeof(((dwa_ctx*)nullptr)->w16) / sizeof(void*) == LOW_COUNT, "w16 slots");
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
  if (e == hipSuccess) return DWA_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? DWA_ENOMEM : DWA_EHIP;
}

size_t field_elems(const dwa_ctx* ctx) { return size_t(ctx->Ls) * 12 * size_t(ctx->Vh); }

}  // namespace dwa

using namespace dwa;

namespace {

int einval(const std::string& msg) {
  set_error(msg);
  return DWA_EINVAL;
}

#define DWA_TRY(expr)             \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != DWA_OK) return rc_; \
  } while (0)
#define DWA_HIP(expr, what) DWA_TRY(hip_fail((expr), what))

// LDS bytes of one fused-hop block (the device code's hop_mix_lds_bytes): the
// [Ls][12][ns+1] output tile and the [72][ns] link area (sharing space when the block
// does one field, nf = 1), plus [8][ns] neighbours; cbytes is the size of one complex
// in the kernel's arithmetic (16 FP64, 8 otherwise).
size_t hop_mix_lds_bytes_host(int ns, int Ls, size_t cbytes, int nf = 1) {
  const size_t tile = size_t(Ls) * 12 * (ns + 1) * cbytes, link = size_t(72) * ns * cbytes;
  return (nf > 1 ? tile + link : std::max(tile, link)) + size_t(8) * ns * 4;
}

void** low_pool(dwa_ctx* ctx, int prec) {
  if (prec == DWA_F32) return ctx->w32;
  if (prec == DWA_BF16) return ctx->w16;
  return ctx->w64;
}

// buffer for the solution accumulated by a low-precision CGLS (FP32 for BF16 storage)
void* xacc_buf(dwa_ctx* ctx, int prec) {
  return prec == DWA_BF16 ? ctx->w32[L_X] : low_pool(ctx, prec)[L_X];
}

double* bank(dwa_ctx* ctx, int i) { return ctx->d_partials + size_t(i) * ctx->partials_per_bank; }

bool valid_prec(int prec) { return prec == DWA_F64 || prec == DWA_F32 || prec == DWA_BF16; }

// ---------------------------------------------------------------------------
// operator building blocks.  Fields are black SoA of precision prec; tb / tr are
// workspace vectors (black / red) of the same precision.

// out = in - 1/4 G^-1 I^-1 H_br N H_rb (B G in); u is the premixed input B G in.
int dbb_from_premix(dwa_ctx* ctx, int prec, void* out, const void* in, const void* u, void* tr,
                    double* partials, int* nblocks, int nrhs = 1) {
  HopOp a{u, tr, nullptr, nullptr, 1.0, 0.0, 0.0, MIX_N, 1, ctx->Ls, nullptr, nrhs};
  DWA_TRY(launch_hop(ctx, prec, a, nullptr));
  HopOp b{tr, out, nullptr, in, -0.25, 0.0, 1.0, MIX_GINV_IINV, 0, ctx->Ls, partials, nrhs};
  return launch_hop(ctx, prec, b, nblocks);
}

// out = in - 1/4 G B^T g5 H_br N^T H_rb w; w is the premixed input g5 I^-T G^-1 in.
int dbbdag_from_premix(dwa_ctx* ctx, int prec, void* out, const void* in, const void* w, void* tr,
                       double* partials, int* nblocks, int nrhs = 1) {
  HopOp a{w, tr, nullptr, nullptr, 1.0, 0.0, 0.0, MIX_NT, 1, ctx->Ls, nullptr, nrhs};
  DWA_TRY(launch_hop(ctx, prec, a, nullptr));
  HopOp b{tr, out, nullptr, in, -0.25, 0.0, 1.0, MIX_G_BT_G5, 0, ctx->Ls, partials, nrhs};
  return launch_hop(ctx, prec, b, nblocks);
}

int apply_dbb(dwa_ctx* ctx, int prec, void* out, const void* in, void* tb, void* tr, int nrhs = 1) {
  DWA_TRY(launch_smix(ctx, prec, MIX_BG, tb, in, nullptr, 0.0, ctx->Ls, nullptr, nullptr, nrhs));
  return dbb_from_premix(ctx, prec, out, in, tb, tr, nullptr, nullptr, nrhs);
}

int apply_dbbdag(dwa_ctx* ctx, int prec, void* out, const void* in, void* tb, void* tr) {
  DWA_TRY(launch_smix(ctx, prec, MIX_G5_IINVT_GINV, tb, in, nullptr, 0.0, ctx->Ls, nullptr,
                      nullptr));
  return dbbdag_from_premix(ctx, prec, out, in, tb, tr, nullptr, nullptr);
}

int read_scalars(dwa_ctx* ctx) {
  DWA_HIP(hipMemcpyAsync(ctx->h_scal, ctx->d_scal, sizeof(DevScalars), hipMemcpyDeviceToHost,
                         ctx->stream),
          "scalar readback");
  DWA_HIP(hipStreamSynchronize(ctx->stream), "stream sync");
  return DWA_OK;
}

// |v|^2 of a field into a host double (synchronising)
int host_norm2(dwa_ctx* ctx, int prec, const void* v, double* out, size_t n = 0) {
  int nb = 0;
  DWA_TRY(launch_norm2(ctx, prec, v, n ? n : field_elems(ctx), bank(ctx, 3), &nb));
  DWA_TRY(launch_sum_partials(ctx, bank(ctx, 3), nb, ctx->d_red));
  DWA_HIP(hipMemcpyAsync(out, ctx->d_red, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
          "norm readback");
  DWA_HIP(hipStreamSynchronize(ctx->stream), "stream sync");
  return DWA_OK;
}

// Single-field solves run on the context's own stream, so that one CG iteration can be
// captured into a hipGraph (capture needs a stream other than the null stream) and
// replayed between the host's convergence checks.  Entry waits for the caller's stream;
// exit drains the solve stream, so the caller's later work sees the results.
struct SolveStream {
  dwa_ctx* ctx;
  hipStream_t saved;
  bool on;
  SolveStream(dwa_ctx* c) : ctx(c), saved(c->stream), on(c->cap_stream && c->stream != c->cap_stream) {
    if (on) {
      (void)hipStreamSynchronize(saved);
      ctx->stream = ctx->cap_stream;
    }
  }
  ~SolveStream() {
    if (on) {
      (void)hipStreamSynchronize(ctx->stream);
      ctx->stream = saved;
    }
  }
};

// The iteration body of a CGLS between two host checks, replayed from a hipGraph (kernel
// nodes only: the body launches kernels and nothing else), or issued eagerly with
// DWA_SOLVE_NO_GRAPH set.  Both give bitwise the same result.
struct BodyGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use;
  explicit BodyGraph(dwa_ctx* ctx) : use(ctx->cap_stream && !std::getenv("DWA_SOLVE_NO_GRAPH")) {}
  ~BodyGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  // capture body() once (it is issued, not run, during capture), then replay it
  template <typename F>
  int run(dwa_ctx* ctx, F&& body) {
    if (!use) return body();
    if (!exec) {
      DWA_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "begin capture");
      const int rc = body();
      const hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
      if (rc != DWA_OK) return rc;
      DWA_HIP(e, "end capture");
      DWA_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    }
    return hip_fail(hipGraphLaunch(exec, ctx->stream), "graph launch");
  }
};

// CGLS on D_bb of precision prec with the workspace pool of that precision.
// rhs is a field of precision prec, x one of precision xacc_prec(prec); a warm start
// (x as given) is supported for FP64 only.  Stops when the recursive
// residual satisfies |r|^2 <= tol^2 |rhs|^2 or after maxiter iterations.
struct CgResult {
  int iters = 0;
  int converged = 0;
  int breakdown = 0;
  double rel_recursive = 0.0;
  long long n_dbb = 0;
};

int cgls(dwa_ctx* ctx, int prec, void* x, const void* rhs, bool warm, double tol, int maxiter,
         int check_every, CgResult* res, bool adj = false) {
  SolveStream solve_stream(ctx);
  void** W = low_pool(ctx, prec);
  const bool p64 = prec == DWA_F64;
  void* r = W[p64 ? W_R : L_R];
  void* p = W[p64 ? W_P : L_P];
  void* z = W[p64 ? W_Z : L_Z];
  void* q = W[p64 ? W_Q : L_Q];
  void* w = W[p64 ? W_W : L_W];
  void* u = W[p64 ? W_U : L_U];
  void* t = W[p64 ? W_T : L_T];
  const size_t n = field_elems(ctx);
  DevScalars* sc = ctx->d_scal;
  int nbA = 0, nbB = 0, nbZ = 0;  // partials: bank 0 |q|^2, bank 1 |r|^2, bank 2 |z|^2
  if (check_every < 1) check_every = 1;

  if (warm && !p64) {
    set_error("warm-started CGLS needs FP64 storage");
    return DWA_EINVAL;
  }
  // A is D_bb, or D_bb^dag for adj (CGLS on the adjoint system); the premixed input of
  // A (u, from p) and of A^dag (w, from r) follow
  const int mixA = adj ? MIX_G5_IINVT_GINV : MIX_BG;
  const int mixAd = adj ? MIX_BG : MIX_G5_IINVT_GINV;
  auto applyA = [&](void* out, const void* in, const void* pre, double* part, int* nb) {
    return adj ? dbbdag_from_premix(ctx, prec, out, in, pre, t, part, nb)
               : dbb_from_premix(ctx, prec, out, in, pre, t, part, nb);
  };
  auto applyAd = [&](void* out, const void* in, const void* pre, double* part, int* nb) {
    return adj ? dbb_from_premix(ctx, prec, out, in, pre, t, part, nb)
               : dbbdag_from_premix(ctx, prec, out, in, pre, t, part, nb);
  };
  if (warm) {
    DWA_TRY(launch_smix(ctx, prec, mixA, u, x, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
    DWA_TRY(applyA(q, x, u, nullptr, nullptr));
    DWA_TRY(launch_axpby(ctx, prec, r, 1.0, rhs, 0.0, n));
    DWA_TRY(launch_axpby(ctx, prec, r, -1.0, q, 1.0, n));
    res->n_dbb += 1;
  } else {
    DWA_TRY(launch_zero(ctx, xacc_prec(prec), x, n));
    DWA_TRY(launch_axpby(ctx, prec, r, 1.0, rhs, 0.0, n));
  }
  // z = A^dag r, gamma = |z|^2, |rhs|^2
  DWA_TRY(launch_smix(ctx, prec, mixAd, w, r, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
  DWA_TRY(applyAd(z, r, w, bank(ctx, 2), &nbZ));
  DWA_TRY(launch_norm2(ctx, prec, rhs, n, bank(ctx, 1), &nbB));
  DWA_TRY(launch_cg_finalize(ctx, 2, sc, bank(ctx, 2), nbZ, bank(ctx, 1), nbB));
  if (warm) {
    DWA_TRY(launch_norm2(ctx, prec, r, n, bank(ctx, 1), &nbB));
    DWA_TRY(launch_cg_finalize(ctx, 4, sc, bank(ctx, 1), nbB, nullptr, 0));
  }
  res->n_dbb += 1;
  DWA_TRY(launch_axpby(ctx, prec, p, 1.0, z, 0.0, n));
  DWA_TRY(launch_smix(ctx, prec, mixA, u, p, nullptr, 0.0, ctx->Ls, nullptr, nullptr));

  const double tol2 = tol * tol;
  // first half of an iteration: q = A p (premixed u), |q|^2; (a = gamma / |q|^2 from those
  // partials inside update 1) x += a p ; r -= a q ; |r|^2 ; w = premix of r for A^dag
  // (gamma = |z|^2 from the current z's partials, also inside update 1)
  auto first_half = [&]() -> int {
    DWA_TRY(applyA(q, p, u, bank(ctx, 0), &nbA));
    return launch_cg_update1(ctx, prec, x, r, w, p, q, sc, bank(ctx, 1), &nbB, adj, 1, bank(ctx, 0), nbA,
                             bank(ctx, 2), nbZ);
  };
  // second half: z = A^dag r ; (beta = |z|^2 / gamma inside update 2) p = z + beta p ;
  // u = premix of p for A
  auto second_half = [&]() -> int {
    DWA_TRY(applyAd(z, r, w, bank(ctx, 2), &nbZ));
    return launch_cg_update2(ctx, prec, p, u, z, sc, adj, 1, bank(ctx, 2), nbZ);
  };
  // The host checks after x and r have been updated; between checks the body (second half
  // of iteration k, first half of k + 1) is replayed from a graph.
  BodyGraph g(ctx);
  int k = 0;
  for (;;) {
    if (k % check_every == 0 || k >= maxiter) {
      // |r|^2 from the last update 1's partials (at k = 0 the set-up's value stands)
      if (k > 0) DWA_TRY(launch_cg_finalize(ctx, 4, sc, bank(ctx, 1), nbB, nullptr, 0));
      DWA_TRY(read_scalars(ctx));
      const DevScalars& h = *ctx->h_scal;
      if (h.flags) {
        res->breakdown = 1;
        break;
      }
      res->rel_recursive = h.b2 > 0 ? std::sqrt(h.rr / h.b2) : 0.0;
      if (h.b2 == 0.0 || h.rr <= tol2 * h.b2) {
        res->converged = 1;
        break;
      }
      if (k >= maxiter) break;
    }
    if (k == 0) {
      DWA_TRY(first_half());
      res->n_dbb += 1;
    } else {
      DWA_TRY(g.run(ctx, [&]() -> int {
        DWA_TRY(second_half());
        return first_half();
      }));
      res->n_dbb += 2;
    }
    ++k;
  }
  res->iters = k;
  return DWA_OK;
}

// rho += -1/2 H chi on the two wall slices of both parities (nr fields field_elems
// apart): the source chi of D_1(1) P (eta, 0, ..., 0) lives on s = 0 and s = Ls - 1
// only, so the hop of every other slice would add zeros.
int wall_hops(dwa_ctx* ctx, void* chi_b, void* chi_r, void* rho_b, void* rho_r, int nr = 1) {
  const size_t slice = size_t(12) * ctx->Vh;
  for (const int s : {0, ctx->Ls - 1}) {
    auto at = [&](void* f) { return static_cast<void*>(static_cast<double2*>(f) + s * slice); };
    const HopOp hb{at(chi_r), at(rho_b), at(rho_b), nullptr, -0.5, 1.0, 0.0, MIX_IDENTITY, 0, 1, nullptr, nr};
    const HopOp hr{at(chi_b), at(rho_r), at(rho_r), nullptr, -0.5, 1.0, 0.0, MIX_IDENTITY, 1, 1, nullptr, nr};
    DWA_TRY(launch_hop(ctx, DWA_F64, hb, nullptr));
    DWA_TRY(launch_hop(ctx, DWA_F64, hr, nullptr));
  }
  return DWA_OK;
}

// |rhs - D_bb x| / |rhs| in FP64 (uses W_Q, W_RES, W_OPB, W_OPR)
int true_residual64(dwa_ctx* ctx, const void* x, const void* rhs, double rhs_norm, double* rel,
                    void* res_out, bool adj = false) {
  void** W = ctx->w64;
  const size_t n = field_elems(ctx);
  if (adj)
    DWA_TRY(apply_dbbdag(ctx, DWA_F64, W[W_Q], x, W[W_OPB], W[W_OPR]));
  else
    DWA_TRY(apply_dbb(ctx, DWA_F64, W[W_Q], x, W[W_OPB], W[W_OPR]));
  void* r = res_out ? res_out : W[W_RES];
  int nb = 0;
  DWA_TRY(launch_residual(ctx, r, rhs, W[W_Q], n, bank(ctx, 3), &nb));
  DWA_TRY(launch_sum_partials(ctx, bank(ctx, 3), nb, ctx->d_red));
  double rr = 0.0;
  DWA_HIP(hipMemcpyAsync(&rr, ctx->d_red, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
          "norm readback");
  DWA_HIP(hipStreamSynchronize(ctx->stream), "stream sync");
  *rel = rhs_norm > 0 ? std::sqrt(rr) / rhs_norm : 0.0;
  return DWA_OK;
}

// Mixed precision: FP64 outer defect correction around an inner CGLS in storage
// precision inner (F32 or BF16, FP32 arithmetic).  Each outer step recomputes the
// true FP64 residual r = rhs - D_bb x, solves D_bb e = r / |r| in low precision to a
// relative residual delta, and accumulates x += |r| e in FP64.
int mixed_solve(dwa_ctx* ctx, int inner, void* x, const void* rhs, const dwa_solve_opts* o,
                dwa_solve_stats* st) {
  void** W = ctx->w64;
  void** L = low_pool(ctx, inner);
  const size_t n = field_elems(ctx);
  double b2 = 0.0;
  DWA_TRY(host_norm2(ctx, DWA_F64, rhs, &b2));
  const double bnorm = std::sqrt(b2);
  if (!o->warm_start) DWA_TRY(launch_zero(ctx, DWA_F64, x, n));
  if (bnorm == 0.0) {
    st->converged = 1;
    st->rel_resid = 0.0;
    return DWA_OK;
  }
  const double delta = (o->delta > 0.0 && o->delta < 1.0) ? o->delta : 0.1;
  int total = 0;
  long long ndbb = 0;
  int outer = 0;
  double rel = 1.0;
  // first residual
  if (o->warm_start) {
    DWA_TRY(true_residual64(ctx, x, rhs, bnorm, &rel, W[W_RES]));
    ndbb += 1;
  } else {
    DWA_TRY(launch_axpby(ctx, DWA_F64, W[W_RES], 1.0, rhs, 0.0, n));
    rel = 1.0;
  }
  int status = DWA_OK;
  double prev_rel = rel;
  int stall = 0;
  while (rel > o->tol) {
    if (total >= o->maxiter) {
      status = DWA_ENOCONV;
      break;
    }
    const double rnorm = rel * bnorm;
    // low-precision rhs: r / |r|
    DWA_TRY(launch_convert(ctx, inner, L[L_OPB], DWA_F64, W[W_RES], n, 1.0 / rnorm));
    // inner target: delta, but not tighter than needed for the final tolerance
    double inner_tol = delta;
    const double need = 0.5 * o->tol / rel;
    if (need > inner_tol) inner_tol = need;
    CgResult cr;
    DWA_TRY(cgls(ctx, inner, xacc_buf(ctx, inner), L[L_OPB], false, inner_tol, o->maxiter - total,
                 o->check_every, &cr));
    total += cr.iters;
    ndbb += cr.n_dbb;
    if (cr.breakdown && cr.iters == 0) {
      status = DWA_EBREAKDOWN;
      break;
    }
    // x += |r| e  (FP64 accumulate)
    DWA_TRY(launch_fold_acc(ctx, xacc_prec(inner), x, xacc_buf(ctx, inner), n, rnorm));
    DWA_TRY(true_residual64(ctx, x, rhs, bnorm, &rel, W[W_RES]));
    ndbb += 1;
    ++outer;
    if (!(rel < 0.9 * prev_rel)) {
      if (++stall >= 3) {
        status = DWA_ENOCONV;
        break;
      }
    } else {
      stall = 0;
    }
    prev_rel = rel;
  }
  st->iters = total;
  st->outer = outer;
  st->converged = rel <= o->tol;
  st->rel_resid = rel;
  st->n_Dbb = ndbb;
  return status;
}

// Mixed precision with reliable updates.  One CGLS runs in the low storage precision
// (FP32 or BF16, FP32 arithmetic) and keeps its search direction p for the whole solve.
// Its recursive residual r_l drifts from the true one at the level of the storage
// rounding, so whenever |r_l| has fallen by delta since the last update the low
// correction x_l is added into the FP64 solution, the true residual rhs - D_bb x is
// recomputed in FP64 and replaces r_l, and CGLS continues from there (z = D_bb^dag r,
// beta = |z|^2 / gamma).  The solve stops on the FP64 residual.
int reliable_solve(dwa_ctx* ctx, int inner, void* x, const void* rhs, const dwa_solve_opts* o,
                   dwa_solve_stats* st, bool adj = false) {
  SolveStream solve_stream(ctx);
  void** W = ctx->w64;
  void** Lw = low_pool(ctx, inner);
  void* r = Lw[L_R];
  void* p = Lw[L_P];
  void* z = Lw[L_Z];
  void* q = Lw[L_Q];
  void* w = Lw[L_W];
  void* u = Lw[L_U];
  void* t = Lw[L_T];
  void* xl = xacc_buf(ctx, inner);
  const int xprec = xacc_prec(inner);
  const size_t n = field_elems(ctx);
  DevScalars* sc = ctx->d_scal;
  int nbA = 0, nbB = 0, nbZ = 0;  // partials: bank 0 |q|^2, bank 1 |r|^2, bank 2 |z|^2
  const int check_every = o->check_every < 1 ? 1 : o->check_every;
  const double delta = (o->delta > 0.0 && o->delta < 1.0) ? o->delta : 0.1;
  // A is D_bb, or D_bb^dag for adj (the adjoint solve); the premixed input of A (u,
  // from p) and of A^dag (w, from r) follow
  const int mixA = adj ? MIX_G5_IINVT_GINV : MIX_BG;
  const int mixAd = adj ? MIX_BG : MIX_G5_IINVT_GINV;
  auto applyA = [&](void* out, const void* in, const void* pre, double* part, int* nb) {
    return adj ? dbbdag_from_premix(ctx, inner, out, in, pre, t, part, nb)
               : dbb_from_premix(ctx, inner, out, in, pre, t, part, nb);
  };
  auto applyAd = [&](void* out, const void* in, const void* pre, double* part, int* nb) {
    return adj ? dbb_from_premix(ctx, inner, out, in, pre, t, part, nb)
               : dbbdag_from_premix(ctx, inner, out, in, pre, t, part, nb);
  };

  double b2 = 0.0;
  DWA_TRY(host_norm2(ctx, DWA_F64, rhs, &b2));
  const double bnorm = std::sqrt(b2);
  if (!o->warm_start) DWA_TRY(launch_zero(ctx, DWA_F64, x, n));
  if (bnorm == 0.0) {
    st->converged = 1;
    st->rel_resid = 0.0;
    return DWA_OK;
  }
  long long ndbb = 0;
  int outer = 0;
  double rel = 1.0;
  if (o->warm_start) {
    DWA_TRY(true_residual64(ctx, x, rhs, bnorm, &rel, W[W_RES], adj));
    ndbb += 1;
  } else {
    DWA_TRY(launch_axpby(ctx, DWA_F64, W[W_RES], 1.0, rhs, 0.0, n));
  }
  if (rel <= o->tol) {
    st->converged = 1;
    st->rel_resid = rel;
    return DWA_OK;
  }
  // low-precision state, scaled so the residual starts at unit norm
  double scale = rel * bnorm;  // FP64 residual norm at the last update
  DWA_TRY(launch_convert(ctx, inner, r, DWA_F64, W[W_RES], n, 1.0 / scale));
  DWA_TRY(launch_zero(ctx, xprec, xl, n));
  DWA_TRY(launch_smix(ctx, inner, mixAd, w, r, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
  DWA_TRY(applyAd(z, r, w, bank(ctx, 2), &nbZ));
  DWA_TRY(launch_norm2(ctx, inner, r, n, bank(ctx, 1), &nbB));
  DWA_TRY(launch_cg_finalize(ctx, 2, sc, bank(ctx, 2), nbZ, bank(ctx, 1), nbB));
  DWA_TRY(launch_axpby(ctx, inner, p, 1.0, z, 0.0, n));
  DWA_TRY(launch_smix(ctx, inner, mixA, u, p, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
  ndbb += 1;

  int k = 0, status = DWA_ENOCONV, stall = 0;
  const bool trace = std::getenv("DWA_TRACE_SOLVE") != nullptr;
  double rmax = 1.0;  // |r_l| (scaled units) at the last update
  double last_rel = rel;
  // first half of an iteration: q = D_bb p ; (a from its |q|^2 partials inside update 1)
  // x_l += a p ; r_l -= a q ; |r_l|^2 ; w = g5 I^-T G^-1 r_l
  auto first_half = [&]() -> int {
    DWA_TRY(applyA(q, p, u, bank(ctx, 0), &nbA));
    return launch_cg_update1(ctx, inner, xl, r, w, p, q, sc, bank(ctx, 1), &nbB, adj, 1, bank(ctx, 0), nbA,
                             bank(ctx, 2), nbZ);
  };
  // second half: z = D_bb^dag r_l ; (beta = |z|^2 / gamma inside update 2) p = z + beta p ;
  // u = B G p
  auto second_half = [&]() -> int {
    DWA_TRY(applyAd(z, r, w, bank(ctx, 2), &nbZ));
    return launch_cg_update2(ctx, inner, p, u, z, sc, adj, 1, bank(ctx, 2), nbZ);
  };
  // between host checks the body (second half of iteration k, first half of k + 1) is
  // replayed from a graph; a reliable update runs eagerly between two bodies
  BodyGraph g(ctx);
  while (k < o->maxiter) {
    if (k == 0) {
      DWA_TRY(first_half());
      ndbb += 1;
    } else {
      DWA_TRY(g.run(ctx, [&]() -> int {
        DWA_TRY(second_half());
        return first_half();
      }));
      ndbb += 2;
    }
    ++k;
    bool update = false, done = false;
    if (k % check_every == 0 || k >= o->maxiter) {
      // |r_l|^2 for the host (only at a check: the next D_bb^dag step recomputes it)
      DWA_TRY(launch_cg_finalize(ctx, 4, sc, bank(ctx, 1), nbB, nullptr, 0));
      DWA_TRY(read_scalars(ctx));
      const DevScalars& h = *ctx->h_scal;
      if (h.flags) {
        if (trace)
          std::fprintf(stderr, "[dwa] breakdown at k=%d: gamma=%.3e qq=%.3e zz=%.3e rr=%.3e flags=%d\n",
                       k, h.gamma, h.qq, h.zz, h.rr, h.flags);
        status = DWA_EBREAKDOWN;
        break;
      }
      const double rl = std::sqrt(h.rr);  // scaled units
      // predicted relative residual of the FP64 problem
      const double pred = rl * scale / bnorm;
      if (trace)
        std::fprintf(stderr, "[dwa] k=%d |r_l|=%.3e pred=%.3e gamma=%.3e a=%.3e beta=%.3e qq=%.3e flags=%d\n",
                     k, rl, pred, h.gamma, h.a, h.beta, h.qq, h.flags);
      if (rl <= delta * rmax || pred <= 0.5 * o->tol || k >= o->maxiter) update = true;
    }
    if (update) {
      // x += scale * x_l (FP64), x_l = 0; true residual; r_l = r / |r|
      DWA_TRY(launch_fold_acc(ctx, xprec, x, xl, n, scale));
      DWA_TRY(true_residual64(ctx, x, rhs, bnorm, &rel, W[W_RES], adj));
      ndbb += 1;
      ++outer;
      if (trace) std::fprintf(stderr, "[dwa] update %d at k=%d: true rel %.3e\n", outer, k, rel);
      if (rel <= o->tol) {
        status = DWA_OK;
        done = true;
      } else {
        if (!(rel < 0.9 * last_rel)) {
          if (++stall >= 3) {
            status = DWA_ENOCONV;
            break;
          }
        } else {
          stall = 0;
        }
        last_rel = rel;
        // the new residual is stored at unit norm: rescale the CGLS state (p by f,
        // gamma = |z|^2 by f^2) so the recurrence continues in the new units
        const double new_scale = rel * bnorm;
        const double f = scale / new_scale;
        DWA_TRY(launch_axpby(ctx, inner, p, f, p, 0.0, n));
        DWA_TRY(launch_scale_gamma(ctx, sc, f * f));
        scale = new_scale;
        DWA_TRY(launch_convert(ctx, inner, r, DWA_F64, W[W_RES], n, 1.0 / scale));
        DWA_TRY(launch_smix(ctx, inner, mixAd, w, r, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
        // (|r_l|^2 is not needed here: the next update 1 sums it before any check)
        rmax = 1.0;
      }
    }
    if (done) break;
  }
  st->iters = k;
  st->outer = outer;
  st->converged = rel <= o->tol;
  st->rel_resid = rel;
  st->n_Dbb = ndbb;
  return status;
}

// Upload the site-local matrices and sweep tables of the context's parameters
// (allocating the device tables on first use; their sizes depend on Ls only).
int upload_smatrices(dwa_ctx* ctx, const std::vector<double>& mix, const SweepTables& sweeps,
                     bool alloc) {
  std::vector<float> mix32(mix.begin(), mix.end());
  std::vector<float> sw32(sweeps.coef.begin(), sweeps.coef.end());
  if (alloc) {
    DWA_HIP(hipMalloc(&ctx->d_mix64, sizeof(double) * mix.size()), "alloc mix");
    DWA_HIP(hipMalloc(&ctx->d_mix32, sizeof(float) * mix.size()), "alloc mix32");
    DWA_HIP(hipMalloc(&ctx->d_sweep_meta, sizeof(int) * sweeps.meta.size()), "alloc sweep meta");
    DWA_HIP(hipMalloc(&ctx->d_sweep64, sizeof(double) * sweeps.coef.size()), "alloc sweep64");
    DWA_HIP(hipMalloc(&ctx->d_sweep32, sizeof(float) * sw32.size()), "alloc sweep32");
  }
  DWA_HIP(hipMemcpy(ctx->d_mix64, mix.data(), sizeof(double) * mix.size(), hipMemcpyHostToDevice), "upload mix");
  DWA_HIP(hipMemcpy(ctx->d_mix32, mix32.data(), sizeof(float) * mix32.size(), hipMemcpyHostToDevice), "upload mix32");
  DWA_HIP(hipMemcpy(ctx->d_sweep_meta, sweeps.meta.data(), sizeof(int) * sweeps.meta.size(), hipMemcpyHostToDevice),
          "upload sweep meta");
  DWA_HIP(hipMemcpy(ctx->d_sweep64, sweeps.coef.data(), sizeof(double) * sweeps.coef.size(), hipMemcpyHostToDevice),
          "upload sweep64");
  DWA_HIP(hipMemcpy(ctx->d_sweep32, sw32.data(), sizeof(float) * sw32.size(), hipMemcpyHostToDevice), "upload sweep32");
  ctx->h_mix = mix;
  ctx->sweep_meta_host = sweeps.meta;
  ctx->dense_mix = std::getenv("DWA_DENSE_MIX") != nullptr;
  for (size_t k = 0; k < sweeps.meta.size(); k += 4)
    if (sweeps.meta[k + 1] == ST_DENSE) ctx->dense_mix = true;
  return DWA_OK;
}

int check_ctx(dwa_ctx* ctx) {
  if (!ctx) return einval("null context");
  if (!ctx->links_set) {
    set_error("links not set (call dwa_set_links first)");
    return DWA_ESTATE;
  }
  return DWA_OK;
}


// ---------------------------------------------------------------------------
// Batches: nrhs fields of one context stored back to back (field_elems apart).

void free_batch(dwa_ctx* ctx) {
  BatchWs& b = ctx->batch;
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto p : b.f64) f(p);
  for (auto& row : b.lo)
    for (auto p : row) f(p);
  f(b.xacc);
  f(b.d_scal);
  f(b.partials);
  f(b.d_coef);
  if (b.h_scal) (void)hipHostFree(b.h_scal);
  if (b.h_coef) (void)hipHostFree(b.h_coef);
  if (b.h_active) (void)hipHostFree(b.h_active);
  if (b.stream) (void)hipStreamDestroy(b.stream);
  b = BatchWs{};
}

double* bbank(dwa_ctx* ctx, int i) {
  return ctx->batch.partials + size_t(i) * ctx->batch.nmax * ctx->batch.bank_elems;
}

// One batched CGLS system: nr fields of one context, all in storage precision prec.
struct BatchSys {
  dwa_ctx* ctx = nullptr;
  int nr = 0;
  int prec = DWA_F64;
  void* x = nullptr;          // solution (storage xacc_prec(prec))
  const void* rhs = nullptr;  // right-hand sides
  void *r = nullptr, *p = nullptr, *z = nullptr, *q = nullptr, *w = nullptr, *u = nullptr,
       *t = nullptr;
  std::vector<double> tol;    // per field; a field with tol < 0 starts frozen
  std::vector<int> iters, converged, breakdown;
  long long n_dbb = 0;
  int nb_r = 0;  // partial sums of |r|^2 per field in bank 1 (set by the first half)
  int nb_z = 0;  // partial sums of |z|^2 per field in bank 2 (set by the second half)
};

// Called at every host check (k > 0) for each system; last is set at maxiter.
using BatchHook = std::function<int(BatchSys&, int k, bool last)>;

void batch_sys_vectors(BatchSys& b) {
  BatchWs& w = b.ctx->batch;
  if (b.prec == DWA_F64) {
    b.r = w.f64[B_R]; b.p = w.f64[B_P]; b.z = w.f64[B_Z]; b.q = w.f64[B_Q];
    b.w = w.f64[B_W]; b.u = w.f64[B_U]; b.t = w.f64[B_T];
  } else {
    void** L = w.lo[b.prec];
    b.r = L[BL_R]; b.p = L[BL_P]; b.z = L[BL_Z]; b.q = L[BL_Q];
    b.w = L[BL_W]; b.u = L[BL_U]; b.t = L[BL_T];
  }
}

// Freeze field k of a system (host-driven: the finalize kernel then keeps x and r).
int batch_freeze(BatchSys& b, int k, hipStream_t st) {
  BatchWs& w = b.ctx->batch;
  w.h_active[k] = 0;
  DWA_HIP(hipMemcpyAsync(&w.d_scal[k].active, &w.h_active[k], sizeof(int), hipMemcpyHostToDevice, st),
          "active flag");
  return DWA_OK;
}

// The CGLS iteration is split at the point where the host looks at the scalars, right
// after x and r have been updated (as in the single-field reliable solver):
//   first half:  q = A p, a = gamma / |q|^2, x += a p, r -= a q, |r|^2 partials,
//                w = premix of r (|r|^2 itself is summed only before a host check)
//   second half: z = A^dag r, beta = |z|^2 / gamma, p = z + beta p, u = premix of p
// The scalars come from the partials inside the updates (no finalize launches): update 1
// sums |q|^2 (bank 0) and gamma = |z|^2 (bank 2), update 2 sums |z|^2 for beta.
// The graph body is (second half, first half); the first iteration runs its first half
// eagerly.  A host check after k bodies therefore sees the residual of k updates of x.
int batch_first_half(BatchSys& b) {
  dwa_ctx* ctx = b.ctx;
  DevScalars* sc = ctx->batch.d_scal;
  int nbA = 0, nbB = 0;
  DWA_TRY(dbb_from_premix(ctx, b.prec, b.q, b.p, b.u, b.t, bbank(ctx, 0), &nbA, b.nr));
  // a = gamma / |q|^2 per field is summed inside update 1 from the hop's partials
  DWA_TRY(launch_cg_update1(ctx, b.prec, b.x, b.r, b.w, b.p, b.q, sc, bbank(ctx, 1), &nbB, false, b.nr,
                            bbank(ctx, 0), nbA, bbank(ctx, 2), b.nb_z));
  b.nb_r = nbB;  // |r|^2 partials: summed into rr only before a host check
  b.n_dbb += b.nr;
  return DWA_OK;
}

int batch_second_half(BatchSys& b) {
  dwa_ctx* ctx = b.ctx;
  DevScalars* sc = ctx->batch.d_scal;
  int nbZ = 0;
  DWA_TRY(dbbdag_from_premix(ctx, b.prec, b.z, b.r, b.w, b.t, bbank(ctx, 2), &nbZ, b.nr));
  b.nb_z = nbZ;
  DWA_TRY(launch_cg_update2(ctx, b.prec, b.p, b.u, b.z, sc, false, b.nr, bbank(ctx, 2), nbZ));
  b.n_dbb += b.nr;
  return DWA_OK;
}

// The replayed body: one iteration of every system in L.
int batch_body(const std::vector<BatchSys*>& L) {
  for (auto* b : L) {
    DWA_TRY(batch_second_half(*b));
    DWA_TRY(batch_first_half(*b));
  }
  return DWA_OK;
}

// CGLS on every field of every system at once.  All work runs on stream st (the
// contexts' streams point at it for the duration).  Between host checks the iteration
// body of the systems with a live field is replayed from one hipGraph (no memset nodes:
// kernels only); a system whose fields have all stopped leaves the body, and the graph
// is captured again without it (its kernels would otherwise keep running with zero step
// lengths: 3-5% of the time of the 3-lattice workload, whose lattices stop at 145, 300
// and 345 iterations).
// Host checks come every check_every iterations.  Without a hook a field stops (is
// frozen on the device) when its recursive residual reaches its tolerance.  With a
// hook, the hook decides at every check (reliable updates): it is called once per
// system with the scalars of its fields on the host.  Iteration counts are those of
// the check at which a field stopped.
int cgls_multi(std::vector<BatchSys>& S, hipStream_t st, int maxiter, int check_every,
               bool use_graph, const BatchHook& hook) {
  if (check_every < 1) check_every = 1;
  for (auto& b : S) {
    dwa_ctx* ctx = b.ctx;
    const size_t n = field_elems(ctx);
    DevScalars* sc = ctx->batch.d_scal;
    int nbA = 0, nbB = 0;
    b.iters.assign(b.nr, 0);
    b.converged.assign(b.nr, 0);
    b.breakdown.assign(b.nr, 0);
    DWA_TRY(launch_zero(ctx, xacc_prec(b.prec), b.x, n, b.nr));
    DWA_TRY(launch_axpby(ctx, b.prec, b.r, 1.0, b.rhs, 0.0, n, b.nr));
    DWA_TRY(launch_smix(ctx, b.prec, MIX_G5_IINVT_GINV, b.w, b.r, nullptr, 0.0, ctx->Ls, nullptr, nullptr, b.nr));
    DWA_TRY(dbbdag_from_premix(ctx, b.prec, b.z, b.r, b.w, b.t, bbank(ctx, 2), &nbA, b.nr));
    b.nb_z = nbA;
    DWA_TRY(launch_norm2(ctx, b.prec, b.rhs, n, bbank(ctx, 1), &nbB, b.nr));
    DWA_TRY(launch_cg_finalize(ctx, 2, sc, bbank(ctx, 2), nbA, bbank(ctx, 1), nbB, b.nr));
    DWA_TRY(launch_axpby(ctx, b.prec, b.p, 1.0, b.z, 0.0, n, b.nr));
    DWA_TRY(launch_smix(ctx, b.prec, MIX_BG, b.u, b.p, nullptr, 0.0, ctx->Ls, nullptr, nullptr, b.nr));
    b.n_dbb = b.nr;
    for (int k = 0; k < b.nr; ++k) {
      ctx->batch.h_active[k] = 1;
      if (b.tol[k] < 0.0) {
        DWA_TRY(batch_freeze(b, k, st));
        b.converged[k] = 1;
      }
    }
  }
  if (std::getenv("DWA_BATCH_NO_GRAPH")) use_graph = false;  // eager replay (diagnostics)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  // the systems with a live field (the body's systems); true when the set changed
  std::vector<BatchSys*> live;
  auto refresh_live = [&]() -> bool {
    std::vector<BatchSys*> now;
    for (auto& b : S)
      for (int f = 0; f < b.nr; ++f)
        if (b.ctx->batch.h_active[f]) {
          now.push_back(&b);
          break;
        }
    const bool changed = now != live;
    live = std::move(now);
    return changed;
  };
  auto body = [&]() -> int {
    if (!use_graph) return batch_body(live);
    if (!exec) {
      DWA_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
      const int rc = batch_body(live);
      const hipError_t e = hipStreamEndCapture(st, &graph);
      DWA_TRY(rc);
      DWA_HIP(e, "end capture");
      DWA_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
      // the capture counted one iteration per system; the replays count themselves
      for (auto* b : live) b->n_dbb -= 2LL * b->nr;
    }
    DWA_HIP(hipGraphLaunch(exec, st), "graph launch");
    for (auto* b : live) b->n_dbb += 2LL * b->nr;
    return DWA_OK;
  };
  int k = 0;
  for (;;) {
    // host check: |r|^2 of the last update (after the first iteration; before it the
    // set-up's rr = |rhs|^2 stands), then every system's scalars
    int active = 0;
    for (auto& b : S) {
      BatchWs& w = b.ctx->batch;
      if (k > 0) {
        const int rc = launch_cg_finalize(b.ctx, 4, w.d_scal, bbank(b.ctx, 1), b.nb_r, nullptr, 0, b.nr);
        if (rc != DWA_OK) {
          cleanup();
          return rc;
        }
      }
      const hipError_t e = hipMemcpyAsync(w.h_scal, w.d_scal, sizeof(DevScalars) * b.nr,
                                          hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "batch scalar readback");
      }
    }
    {
      const hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "batch sync");
      }
    }
    for (auto& b : S) {
      BatchWs& w = b.ctx->batch;
      for (int f = 0; f < b.nr; ++f) {
        if (!w.h_active[f]) continue;
        const DevScalars& h = w.h_scal[f];
        bool stop = false;
        if (h.flags) {
          b.breakdown[f] = 1;
          stop = true;
        } else if (!hook && (h.b2 == 0.0 || h.rr <= b.tol[f] * b.tol[f] * h.b2)) {
          b.converged[f] = 1;
          stop = true;
        }
        if (stop) {
          b.iters[f] = k;
          const int rc = batch_freeze(b, f, st);
          if (rc != DWA_OK) {
            cleanup();
            return rc;
          }
        }
      }
      if (hook && k > 0) {
        const int rc = hook(b, k, k >= maxiter);
        if (rc != DWA_OK) {
          cleanup();
          return rc;
        }
      }
      for (int f = 0; f < b.nr; ++f) active += w.h_active[f] ? 1 : 0;
    }
    if (active == 0 || k >= maxiter) break;
    if (refresh_live()) cleanup();  // capture the body again for the systems still live
    if (k == 0) {
      // first half of the first iteration, eagerly; the body is captured at its first run
      for (auto* b : live) {
        const int rc = batch_first_half(*b);
        if (rc != DWA_OK) {
          cleanup();
          return rc;
        }
      }
      k = 1;
    } else {
      const int rc = body();
      if (rc != DWA_OK) {
        cleanup();
        return rc;
      }
      ++k;
    }
    while (k % check_every != 0 && k < maxiter) {
      const int rc = body();
      if (rc != DWA_OK) {
        cleanup();
        return rc;
      }
      ++k;
    }
  }
  for (auto& b : S)
    for (int f = 0; f < b.nr; ++f)
      if (b.ctx->batch.h_active[f]) b.iters[f] = k;  // stopped by maxiter
  cleanup();
  return DWA_OK;
}

// Per-field |v|^2 of a batch (synchronising on st).
int batch_norms(dwa_ctx* ctx, int prec, const void* v, int nr, hipStream_t st, double* out) {
  int nb = 0;
  DWA_TRY(launch_norm2(ctx, prec, v, field_elems(ctx), bbank(ctx, 3), &nb, nr));
  std::vector<double> h(size_t(nb) * nr);
  DWA_HIP(hipMemcpyAsync(h.data(), bbank(ctx, 3), sizeof(double) * h.size(), hipMemcpyDeviceToHost, st),
          "batch norm readback");
  DWA_HIP(hipStreamSynchronize(st), "batch norm sync");
  for (int f = 0; f < nr; ++f) {
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) acc += h[size_t(f) * nb + i];
    out[f] = acc;
  }
  return DWA_OK;
}

// RES = PHI - D_bb X for every field (FP64) and its norms.
int batch_true_residual(dwa_ctx* ctx, int nr, hipStream_t st, double* res2) {
  BatchWs& w = ctx->batch;
  const size_t n = field_elems(ctx);
  DWA_TRY(apply_dbb(ctx, DWA_F64, w.f64[B_Q], w.f64[B_X], w.f64[B_OPB], w.f64[B_OPR], nr));
  int nb = 0;
  DWA_TRY(launch_residual(ctx, w.f64[B_RES], w.f64[B_PHI], w.f64[B_Q], n, bbank(ctx, 3), &nb, nr));
  std::vector<double> h(size_t(nb) * nr);
  DWA_HIP(hipMemcpyAsync(h.data(), bbank(ctx, 3), sizeof(double) * h.size(), hipMemcpyDeviceToHost, st),
          "batch residual readback");
  DWA_HIP(hipStreamSynchronize(st), "batch residual sync");
  for (int f = 0; f < nr; ++f) {
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) acc += h[size_t(f) * nb + i];
    res2[f] = acc;
  }
  return DWA_OK;
}

// Result of a batched solve of D_bb X = PHI over several contexts (per context, per
// field): FP64 relative residual of the last recomputation (mixed precision), |PHI|,
// CG iterations, FP64 residual recomputations, and (FP64 inner solves) whether the
// recursive residual met the tolerance.
struct MultiSolve {
  std::vector<std::vector<double>> rel, bnorm;
  std::vector<std::vector<int>> iters, outer, fp64_conv;
};

// Solve D_bb X = PHI (CGNE, Sec. 3) for the nrhs[i] fields held in the batch workspace of
// every context (B_PHI -> B_X, FP64 black SoA), all on stream st: FP64 CGLS, or
// low-precision CGLS with FP64 reliable updates or defect correction (opts).
int multi_solve(dwa_ctx* const* ctxs, int nctx, const int* nrhs, const dwa_solve_opts* o,
                hipStream_t st, MultiSolve& M) {
  const int inner = o->inner_prec;
  auto& rel = M.rel;
  auto& bnorm = M.bnorm;
  auto& iters = M.iters;
  auto& outer = M.outer;
  auto& fp64_conv = M.fp64_conv;
  rel.assign(nctx, {});
  bnorm.assign(nctx, {});
  iters.assign(nctx, {});
  outer.assign(nctx, {});
  fp64_conv.assign(nctx, {});
  for (int i = 0; i < nctx; ++i) {
    rel[i].assign(nrhs[i], 1.0);
    bnorm[i].assign(nrhs[i], 0.0);
    iters[i].assign(nrhs[i], 0);
    outer[i].assign(nrhs[i], 0);
    DWA_TRY(batch_norms(ctxs[i], DWA_F64, ctxs[i]->batch.f64[B_PHI], nrhs[i], st, bnorm[i].data()));
    for (auto& v : bnorm[i]) v = std::sqrt(v);
  }
  if (inner == DWA_F64) {
    std::vector<BatchSys> S(nctx);
    for (int i = 0; i < nctx; ++i) {
      S[i].ctx = ctxs[i];
      S[i].nr = nrhs[i];
      S[i].prec = DWA_F64;
      S[i].x = ctxs[i]->batch.f64[B_X];
      S[i].rhs = ctxs[i]->batch.f64[B_PHI];
      S[i].tol.assign(nrhs[i], o->tol);
      batch_sys_vectors(S[i]);
    }
    DWA_TRY(cgls_multi(S, st, o->maxiter, o->check_every, true, BatchHook{}));
    for (int i = 0; i < nctx; ++i) {
      iters[i] = S[i].iters;
      fp64_conv[i] = S[i].converged;
    }
  } else if (o->mixed_mode != DWA_MIXED_DEFECT) {
    // reliable updates: one low-precision CGLS per field for the whole solve, the
    // scheme of the single-field solver.  At a host check where some field of a
    // context has reduced its low-precision residual by delta (or is predicted to
    // have converged), every live field of that context folds x_l into X, gets its
    // true FP64 residual, and continues from it at unit norm with p and gamma
    // rescaled.  (One batched FP64 D_bb serves all fields of the context, so they
    // are updated together.)
    const double delta = (o->delta > 0.0 && o->delta < 1.0) ? o->delta : 0.1;
    std::vector<std::vector<double>> scale(nctx), rmax(nctx), last(nctx);
    std::vector<std::vector<int>> stall(nctx);
    std::vector<BatchSys> S(nctx);
    for (int i = 0; i < nctx; ++i) {
      dwa_ctx* ctx = ctxs[i];
      BatchWs& w = ctx->batch;
      const int nr = nrhs[i];
      const size_t n = field_elems(ctx);
      scale[i] = bnorm[i];
      rmax[i].assign(nr, 1.0);
      last[i].assign(nr, 1.0);
      stall[i].assign(nr, 0);
      DWA_TRY(launch_zero(ctx, DWA_F64, w.f64[B_X], n, nr));
      S[i].ctx = ctx;
      S[i].nr = nr;
      S[i].prec = inner;
      S[i].x = w.xacc;
      S[i].rhs = w.lo[inner][BL_RHS];
      S[i].tol.assign(nr, 0.0);
      for (int f = 0; f < nr; ++f) {
        w.h_coef[f] = bnorm[i][f] > 0.0 ? 1.0 / bnorm[i][f] : 0.0;
        if (bnorm[i][f] == 0.0) {
          S[i].tol[f] = -1.0;
          rel[i][f] = 0.0;
        }
      }
      batch_sys_vectors(S[i]);
      DWA_HIP(hipMemcpyAsync(w.d_coef, w.h_coef, sizeof(double) * nr, hipMemcpyHostToDevice, st), "coef upload");
      DWA_TRY(launch_convert(ctx, inner, w.lo[inner][BL_RHS], DWA_F64, w.f64[B_PHI], n, 0.0, nr, w.d_coef));
      // the pinned coefficients are rewritten below only after a synchronisation
      DWA_HIP(hipStreamSynchronize(st), "coef sync");
    }
    const BatchHook hook = [&](BatchSys& b, int k, bool at_end) -> int {
      const int i = int(&b - S.data());
      dwa_ctx* ctx = b.ctx;
      BatchWs& w = ctx->batch;
      const int nr = b.nr;
      const size_t n = field_elems(ctx);
      bool trig = at_end;
      for (int f = 0; f < nr; ++f) {
        if (!w.h_active[f]) continue;
        const double rl = std::sqrt(w.h_scal[f].rr);
        if (rl <= delta * rmax[i][f] || rl * scale[i][f] / bnorm[i][f] <= 0.5 * o->tol) trig = true;
      }
      if (!trig) return DWA_OK;
      // X += scale x_l (FP64) for the live fields, x_l = 0, true residuals
      std::vector<int> live(nr);
      for (int f = 0; f < nr; ++f) {
        live[f] = w.h_active[f];
        w.h_coef[f] = live[f] ? scale[i][f] : 0.0;
      }
      DWA_HIP(hipMemcpyAsync(w.d_coef, w.h_coef, sizeof(double) * nr, hipMemcpyHostToDevice, st), "coef upload");
      DWA_TRY(launch_fold_acc(ctx, xacc_prec(inner), w.f64[B_X], w.xacc, n, 0.0, nr, w.d_coef));
      std::vector<double> r2(nr);
      DWA_TRY(batch_true_residual(ctx, nr, st, r2.data()));  // synchronises
      std::vector<double> fac(nr, 1.0);
      for (int f = 0; f < nr; ++f) {
        if (!live[f]) continue;
        const double r = std::sqrt(r2[f]) / bnorm[i][f];
        rel[i][f] = r;
        outer[i][f] += 1;
        bool stop = false;
        if (r <= o->tol) {
          b.converged[f] = 1;
          stop = true;
        } else {
          if (!(r < 0.9 * last[i][f])) stop = ++stall[i][f] >= 3;
          else stall[i][f] = 0;
          last[i][f] = r;
        }
        if (stop) {
          b.iters[f] = k;
          DWA_TRY(batch_freeze(b, f, st));
          continue;
        }
        const double ns = r * bnorm[i][f];
        fac[f] = scale[i][f] / ns;
        scale[i][f] = ns;
        rmax[i][f] = 1.0;
      }
      // continue in the new units: p *= fac, gamma *= fac^2, r_l = RES / scale
      for (int f = 0; f < nr; ++f) {
        w.h_coef[2 * f] = fac[f];
        w.h_coef[2 * f + 1] = 0.0;
        w.h_coef[2 * nr + f] = fac[f] * fac[f];
        // a zero source has scale 0 (frozen from the start): keep its r at 0
        w.h_coef[3 * nr + f] = scale[i][f] > 0.0 ? 1.0 / scale[i][f] : 0.0;
      }
      DWA_HIP(hipMemcpyAsync(w.d_coef, w.h_coef, sizeof(double) * 4 * nr, hipMemcpyHostToDevice, st),
              "coef upload");
      DWA_TRY(launch_axpby(ctx, inner, b.p, 1.0, b.p, 0.0, n, nr, w.d_coef));
      DWA_TRY(launch_scale_gamma(ctx, w.d_scal, 1.0, nr, w.d_coef + 2 * nr));
      DWA_TRY(launch_convert(ctx, inner, b.r, DWA_F64, w.f64[B_RES], n, 0.0, nr, w.d_coef + 3 * nr));
      DWA_TRY(launch_smix(ctx, inner, MIX_G5_IINVT_GINV, b.w, b.r, nullptr, 0.0, ctx->Ls, nullptr, nullptr, nr));
      DWA_HIP(hipStreamSynchronize(st), "coef sync");
      return DWA_OK;
    };
    DWA_TRY(cgls_multi(S, st, o->maxiter, o->check_every, true, hook));
    for (int i = 0; i < nctx; ++i) iters[i] = S[i].iters;
  } else {
    // defect correction: FP64 residuals, one batched low-precision CGLS per round
    const double delta = (o->delta > 0.0 && o->delta < 1.0) ? o->delta : 0.1;
    std::vector<std::vector<int>> stall(nctx);
    std::vector<std::vector<double>> prev(nctx);
    for (int i = 0; i < nctx; ++i) {
      BatchWs& w = ctxs[i]->batch;
      const size_t n = field_elems(ctxs[i]);
      DWA_TRY(launch_zero(ctxs[i], DWA_F64, w.f64[B_X], n, nrhs[i]));
      DWA_TRY(launch_axpby(ctxs[i], DWA_F64, w.f64[B_RES], 1.0, w.f64[B_PHI], 0.0, n, nrhs[i]));
      stall[i].assign(nrhs[i], 0);
      prev[i].assign(nrhs[i], 1.0);
      for (int f = 0; f < nrhs[i]; ++f)
        if (bnorm[i][f] == 0.0) rel[i][f] = 0.0;
    }
    int total = 0;
    for (;;) {
      // one batched low-precision CGLS over the contexts that still have live fields
      std::vector<BatchSys> S;
      std::vector<int> which;
      for (int i = 0; i < nctx; ++i) {
        dwa_ctx* ctx = ctxs[i];
        BatchWs& w = ctx->batch;
        const int nr = nrhs[i];
        const size_t n = field_elems(ctx);
        BatchSys b;
        b.ctx = ctx;
        b.nr = nr;
        b.prec = inner;
        b.x = w.xacc;
        b.rhs = w.lo[inner][BL_RHS];
        b.tol.assign(nr, -1.0);
        batch_sys_vectors(b);
        bool live_any = false;
        for (int f = 0; f < nr; ++f) {
          const bool live = rel[i][f] > o->tol && stall[i][f] < 3;
          w.h_coef[f] = live ? 1.0 / (rel[i][f] * bnorm[i][f]) : 0.0;
          if (live) {
            b.tol[f] = std::max(delta, 0.5 * o->tol / rel[i][f]);
            live_any = true;
          }
        }
        if (!live_any) continue;
        // right-hand sides r / |r| in the inner storage precision
        DWA_HIP(hipMemcpyAsync(w.d_coef, w.h_coef, sizeof(double) * nr, hipMemcpyHostToDevice, st), "coef upload");
        DWA_TRY(launch_convert(ctx, inner, w.lo[inner][BL_RHS], DWA_F64, w.f64[B_RES], n, 0.0, nr, w.d_coef));
        S.push_back(std::move(b));
        which.push_back(i);
      }
      if (S.empty() || total >= o->maxiter) break;
      DWA_TRY(cgls_multi(S, st, o->maxiter - total, o->check_every, true, BatchHook{}));
      int round_max = 0;
      for (size_t j = 0; j < S.size(); ++j) {
        const int i = which[j];
        dwa_ctx* ctx = ctxs[i];
        BatchWs& w = ctx->batch;
        const int nr = nrhs[i];
        const size_t n = field_elems(ctx);
        for (int f = 0; f < nr; ++f) {
          const bool live = S[j].tol[f] >= 0.0;
          w.h_coef[f] = live ? rel[i][f] * bnorm[i][f] : 0.0;
          if (live) {
            iters[i][f] += S[j].iters[f];
            outer[i][f] += 1;
            round_max = std::max(round_max, S[j].iters[f]);
          }
        }
        // X += |r| e in FP64, then the new residuals
        DWA_HIP(hipMemcpyAsync(w.d_coef, w.h_coef, sizeof(double) * nr, hipMemcpyHostToDevice, st), "coef upload");
        DWA_TRY(launch_fold_acc(ctx, xacc_prec(inner), w.f64[B_X], w.xacc, n, 0.0, nr, w.d_coef));
        std::vector<double> r2(nr);
        DWA_TRY(batch_true_residual(ctx, nr, st, r2.data()));
        for (int f = 0; f < nr; ++f) {
          if (S[j].tol[f] < 0.0) continue;
          const double r = bnorm[i][f] > 0.0 ? std::sqrt(r2[f]) / bnorm[i][f] : 0.0;
          if (!(r < 0.9 * prev[i][f])) stall[i][f] += 1;
          else stall[i][f] = 0;
          prev[i][f] = r;
          rel[i][f] = r;
        }
      }
      total += std::max(round_max, 1);
    }
  }
  return DWA_OK;
}

}  // namespace

extern "C" {

const char* dwa_strerror(int status) {
  switch (status) {
    case DWA_OK: return "ok";
    case DWA_EINVAL: return "invalid argument";
    case DWA_ENOMEM: return "device out of memory";
    case DWA_EHIP: return "HIP runtime error";
    case DWA_ENOCONV: return "solver did not converge";
    case DWA_EBREAKDOWN: return "CG breakdown";
    case DWA_ENAN: return "non-finite input";
    case DWA_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* dwa_last_error(void) { return dwa::g_last_error.c_str(); }

int dwa_create(dwa_ctx** out, const dwa_params* p, void* stream) {
  if (!out) return einval("null output pointer");
  *out = nullptr;
  if (!p) return einval("null params");
  for (int d = 0; d < 4; ++d)
    if (p->dims[d] < 2 || (p->dims[d] & 1))
      return einval("every lattice extent must be even and >= 2");
  if (p->Ls < 2 || p->Ls > 32) return einval("Ls must be in [2, 32]");
  if (!p->b || !p->c) return einval("null b or c");
  if (!std::isfinite(p->alpha) || p->alpha == 0.0) return einval("alpha must be finite and non-zero");
  if (!std::isfinite(p->M5) || !std::isfinite(p->m)) return einval("M5 and m must be finite");
  for (int s = 0; s < p->Ls; ++s)
    if (!std::isfinite(p->b[s]) || !std::isfinite(p->c[s])) return einval("b, c must be finite");
  const long long V = (long long)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
  // kernels address one FP64 half field (Ls * 12 * V/2 complex numbers of 16 bytes)
  // with 32-bit byte offsets
  if ((long long)p->Ls * 12 * (V / 2) * 16 >= (1LL << 32))
    return einval("lattice too large: an FP64 half field must stay below 4 GiB");
  std::vector<double> mix;
  std::string err;
  SweepTables sweeps;
  if (!build_smatrices(p->Ls, p->M5, p->m, p->alpha, p->b, p->c, mix, err, &sweeps))
    return einval(err);

  dwa_ctx* ctx = new dwa_ctx();
  for (int d = 0; d < 4; ++d) ctx->dims[d] = p->dims[d];
  ctx->Ls = p->Ls;
  ctx->V = V;
  ctx->Vh = V / 2;
  ctx->M5 = p->M5;
  ctx->m = p->m;
  ctx->alpha = p->alpha;
  ctx->b.assign(p->b, p->b + p->Ls);
  ctx->c.assign(p->c, p->c + p->Ls);
  ctx->antiperiodic_t = p->antiperiodic_t ? 1 : 0;
  ctx->stream = (hipStream_t)stream;
  ctx->h_mix = mix;

  auto fail = [&](int rc) {
    dwa_destroy(ctx);
    return rc;
  };
  int rc = hip_fail(hipGetDevice(&ctx->device), "hipGetDevice");
  if (rc) return fail(rc);
  if ((rc = scratch_init(ctx->device))) return fail(rc);
  if ((rc = hip_fail(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "solve stream")))
    return fail(rc);

  // geometry: checkerboard <-> lexicographic and neighbour tables
  const int Lx = p->dims[0], Ly = p->dims[1], Lz = p->dims[2], Lt = p->dims[3];
  const long long Vh = ctx->Vh;
  std::vector<int> cb2lex(2 * Vh), nbr(size_t(16) * Vh);
  for (long long lex = 0; lex < V; ++lex) {
    long long r = lex;
    int x = r % Lx; r /= Lx;
    int y = r % Ly; r /= Ly;
    int z = r % Lz;
    int t = (int)(r / Lz);
    int par = (x + y + z + t) & 1;
    cb2lex[par * Vh + lex / 2] = (int)lex;
  }
  for (int par = 0; par < 2; ++par)
    for (long long cb = 0; cb < Vh; ++cb) {
      long long lex = cb2lex[par * Vh + cb];
      long long r = lex;
      int c4[4];
      c4[0] = r % Lx; r /= Lx;
      c4[1] = r % Ly; r /= Ly;
      c4[2] = r % Lz;
      c4[3] = (int)(r / Lz);
      for (int dir = 0; dir < 8; ++dir) {
        int mu = dir & 3, step = dir < 4 ? 1 : -1;
        int n4[4] = {c4[0], c4[1], c4[2], c4[3]};
        n4[mu] = (n4[mu] + step + p->dims[mu]) % p->dims[mu];
        long long nlex = n4[0] + (long long)Lx * (n4[1] + (long long)Ly * (n4[2] + (long long)Lz * n4[3]));
        nbr[(size_t(par) * 8 + dir) * Vh + cb] = (int)(nlex / 2);
      }
    }
  if ((rc = hip_fail(hipMalloc(&ctx->d_cb2lex, sizeof(int) * cb2lex.size()), "alloc cb2lex")))
    return fail(rc);
  if ((rc = hip_fail(hipMalloc(&ctx->d_nbr, sizeof(int) * nbr.size()), "alloc nbr"))) return fail(rc);
  if ((rc = hip_fail(hipMemcpy(ctx->d_cb2lex, cb2lex.data(), sizeof(int) * cb2lex.size(),
                               hipMemcpyHostToDevice), "upload cb2lex")))
    return fail(rc);
  if ((rc = hip_fail(hipMemcpy(ctx->d_nbr, nbr.data(), sizeof(int) * nbr.size(),
                               hipMemcpyHostToDevice), "upload nbr")))
    return fail(rc);
  // fused-hop traversals: chunks of NS consecutive checkerboard sites in one of three
  // orders (HopOrder); contiguous ranges of the order go to one XCD (the kernel remaps
  // block ids accordingly).  SLAB walks (t-slab, z, t within the slab, y, x) so that a
  // run of blocks on one XCD touches a compact slab and the t and z neighbours are
  // re-read from L2, not HBM.  One table per order and tile size.
  for (int ord = 0; ord < ORDER_COUNT; ++ord)
    for (int bi = 0; bi < kTileCount; ++bi) {
      const int NS = kTiles[bi];
      const long long nchunk = (Vh + NS - 1) / NS;
      std::vector<int> order(nchunk);
      for (long long c = 0; c < nchunk; ++c) order[c] = (int)c;
      if (ord != ORDER_LEX) {
        const bool zdom = ord == ORDER_ZDOM && Lz % 8 == 0;
        const int ts = Lt >= 16 ? Lt / 8 : 1;
        const int zpd = Lz / 8;
        std::vector<long long> key(nchunk);
        for (long long c = 0; c < nchunk; ++c) {
          long long r = cb2lex[c * NS];
          const long long x = r % Lx; r /= Lx;
          const long long y = r % Ly; r /= Ly;
          const long long z = r % Lz;
          const long long t = r / Lz;
          key[c] = zdom ? ((((z / zpd) * Lt + t) * zpd + z % zpd) * Ly + y) * Lx + x
                        : ((((t / ts) * Lz + z) * ts + (t % ts)) * Ly + y) * Lx + x;
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
      }
      int*& d = ctx->d_blkmap[ord][bi];
      if ((rc = hip_fail(hipMalloc(&d, sizeof(int) * order.size()), "alloc blkmap"))) return fail(rc);
      if ((rc = hip_fail(hipMemcpy(d, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice),
                         "upload blkmap")))
        return fail(rc);
    }
  // default tuning: 32 sites per block for FP32 / BF16 (one 128-byte line per colour-
  // spin component and slice), 16 for FP64 (whose LDS tile is twice as large), slab
  // order; DWA_HOP_ORDER=slab|lex|zdom overrides the order (dwa_autotune replaces both)
  {
    int ord = ORDER_SLAB;
    if (const char* e = std::getenv("DWA_HOP_ORDER"))
      ord = std::string(e) == "lex" ? ORDER_LEX : (std::string(e) == "zdom" ? ORDER_ZDOM : ORDER_SLAB);
    for (int pr = 0; pr < 3; ++pr) {
      ctx->tune[pr].ns = pr == DWA_F64 ? 16 : 32;
      ctx->tune[pr].order = ord;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) == hipSuccess &&
        lds > 0)
      ctx->max_lds = size_t(lds);
  }
  // s-matrices
  if ((rc = upload_smatrices(ctx, mix, sweeps, true))) return fail(rc);
  if (const char* e = std::getenv("DWA_HOP_MIN_LDS_KB"))
    ctx->hop_min_lds = std::min<size_t>(size_t(std::max(0, std::atoi(e))) * 1024, 160 * 1024);
  // links and workspace
  const size_t n = field_elems(ctx);
  for (int pr = 0; pr < 3; ++pr)
    if ((rc = hip_fail(hipMalloc(&ctx->prec[pr].links, elem_bytes(pr) * 2 * 4 * 9 * Vh), "alloc links")))
      return fail(rc);
  for (int i = 0; i < W64_COUNT; ++i)
    if ((rc = hip_fail(hipMalloc(&ctx->w64[i], 16 * n), "alloc fp64 workspace"))) return fail(rc);
  for (int i = 0; i < LOW_COUNT; ++i) {
    if ((rc = hip_fail(hipMalloc(&ctx->w32[i], 8 * n), "alloc fp32 workspace"))) return fail(rc);
    if ((rc = hip_fail(hipMalloc(&ctx->w16[i], 4 * n), "alloc bf16 workspace"))) return fail(rc);
  }
  ctx->partials_per_bank = size_t(Vh) + 8192;
  if ((rc = hip_fail(hipMalloc(&ctx->d_partials, sizeof(double) * kBanks * ctx->partials_per_bank), "alloc partials")))
    return fail(rc);
  if ((rc = hip_fail(hipMalloc(&ctx->d_scal, sizeof(DevScalars)), "alloc scalars"))) return fail(rc);
  if ((rc = hip_fail(hipHostMalloc(&ctx->h_scal, sizeof(DevScalars), hipHostMallocDefault), "alloc pinned")))
    return fail(rc);
  if ((rc = hip_fail(hipMalloc(&ctx->d_red, sizeof(double) * 8), "alloc red"))) return fail(rc);
  if ((rc = hip_fail(hipMemset(ctx->d_scal, 0, sizeof(DevScalars)), "clear scalars"))) return fail(rc);
  *out = ctx;
  return DWA_OK;
}

int dwa_destroy(dwa_ctx* ctx) {
  if (!ctx) return DWA_OK;
  free_batch(ctx);
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(ctx->d_nbr);
  f(ctx->d_cb2lex);
  for (auto& row : ctx->d_blkmap)
    for (auto p : row) f(p);
  f(ctx->d_mix64);
  f(ctx->d_mix32);
  f(ctx->d_sweep_meta);
  f(ctx->d_sweep64);
  f(ctx->d_sweep32);
  for (auto& pr : ctx->prec) f(pr.links);
  for (auto p : ctx->w64) f(p);
  for (auto p : ctx->w32) f(p);
  for (auto p : ctx->w16) f(p);
  f(ctx->d_partials);
  f(ctx->d_scal);
  f(ctx->d_red);
  if (ctx->h_scal) (void)hipHostFree(ctx->h_scal);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return DWA_OK;
}

int dwa_set_alpha(dwa_ctx* ctx, double alpha) {
  if (!ctx) return einval("null context");
  if (!std::isfinite(alpha) || alpha == 0.0) return einval("alpha must be finite and non-zero");
  std::vector<double> mix;
  std::string err;
  SweepTables sweeps;
  if (!build_smatrices(ctx->Ls, ctx->M5, ctx->m, alpha, ctx->b.data(), ctx->c.data(), mix, err, &sweeps))
    return einval(err);
  // work already queued may read the current tables
  DWA_HIP(hipStreamSynchronize(ctx->stream), "set_alpha sync");
  DWA_TRY(upload_smatrices(ctx, mix, sweeps, false));
  ctx->alpha = alpha;
  return DWA_OK;
}

int dwa_set_links(dwa_ctx* ctx, const void* U) {
  if (!ctx) return einval("null context");
  if (!U) return einval("null links");
  for (int pr = 0; pr < 3; ++pr) DWA_TRY(launch_pack_links(ctx, pr, ctx->prec[pr].links, U));
  DWA_HIP(hipStreamSynchronize(ctx->stream), "set links sync");
  ctx->links_set = true;
  return DWA_OK;
}

size_t dwa_field_bytes(const dwa_ctx* ctx, int prec, int nrhs) {
  if (!ctx || !valid_prec(prec) || nrhs < 1) return 0;
  return elem_bytes(prec) * field_elems(ctx) * size_t(nrhs);
}

int dwa_get_sizes(const dwa_ctx* ctx, long long* V, int* Ls) {
  if (!ctx) return einval("null context");
  if (V) *V = ctx->V;
  if (Ls) *Ls = ctx->Ls;
  return DWA_OK;
}

int dwa_pack_spinor5(dwa_ctx* ctx, int prec, void* dst, const void* src, int parity) {
  if (!ctx) return einval("null context");
  if (!dst || !src) return einval("null field");
  if (!valid_prec(prec)) return einval("bad precision");
  if (parity != 0 && parity != 1) return einval("parity must be 0 or 1");
  return launch_pack5(ctx, prec, dst, src, parity, ctx->Ls);
}

int dwa_unpack_spinor5(dwa_ctx* ctx, int prec, void* dst, const void* src, int parity) {
  if (!ctx) return einval("null context");
  if (!dst || !src) return einval("null field");
  if (!valid_prec(prec)) return einval("bad precision");
  if (parity != 0 && parity != 1) return einval("parity must be 0 or 1");
  return launch_unpack5(ctx, prec, dst, src, parity, ctx->Ls);
}

int dwa_apply_Dw(dwa_ctx* ctx, void* out, const void* in, int nslices) {
  DWA_TRY(check_ctx(ctx));
  if (!out || !in) return einval("null field");
  if (nslices < 1) return einval("nslices must be >= 1");
  void** W = ctx->w64;
  const size_t vol12 = size_t(ctx->V) * 12;
  for (int s0 = 0; s0 < nslices; s0 += ctx->Ls) {
    const int ns = (nslices - s0) < ctx->Ls ? (nslices - s0) : ctx->Ls;
    const double2* src = (const double2*)in + s0 * vol12;
    double2* dst = (double2*)out + s0 * vol12;
    DWA_TRY(launch_pack5(ctx, DWA_F64, W[W_OPB], src, 0, ns));
    DWA_TRY(launch_pack5(ctx, DWA_F64, W[W_OPR], src, 1, ns));
    // out_p = (4 + M5) in_p - 1/2 H in_{1-p}
    HopOp hb{W[W_OPR], W[W_CHI_B], W[W_OPB], nullptr, -0.5, 4.0 + ctx->M5, 0.0, MIX_IDENTITY, 0, ns, nullptr};
    HopOp hr{W[W_OPB], W[W_CHI_R], W[W_OPR], nullptr, -0.5, 4.0 + ctx->M5, 0.0, MIX_IDENTITY, 1, ns, nullptr};
    DWA_TRY(launch_hop(ctx, DWA_F64, hb, nullptr));
    DWA_TRY(launch_hop(ctx, DWA_F64, hr, nullptr));
    DWA_TRY(launch_unpack5(ctx, DWA_F64, dst, W[W_CHI_B], 0, ns));
    DWA_TRY(launch_unpack5(ctx, DWA_F64, dst, W[W_CHI_R], 1, ns));
  }
  return DWA_OK;
}

int dwa_apply_Dbb(dwa_ctx* ctx, int prec, void* out, const void* in) {
  DWA_TRY(check_ctx(ctx));
  if (!out || !in) return einval("null field");
  if (!valid_prec(prec)) return einval("bad precision");
  if (out == in) return einval("out and in must not overlap");
  void** W = low_pool(ctx, prec);
  const bool p64 = prec == DWA_F64;
  return apply_dbb(ctx, prec, out, in, W[p64 ? W_OPB : L_OPB], W[p64 ? W_OPR : L_OPR]);
}

int dwa_apply_Dbb_batch(dwa_ctx* ctx, int prec, int nrhs, void* out, const void* in,
                        double* out_norm2) {
  DWA_TRY(check_ctx(ctx));
  if (!out || !in) return einval("null field");
  if (!valid_prec(prec)) return einval("bad precision");
  if (out == in) return einval("out and in must not overlap");
  if (nrhs < 1 || nrhs > ctx->batch.nmax) return einval("batch larger than reserved (dwa_reserve_batch)");
  BatchWs& w = ctx->batch;
  void* tb = prec == DWA_F64 ? w.f64[B_OPB] : w.lo[prec][BL_U];
  void* tr = prec == DWA_F64 ? w.f64[B_OPR] : w.lo[prec][BL_T];
  if (!out_norm2) return apply_dbb(ctx, prec, out, in, tb, tr, nrhs);
  // with the per-field |out|^2 from the partial sums of the second hop
  int nb = 0;
  DWA_TRY(launch_smix(ctx, prec, MIX_BG, tb, in, nullptr, 0.0, ctx->Ls, nullptr, nullptr, nrhs));
  DWA_TRY(dbb_from_premix(ctx, prec, out, in, tb, tr, bbank(ctx, 0), &nb, nrhs));
  std::vector<double> h(size_t(nb) * nrhs);
  DWA_HIP(hipMemcpyAsync(h.data(), bbank(ctx, 0), sizeof(double) * h.size(), hipMemcpyDeviceToHost, ctx->stream),
          "norm readback");
  DWA_HIP(hipStreamSynchronize(ctx->stream), "norm sync");
  for (int f = 0; f < nrhs; ++f) {
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) acc += h[size_t(f) * nb + i];
    out_norm2[f] = acc;
  }
  return DWA_OK;
}

int dwa_apply_Dbb_dag(dwa_ctx* ctx, int prec, void* out, const void* in) {
  DWA_TRY(check_ctx(ctx));
  if (!out || !in) return einval("null field");
  if (!valid_prec(prec)) return einval("bad precision");
  if (out == in) return einval("out and in must not overlap");
  void** W = low_pool(ctx, prec);
  const bool p64 = prec == DWA_F64;
  return apply_dbbdag(ctx, prec, out, in, W[p64 ? W_OPB : L_OPB], W[p64 ? W_OPR : L_OPR]);
}

int dwa_set_tuning(dwa_ctx* ctx, int prec, int ns, int order, int nf, int dense) {
  DWA_TRY(check_ctx(ctx));
  if (!valid_prec(prec)) return einval("bad precision");
  if (!valid_tile(ns)) return einval("tile must be 8, 16 or 32 sites");
  if (order < 0 || order >= ORDER_COUNT) return einval("order must be 0, 1 or 2");
  if (nf < 1 || nf > 64) return einval("fields per block must be in [1, 64]");
  if (dense != 0 && dense != 1) return einval("dense must be 0 or 1");
  if (!hop_specialised(ctx->Ls, ctx->dense_mix || dense) && ns != 8)
    return einval("the generic hop kernel (this Ls, or dense matrices) runs 8 sites per block");
  const size_t lds = hop_mix_lds_bytes_host(ns, ctx->Ls, prec == DWA_F64 ? 16 : 8, nf);
  if (std::max(lds, ctx->hop_min_lds) > ctx->max_lds) return einval("tile's LDS exceeds the device limit");
  ctx->tune[prec].ns = ns;
  ctx->tune[prec].order = order;
  ctx->tune[prec].nf = nf;
  ctx->tune[prec].dense = dense != 0;
  return DWA_OK;
}

int dwa_get_tuning(const dwa_ctx* ctx, int prec, int* ns, int* order, int* nf, int* dense) {
  if (!ctx) return einval("null context");
  if (!valid_prec(prec)) return einval("bad precision");
  if (ns) *ns = hop_sites_per_block(ctx, prec);
  if (order) *order = ctx->tune[prec].order;
  if (nf) *nf = ctx->tune[prec].nf;
  if (dense) *dense = use_dense(ctx, prec) ? 1 : 0;
  return DWA_OK;
}

int dwa_autotune(dwa_ctx* ctx, int prec, int reps, dwa_tune_entry* entries, int max_entries,
                 int* n_entries) {
  DWA_TRY(check_ctx(ctx));
  if (!valid_prec(prec)) return einval("bad precision");
  if (!ctx->links_set) {
    set_error("set the links first");
    return DWA_ESTATE;
  }
  if (n_entries) *n_entries = 0;
  if (reps <= 0) reps = 10;
  const bool p64 = prec == DWA_F64;
  const int Ls = ctx->Ls;
  const size_t n = field_elems(ctx);
  // one timed configuration: the hop pair of D_bb, t = N H x ; q = G^-1 I^-1 (-1/4 H t) + x,
  // on nr fields back to back
  struct Cand {
    HopTune t;
    int nrhs;
    double us;
  };
  std::vector<Cand> cands;
  const bool spec = hop_specialised(Ls, ctx->dense_mix);
  const HopTune saved = ctx->tune[prec];
  for (int ns : {8, 16, 32}) {
    if (!spec && ns != 8) continue;
    for (int ord = 0; ord < ORDER_COUNT; ++ord) {
      if (ord == ORDER_ZDOM && ctx->dims[2] % 8 != 0) continue;  // same as SLAB there
      HopTune c = saved;
      c.ns = ns;
      c.order = ord;
      c.dense = false;
      cands.push_back(Cand{c, 1, -1.0});
    }
  }
  // the dense fifth-dimension matrices (generic 8-site kernel) against the sweeps, when
  // the sweeps are valid at all
  if (!ctx->dense_mix)
    for (int ord = 0; ord < ORDER_COUNT; ++ord) {
      if (ord == ORDER_ZDOM && ctx->dims[2] % 8 != 0) continue;
      HopTune c = saved;
      c.ns = 8;
      c.order = ord;
      c.dense = true;
      cands.push_back(Cand{c, 1, -1.0});
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DWA_HIP(hipEventCreate(&e0), "event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(hipErrorOutOfMemory, "event");
  }
  auto time_pair = [&](Cand& c, void* x, void* t, void* q) -> int {
    ctx->tune[prec] = c.t;
    const size_t lds = hop_mix_lds_bytes_host(c.t.ns, Ls, p64 ? 16 : 8, c.nrhs > 1 ? c.t.nf : 1);
    if (std::max(lds, ctx->hop_min_lds) > ctx->max_lds) return DWA_OK;  // cannot run here
    const HopOp ha{x, t, nullptr, nullptr, 1.0, 0.0, 0.0, MIX_N, 1, Ls, nullptr, c.nrhs};
    const HopOp hb{t, q, nullptr, x, -0.25, 0.0, 1.0, MIX_GINV_IINV, 0, Ls, nullptr, c.nrhs};
    auto pair = [&]() -> int {
      DWA_TRY(launch_hop(ctx, prec, ha, nullptr));
      return launch_hop(ctx, prec, hb, nullptr);
    };
    DWA_TRY(pair());
    DWA_TRY(pair());  // warm-up
    DWA_HIP(hipEventRecord(e0, ctx->stream), "event record");
    for (int r = 0; r < reps; ++r) DWA_TRY(pair());
    DWA_HIP(hipEventRecord(e1, ctx->stream), "event record");
    DWA_HIP(hipEventSynchronize(e1), "event sync");
    float ms = 0.0f;
    DWA_HIP(hipEventElapsedTime(&ms, e0, e1), "event time");
    c.us = double(ms) * 1e3 / reps;
    return DWA_OK;
  };
  auto best_of = [&](size_t from) {
    long long b = -1;
    for (size_t k = from; k < cands.size(); ++k)
      if (cands[k].us >= 0 && (b < 0 || cands[k].us < cands[size_t(b)].us)) b = (long long)k;
    return b;
  };
  int rc = DWA_OK;
  // tile and order, on the context's single-field workspace
  {
    void** W = p64 ? ctx->w64 : low_pool(ctx, prec);
    void* x = W[p64 ? W_OPB : L_OPB];
    void* t = W[p64 ? W_OPR : L_OPR];
    void* q = W[p64 ? W_Q : L_Q];
    if ((rc = launch_zero(ctx, prec, x, n)) == DWA_OK) rc = launch_zero(ctx, prec, t, n);
    for (size_t k = 0; k < cands.size() && rc == DWA_OK; ++k) rc = time_pair(cands[k], x, t, q);
  }
  long long best = rc == DWA_OK ? best_of(0) : -1;
  HopTune chosen = best >= 0 ? cands[size_t(best)].t : saved;
  // fields per block, on a batch of up to 12 fields when one is reserved
  const int nb = std::min(ctx->batch.nmax, 12);
  if (rc == DWA_OK && best >= 0 && nb >= 2) {
    BatchWs& w = ctx->batch;
    void* x = p64 ? w.f64[B_OPB] : w.lo[prec][BL_W];
    void* t = p64 ? w.f64[B_OPR] : w.lo[prec][BL_T];
    void* q = p64 ? w.f64[B_Q] : w.lo[prec][BL_Q];
    if ((rc = launch_zero(ctx, prec, x, n, nb)) == DWA_OK) rc = launch_zero(ctx, prec, t, n, nb);
    const size_t from = cands.size();
    for (int nf : {1, 2, 3, 4, 6, 12}) {
      if (nf > nb) continue;
      HopTune c = chosen;
      c.nf = nf;
      cands.push_back(Cand{c, nb, -1.0});
    }
    for (size_t k = from; k < cands.size() && rc == DWA_OK; ++k) rc = time_pair(cands[k], x, t, q);
    const long long bb = rc == DWA_OK ? best_of(from) : -1;
    if (bb >= 0) chosen.nf = cands[size_t(bb)].t.nf;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tune[prec] = (rc == DWA_OK && best >= 0) ? chosen : saved;
  if (rc != DWA_OK) return rc;
  if (entries)
    for (size_t k = 0; k < cands.size() && int(k) < max_entries; ++k)
      entries[k] = dwa_tune_entry{prec, cands[k].t.ns, cands[k].t.order, cands[k].t.nf,
                                  (cands[k].t.dense || ctx->dense_mix) ? 1 : 0, cands[k].nrhs, cands[k].us};
  if (n_entries) *n_entries = int(cands.size());
  return DWA_OK;
}

int dwa_apply_hop(dwa_ctx* ctx, int prec, int parity_out, int kind, void* out, const void* in) {
  DWA_TRY(check_ctx(ctx));
  if (!out || !in) return einval("null field");
  if (!valid_prec(prec)) return einval("bad precision");
  if (parity_out != 0 && parity_out != 1) return einval("parity must be 0 or 1");
  if (kind != MIX_IDENTITY && kind != MIX_N && kind != MIX_NT && kind != MIX_GINV_IINV &&
      kind != MIX_G_BT_G5)
    return einval("hop output matrix must be one of kinds 0, 2, 3, 5, 6");
  if (out == in) return einval("out and in must not overlap");
  HopOp h{in, out, nullptr, nullptr, 1.0, 0.0, 0.0, kind, parity_out, ctx->Ls, nullptr};
  return launch_hop(ctx, prec, h, nullptr);
}

int dwa_cgne_solve(dwa_ctx* ctx, void* x, const void* rhs, const dwa_solve_opts* o,
                   dwa_solve_stats* stats) {
  DWA_TRY(check_ctx(ctx));
  if (!x || !rhs || !o) return einval("null argument");
  if (!(o->tol >= 0.0) || o->maxiter < 0) return einval("bad tolerance or maxiter");
  if (!valid_prec(o->inner_prec)) return einval("bad inner precision");
  if (o->mixed_mode != DWA_MIXED_RELIABLE && o->mixed_mode != DWA_MIXED_DEFECT)
    return einval("bad mixed_mode");
  if (x == rhs) return einval("x and rhs must not overlap");
  dwa_solve_stats st{};
  const auto t0 = std::chrono::steady_clock::now();
  int status = DWA_OK;
  if (o->inner_prec == DWA_F64) {
    CgResult cr;
    DWA_TRY(cgls(ctx, DWA_F64, x, rhs, o->warm_start != 0, o->tol, o->maxiter, o->check_every, &cr));
    double b2 = 0.0;
    DWA_TRY(host_norm2(ctx, DWA_F64, rhs, &b2));
    double rel = 0.0;
    DWA_TRY(true_residual64(ctx, x, rhs, std::sqrt(b2), &rel, nullptr));
    st.iters = cr.iters;
    st.outer = 0;
    st.converged = cr.converged;
    st.rel_resid = rel;
    st.n_Dbb = cr.n_dbb + 1;
    if (cr.breakdown) status = DWA_EBREAKDOWN;
    else if (!cr.converged) status = DWA_ENOCONV;
  } else {
    status = o->mixed_mode == DWA_MIXED_DEFECT ? mixed_solve(ctx, o->inner_prec, x, rhs, o, &st)
                                               : reliable_solve(ctx, o->inner_prec, x, rhs, o, &st);
    if (status != DWA_OK && status != DWA_ENOCONV && status != DWA_EBREAKDOWN) return status;
  }
  DWA_HIP(hipStreamSynchronize(ctx->stream), "solve sync");
  st.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  if (status == DWA_ENOCONV) set_error("solver reached maxiter or stagnated");
  if (status == DWA_EBREAKDOWN) set_error("CG breakdown (|D_bb p|^2 or |D_bb^dag r|^2 not positive/finite)");
  return status;
}

// CGLS on one of the Schur forms of Sec. 3 for D_bb x = rhs (FP64, plain: every scalar goes
// through the host, so the three forms run the same algorithm):
//   form 0: eq.(redblack),  A = D_bb = 1 - I_bb^-1 D_br I_rr^-1 D_rb,  b = rhs;
//   form 1: eq.(redblack1), A = I_bb D_bb = I_bb - D_br I_rr^-1 D_rb,  b = I_bb rhs;
//   form 2: eq.(redblack1) with its rows scaled, A = W I_bb D_bb, b = W I_bb rhs, W dividing
//           every row s whose coefficient max(b_s, c_s) exceeds one by that coefficient.
// All three have the solution x of D_bb x = rhs.  Stops when |b - A x| <= tol |b| (the
// form's own residual); *rel receives |rhs - D_bb x| / |rhs| of the result.
// Workspace: W_R, W_P, W_Z, W_Q, W_W, W_U, W_RES, W_OPB, W_OPR.
static int cgls_form(dwa_ctx* ctx, int form, void* x, const void* rhs, double tol, int maxiter,
                     CgResult* res, double* rel) {
  void** W = ctx->w64;
  const size_t n = field_elems(ctx);
  void *r = W[W_R], *p = W[W_P], *z = W[W_Z], *q = W[W_Q], *tmp = W[W_W], *b = W[W_RES];
  const int mixA = form == 2 ? MIX_W_I : MIX_I_ALPHA, mixAT = form == 2 ? MIX_W_I_T : MIX_I_ALPHA_T;
  auto applyA = [&](void* out, const void* in) -> int {
    if (form == 0) return apply_dbb(ctx, DWA_F64, out, in, W[W_OPB], W[W_OPR]);
    DWA_TRY(apply_dbb(ctx, DWA_F64, tmp, in, W[W_OPB], W[W_OPR]));
    return launch_smix(ctx, DWA_F64, mixA, out, tmp, nullptr, 0.0, ctx->Ls, nullptr, nullptr);
  };
  auto applyAd = [&](void* out, const void* in) -> int {
    if (form == 0) return apply_dbbdag(ctx, DWA_F64, out, in, W[W_OPB], W[W_OPR]);
    DWA_TRY(launch_smix(ctx, DWA_F64, mixAT, tmp, in, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
    return apply_dbbdag(ctx, DWA_F64, out, tmp, W[W_OPB], W[W_OPR]);
  };
  if (form == 0) DWA_TRY(launch_axpby(ctx, DWA_F64, b, 1.0, rhs, 0.0, n));
  else DWA_TRY(launch_smix(ctx, DWA_F64, mixA, b, rhs, nullptr, 0.0, ctx->Ls, nullptr, nullptr));
  double b2 = 0.0, r2 = 0.0, gamma = 0.0, q2 = 0.0;
  DWA_TRY(host_norm2(ctx, DWA_F64, b, &b2));
  DWA_TRY(launch_zero(ctx, DWA_F64, x, n));
  DWA_TRY(launch_axpby(ctx, DWA_F64, r, 1.0, b, 0.0, n));
  DWA_TRY(applyAd(z, r));
  DWA_TRY(host_norm2(ctx, DWA_F64, z, &gamma));
  DWA_TRY(launch_axpby(ctx, DWA_F64, p, 1.0, z, 0.0, n));
  res->n_dbb += 1;
  r2 = b2;
  int k = 0;
  while (b2 > 0.0 && r2 > tol * tol * b2 && k < maxiter) {
    DWA_TRY(applyA(q, p));
    DWA_TRY(host_norm2(ctx, DWA_F64, q, &q2));
    if (!(q2 > 0.0) || !std::isfinite(q2)) {
      res->breakdown = 1;
      break;
    }
    const double a = gamma / q2;
    DWA_TRY(launch_axpby(ctx, DWA_F64, x, a, p, 1.0, n));
    DWA_TRY(launch_axpby(ctx, DWA_F64, r, -a, q, 1.0, n));
    DWA_TRY(host_norm2(ctx, DWA_F64, r, &r2));
    DWA_TRY(applyAd(z, r));
    double g2 = 0.0;
    DWA_TRY(host_norm2(ctx, DWA_F64, z, &g2));
    DWA_TRY(launch_axpby(ctx, DWA_F64, p, 1.0, z, g2 / gamma, n));
    gamma = g2;
    res->n_dbb += 2;
    ++k;
  }
  res->iters = k;
  res->converged = b2 == 0.0 || r2 <= tol * tol * b2;
  res->rel_recursive = b2 > 0.0 ? std::sqrt(r2 / b2) : 0.0;
  double rh2 = 0.0;
  DWA_TRY(host_norm2(ctx, DWA_F64, rhs, &rh2));
  return true_residual64(ctx, x, rhs, std::sqrt(rh2), rel, nullptr);
}

// y = [P^-1 D_1(m)^-1 D_1(ms) P (eta, 0, ..., 0)]_1 = D_OV(m)^-1 D_OV(ms) eta (App. A and B,
// eq.(startprop) and eq.(tosolve)), m the context's mass; solved through D_alpha(m) =
// D_1(m) G, whose G drops out of the extraction.  ms = 1 is the propagator (D_OV(1) = 1).
// form < 0: the Schur system is solved by dwa_cgne_solve (all options); form 0..2: by
// cgls_form in FP64 (opts->tol and maxiter only).
static int propagator_impl(dwa_ctx* ctx, double ms, void* y1, const void* eta, const dwa_solve_opts* o,
                           dwa_solve_stats* stats, void* psi5, int form = -1) {
  DWA_TRY(check_ctx(ctx));
  if (!y1 || !eta || !o) return einval("null argument");
  void** W = ctx->w64;
  // reject non-finite sources before any arithmetic
  int* d_flag = reinterpret_cast<int*>(ctx->d_red);
  DWA_HIP(hipMemsetAsync(d_flag, 0, sizeof(int), ctx->stream), "clear flag");
  DWA_TRY(launch_check_finite(ctx, eta, size_t(ctx->V) * 12, d_flag));
  int h_flag = 0;
  DWA_HIP(hipMemcpyAsync(&h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "flag readback");
  DWA_HIP(hipStreamSynchronize(ctx->stream), "flag sync");
  if (h_flag) {
    set_error("source contains NaN or Inf");
    return DWA_ENAN;
  }
  const int Ls = ctx->Ls;
  // rho = D_1(ms) P (eta, 0, ..., 0): wall slices only
  DWA_TRY(launch_source(ctx, W[W_CHI_B], W[W_CHI_R], W[W_RHO_B], W[W_RHO_R], eta, ms));
  DWA_TRY(wall_hops(ctx, W[W_CHI_B], W[W_CHI_R], W[W_RHO_B], W[W_RHO_R]));
  // phi' = I_bb^-1 (rho_b - D_br I_rr^-1 rho_r) = G^-1 I^-1 (rho_b + 1/2 H_br N rho_r)
  DWA_TRY(launch_smix(ctx, DWA_F64, MIX_N, W[W_T], W[W_RHO_R], nullptr, 0.0, Ls, nullptr, nullptr));
  HopOp prep{W[W_T], W[W_PHI], W[W_RHO_B], nullptr, 0.5, 1.0, 0.0, MIX_GINV_IINV, 0, Ls, nullptr};
  DWA_TRY(launch_hop(ctx, DWA_F64, prep, nullptr));
  // D_bb psi_b = phi'
  int status = DWA_OK;
  if (form < 0) {
    dwa_solve_opts so = *o;
    so.warm_start = 0;
    status = dwa_cgne_solve(ctx, W[W_PSI_B], W[W_PHI], &so, stats);
    if (status != DWA_OK && status != DWA_ENOCONV) return status;
  } else {
    const auto t0 = std::chrono::steady_clock::now();
    CgResult cr;
    double rel = 0.0;
    DWA_TRY(cgls_form(ctx, form, W[W_PSI_B], W[W_PHI], o->tol, o->maxiter, &cr, &rel));
    status = cr.breakdown ? DWA_EBREAKDOWN : (cr.converged ? DWA_OK : DWA_ENOCONV);
    if (stats) {
      *stats = dwa_solve_stats{};
      stats->iters = cr.iters;
      stats->converged = cr.converged;
      stats->rel_resid = rel;
      stats->n_Dbb = cr.n_dbb + 1;
      stats->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status == DWA_EBREAKDOWN) return status;
  }
  // psi_r = I_rr^-1 (rho_r - D_rb psi_b) = G^-1 I^-1 (rho_r + 1/2 H_rb B G psi_b)
  DWA_TRY(launch_smix(ctx, DWA_F64, MIX_BG, W[W_OPB], W[W_PSI_B], nullptr, 0.0, Ls, nullptr, nullptr));
  HopOp rec{W[W_OPB], W[W_PSI_R], W[W_RHO_R], nullptr, 0.5, 1.0, 0.0, MIX_GINV_IINV, 1, Ls, nullptr};
  DWA_TRY(launch_hop(ctx, DWA_F64, rec, nullptr));
  DWA_TRY(launch_extract(ctx, y1, W[W_PSI_B], W[W_PSI_R]));
  if (psi5) {
    DWA_TRY(launch_unpack5(ctx, DWA_F64, psi5, W[W_PSI_B], 0, Ls));
    DWA_TRY(launch_unpack5(ctx, DWA_F64, psi5, W[W_PSI_R], 1, Ls));
  }
  DWA_HIP(hipStreamSynchronize(ctx->stream), "propagator sync");
  return status;
}

int dwa_propagator(dwa_ctx* ctx, void* y1, const void* eta, const dwa_solve_opts* o,
                   dwa_solve_stats* stats, void* psi5) {
  return propagator_impl(ctx, 1.0, y1, eta, o, stats, psi5);
}

int dwa_propagator_form(dwa_ctx* ctx, int form, void* y1, const void* eta, const dwa_solve_opts* o,
                        dwa_solve_stats* stats) {
  if (form < 0 || form > 2) return einval("form must be 0, 1 or 2");
  if (o && !(o->tol > 0.0)) return einval("bad tolerance");
  if (o && o->maxiter < 0) return einval("bad maxiter");
  return propagator_impl(ctx, 1.0, y1, eta, o, stats, nullptr, form);
}

int dwa_overlap_apply(dwa_ctx* ctx, double m, void* out, const void* in, const dwa_solve_opts* o,
                      dwa_solve_stats* stats) {
  DWA_TRY(check_ctx(ctx));
  if (ctx->m != 1.0) return einval("dwa_overlap_apply needs a context of mass 1 (the D_1(1) solve)");
  if (!std::isfinite(m)) return einval("mass must be finite");
  if (!out || !in || !o) return einval("null argument");
  if (out == in) return einval("out and in must not overlap");
  return propagator_impl(ctx, m, out, in, o, stats, nullptr);
}

int dwa_alpha_sweep(dwa_ctx* ctx, const double* alphas, int n, void* y1, const void* eta,
                    const dwa_solve_opts* o, dwa_solve_stats* stats) {
  DWA_TRY(check_ctx(ctx));
  if (!alphas || n < 1 || !y1 || !eta || !o || !stats) return einval("null argument or n < 1");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(alphas[i]) || alphas[i] == 0.0) return einval("alpha must be finite and non-zero");
  const double alpha0 = ctx->alpha;
  const size_t field_bytes = size_t(ctx->V) * 12 * 16;
  int first = DWA_OK;
  for (int i = 0; i < n; ++i) {
    int rc = dwa_set_alpha(ctx, alphas[i]);
    if (rc == DWA_OK)
      rc = dwa_propagator(ctx, static_cast<char*>(y1) + i * field_bytes, eta, o, &stats[i], nullptr);
    if (rc != DWA_OK && rc != DWA_ENOCONV) {
      (void)dwa_set_alpha(ctx, alpha0);
      return rc;
    }
    if (rc != DWA_OK && first == DWA_OK) first = rc;
  }
  DWA_TRY(dwa_set_alpha(ctx, alpha0));
  if (first == DWA_ENOCONV) set_error("solver reached maxiter or stagnated for some alpha");
  return first;
}

// Per-slice Re <a, b> over both parities (a times g5 when g5), summed on the host in
// a fixed order.  a[2] / b[2]: black and red SoA fields of nslices slices.
static int host_slice_dots(dwa_ctx* ctx, const void* const a[2], const void* const b[2], int nslices,
                    bool g5, double* out) {
  const int nb = slice_dot_blocks(12 * size_t(ctx->Vh));
  std::vector<double> h(size_t(nslices) * nb);
  for (int s = 0; s < nslices; ++s) out[s] = 0.0;
  for (int par = 0; par < 2; ++par) {
    DWA_TRY(launch_slice_dot(ctx, a[par], b[par], nslices, ctx->Vh, g5, bank(ctx, 2)));
    DWA_HIP(hipMemcpyAsync(h.data(), bank(ctx, 2), sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                           ctx->stream), "dot readback");
    DWA_HIP(hipStreamSynchronize(ctx->stream), "dot sync");
    for (int s = 0; s < nslices; ++s)
      for (int k = 0; k < nb; ++k) out[s] += h[size_t(s) * nb + k];
  }
  return DWA_OK;
}

int dwa_propagator_adjoint(dwa_ctx* ctx, void* gU, void* geta, double* galpha, double* gb,
                           double* gc, double* L, void* y1, const void* eta, const void* eta_p,
                           const dwa_solve_opts* o, dwa_solve_stats* stats) {
  DWA_TRY(check_ctx(ctx));
  if (!eta || !eta_p || !o) return einval("null argument");
  const int Ls = ctx->Ls;
  const size_t Vh = size_t(ctx->Vh);
  const size_t n = field_elems(ctx);
  const size_t slice = 12 * Vh;  // complex numbers per half-field slice
  void** W = ctx->w64;
  dwa_solve_stats st[2]{};

  // forward: psi (W_PSI_B/R), chi' = B_1 P b (W_CHI_B/R), y_1
  void* ybuf = y1 ? y1 : W[W_X];
  int status = dwa_propagator(ctx, ybuf, eta, o, &st[0], nullptr);
  if (status != DWA_OK && status != DWA_ENOCONV) return status;
  if (L) {
    const void* a[2] = {eta_p, nullptr};
    const void* b[2] = {ybuf, nullptr};
    const int nb = slice_dot_blocks(12 * 2 * Vh);
    std::vector<double> h(nb);
    DWA_TRY(launch_slice_dot(ctx, a[0], b[0], 1, 2 * Vh, false, bank(ctx, 2)));
    DWA_HIP(hipMemcpyAsync(h.data(), bank(ctx, 2), sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream),
            "loss readback");
    DWA_HIP(hipStreamSynchronize(ctx->stream), "loss sync");
    double v = 0.0;
    for (int k = 0; k < nb; ++k) v += h[k];
    *L = v;
  }

  // adjoint: D_alpha^dag lambda = f = E^dag eta' through the red-black Schur form,
  //   g_b = f_b - D_rb^dag I^-dag f_r = f_b + 1/2 G B^T g5 H_br (g5 I_1^-T G^-1 f_r),
  //   D_bb^dag mu_b = g_b (CGLS on D_bb^dag),  g5 lambda_b = g5 I_1^-T G^-1 mu_b,
  //   g5 lambda_r = g5 I_1^-T G^-1 (f_r + 1/2 G B^T g5 H_rb (g5 lambda_b)).
  void* f_b = W[W_RHO_B];
  void* f_r = W[W_RHO_R];
  DWA_TRY(launch_adj_source(ctx, f_b, f_r, eta_p));
  DWA_TRY(launch_smix(ctx, DWA_F64, MIX_G5_IINVT_GINV, W[W_OPR], f_r, nullptr, 0.0, Ls, nullptr, nullptr));
  HopOp hg{W[W_OPR], W[W_PHI], nullptr, f_b, 0.5, 0.0, 1.0, MIX_G_BT_G5, 0, Ls, nullptr};
  DWA_TRY(launch_hop(ctx, DWA_F64, hg, nullptr));
  {
    const auto t0 = std::chrono::steady_clock::now();
    CgResult cr;
    if (o->inner_prec == DWA_F64) {
      DWA_TRY(cgls(ctx, DWA_F64, W[W_X], W[W_PHI], false, o->tol, o->maxiter, o->check_every, &cr, true));
    } else {
      // the forward solve's inner precision, with reliable updates, from x = 0
      dwa_solve_opts oa = *o;
      oa.warm_start = 0;
      dwa_solve_stats sa{};
      const int rc = reliable_solve(ctx, o->inner_prec, W[W_X], W[W_PHI], &oa, &sa, true);
      if (rc != DWA_OK && rc != DWA_ENOCONV && rc != DWA_EBREAKDOWN) return rc;
      cr.iters = sa.iters;
      cr.converged = sa.converged;
      cr.breakdown = rc == DWA_EBREAKDOWN;
      cr.n_dbb = sa.n_Dbb;
      st[1].outer = sa.outer;
    }
    double g2 = 0.0;
    DWA_TRY(host_norm2(ctx, DWA_F64, W[W_PHI], &g2));
    DWA_TRY(apply_dbbdag(ctx, DWA_F64, W[W_Q], W[W_X], W[W_OPB], W[W_OPR]));
    DWA_TRY(launch_axpby(ctx, DWA_F64, W[W_RES], 1.0, W[W_PHI], 0.0, n));
    DWA_TRY(launch_axpby(ctx, DWA_F64, W[W_RES], -1.0, W[W_Q], 1.0, n));
    double r2 = 0.0;
    DWA_TRY(host_norm2(ctx, DWA_F64, W[W_RES], &r2));
    st[1].iters = cr.iters;
    st[1].converged = cr.converged;
    st[1].rel_resid = g2 > 0 ? std::sqrt(r2 / g2) : 0.0;
    st[1].n_Dbb = cr.n_dbb + 1;
    st[1].time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (cr.breakdown) {
      set_error("CG breakdown in the adjoint solve");
      return DWA_EBREAKDOWN;
    }
    if (!cr.converged && status == DWA_OK) status = DWA_ENOCONV;
  }
  void* lt_b = W[W_P];
  void* lt_r = W[W_Z];
  DWA_TRY(launch_smix(ctx, DWA_F64, MIX_G5_IINVT_GINV, lt_b, W[W_X], nullptr, 0.0, Ls, nullptr, nullptr));
  HopOp hl{lt_b, W[W_Q], nullptr, f_r, 0.5, 0.0, 1.0, MIX_G_BT_G5, 1, Ls, nullptr};
  DWA_TRY(launch_hop(ctx, DWA_F64, hl, nullptr));
  DWA_TRY(launch_smix(ctx, DWA_F64, MIX_G5_IINVT_GINV, lt_r, W[W_Q], nullptr, 0.0, Ls, nullptr, nullptr));
  const void* lt[2] = {lt_b, lt_r};

  // links: phi = B_1 P b - B G psi on both parities, then the force kernel
  if (gU) {
    void* ph_b = W[W_R];
    void* ph_r = W[W_T];
    DWA_TRY(launch_smix(ctx, DWA_F64, MIX_BG, ph_b, W[W_PSI_B], nullptr, 0.0, Ls, nullptr, nullptr));
    DWA_TRY(launch_smix(ctx, DWA_F64, MIX_BG, ph_r, W[W_PSI_R], nullptr, 0.0, Ls, nullptr, nullptr));
    DWA_TRY(launch_axpby(ctx, DWA_F64, ph_b, 1.0, W[W_CHI_B], -1.0, n));
    DWA_TRY(launch_axpby(ctx, DWA_F64, ph_r, 1.0, W[W_CHI_R], -1.0, n));
    DWA_TRY(launch_force(ctx, gU, lt_b, lt_r, ph_b, ph_r));
  }

  // b_s, c_s: Re <lambda_s, (D_w omega)_s> with D_w omega = (4 + M5) omega - 1/2 H omega
  auto dw_full = [&](void* out_b, void* out_r, const void* in_b, const void* in_r) {
    HopOp ob{in_r, out_b, in_b, nullptr, -0.5, 4.0 + ctx->M5, 0.0, MIX_IDENTITY, 0, Ls, nullptr};
    HopOp orr{in_b, out_r, in_r, nullptr, -0.5, 4.0 + ctx->M5, 0.0, MIX_IDENTITY, 1, Ls, nullptr};
    int rc = launch_hop(ctx, DWA_F64, ob, nullptr);
    return rc == DWA_OK ? launch_hop(ctx, DWA_F64, orr, nullptr) : rc;
  };
  if (gb || gc) {
    DWA_TRY(launch_omega(ctx, W[W_W], W[W_U], W[W_PSI_B], eta, 0));
    DWA_TRY(launch_omega(ctx, W[W_OPB], W[W_OPR], W[W_PSI_R], eta, 1));
    const void* dws[2] = {W[W_RES], W[W_PHI]};
    if (gb) {
      DWA_TRY(dw_full(W[W_RES], W[W_PHI], W[W_W], W[W_OPB]));
      DWA_TRY(host_slice_dots(ctx, lt, dws, Ls, true, gb));
    }
    if (gc) {
      DWA_TRY(dw_full(W[W_RES], W[W_PHI], W[W_U], W[W_OPR]));
      DWA_TRY(host_slice_dots(ctx, lt, dws, Ls, true, gc));
    }
  }

  // alpha: d D_alpha / d alpha = D_1 dG/dalpha = D_alpha (J / alpha), J = diag(P+, 1, .., 1, P-),
  // so dL/dalpha = -Re <lambda, D_alpha J psi> / alpha, with D_alpha = I_1 G - 1/2 H B G
  if (galpha) {
    void* v[2] = {W[W_W], W[W_U]};
    void* out[2] = {W[W_OPB], W[W_PHI]};
    DWA_TRY(launch_jpsi(ctx, v[0], W[W_PSI_B]));
    DWA_TRY(launch_jpsi(ctx, v[1], W[W_PSI_R]));
    for (int par = 0; par < 2; ++par) {
      DWA_TRY(launch_smix(ctx, DWA_F64, MIX_BG, W[W_OPR], v[1 - par], nullptr, 0.0, Ls, nullptr, nullptr));
      HopOp hh{W[W_OPR], W[W_RES], nullptr, nullptr, -0.5, 0.0, 0.0, MIX_IDENTITY, par, Ls, nullptr};
      DWA_TRY(launch_hop(ctx, DWA_F64, hh, nullptr));
      DWA_TRY(launch_smix(ctx, DWA_F64, MIX_I_ALPHA, out[par], v[par], W[W_RES], 1.0, Ls, nullptr, nullptr));
    }
    std::vector<double> d(Ls);
    const void* outc[2] = {out[0], out[1]};
    DWA_TRY(host_slice_dots(ctx, lt, outc, Ls, true, d.data()));
    double sum = 0.0;
    for (int s2 = 0; s2 < Ls; ++s2) sum += d[s2];
    *galpha = -sum / ctx->alpha;
  }

  // eta: u = D_w^dag lambda = g5 D_w (g5 lambda) on the wall slices, then combine
  if (geta) {
    const size_t last = size_t(Ls - 1);
    for (int par = 0; par < 2; ++par) {
      void* dst = par ? W[W_PHI] : W[W_RES];
      const void* own = lt[par];
      const void* other = lt[1 - par];
      for (int k = 0; k < 2; ++k) {
        const size_t sidx = k ? last : 0;
        HopOp h{static_cast<const double2*>(other) + sidx * slice, static_cast<double2*>(dst) + k * slice,
                static_cast<const double2*>(own) + sidx * slice, nullptr, -0.5, 4.0 + ctx->M5, 0.0,
                MIX_IDENTITY, par, 1, nullptr};
        DWA_TRY(launch_hop(ctx, DWA_F64, h, nullptr));
      }
    }
    DWA_TRY(launch_geta(ctx, geta, lt_b, lt_r, W[W_RES], W[W_PHI]));
  }
  DWA_HIP(hipStreamSynchronize(ctx->stream), "adjoint sync");
  if (stats) {
    stats[0] = st[0];
    stats[1] = st[1];
  }
  if (status == DWA_ENOCONV) set_error("forward or adjoint solve reached maxiter");
  return status;
}

int dwa_reserve_batch(dwa_ctx* ctx, int nmax) {
  if (!ctx) return einval("null context");
  if (nmax < 1 || nmax > 4096) return einval("batch size must be in [1, 4096]");
  DWA_HIP(hipStreamSynchronize(ctx->stream), "reserve sync");
  free_batch(ctx);
  BatchWs& b = ctx->batch;
  const size_t n = field_elems(ctx);
  auto fail = [&](int rc) {
    free_batch(ctx);
    return rc;
  };
  int rc = DWA_OK;
  for (int i = 0; i < B_COUNT; ++i)
    if ((rc = hip_fail(hipMalloc(&b.f64[i], 16 * n * nmax), "alloc batch fp64"))) return fail(rc);
  for (int pr : {DWA_F32, DWA_BF16})
    for (int i = 0; i < BL_COUNT; ++i)
      if ((rc = hip_fail(hipMalloc(&b.lo[pr][i], elem_bytes(pr) * n * nmax), "alloc batch low")))
        return fail(rc);
  if ((rc = hip_fail(hipMalloc(&b.xacc, 8 * n * nmax), "alloc batch acc"))) return fail(rc);
  if ((rc = hip_fail(hipMalloc(&b.d_scal, sizeof(DevScalars) * nmax), "alloc batch scalars"))) return fail(rc);
  if ((rc = hip_fail(hipMemset(b.d_scal, 0, sizeof(DevScalars) * nmax), "clear batch scalars"))) return fail(rc);
  b.bank_elems = size_t(ctx->Vh) + 8192;
  if ((rc = hip_fail(hipMalloc(&b.partials, sizeof(double) * 4 * nmax * b.bank_elems), "alloc batch partials")))
    return fail(rc);
  if ((rc = hip_fail(hipMalloc(&b.d_coef, sizeof(double) * 4 * nmax), "alloc batch coefficients"))) return fail(rc);
  if ((rc = hip_fail(hipHostMalloc(&b.h_scal, sizeof(DevScalars) * nmax, hipHostMallocDefault), "alloc pinned")))
    return fail(rc);
  if ((rc = hip_fail(hipHostMalloc(&b.h_coef, sizeof(double) * 4 * nmax, hipHostMallocDefault), "alloc pinned")))
    return fail(rc);
  if ((rc = hip_fail(hipHostMalloc(&b.h_active, sizeof(int) * nmax, hipHostMallocDefault), "alloc pinned")))
    return fail(rc);
  if ((rc = hip_fail(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking), "batch stream")))
    return fail(rc);
  b.nmax = nmax;
  return DWA_OK;
}

int dwa_propagator_multi(dwa_ctx* const* ctxs, int nctx, const int* nrhs, void* const* y1,
                         const void* const* eta, const dwa_solve_opts* o, dwa_solve_stats* stats) {
  if (!ctxs || nctx < 1 || !nrhs || !y1 || !eta || !o) return einval("null argument or nctx < 1");
  if (!(o->tol > 0.0) || o->maxiter < 0) return einval("bad tolerance or maxiter");
  if (!valid_prec(o->inner_prec)) return einval("bad inner precision");
  for (int i = 0; i < nctx; ++i) {
    DWA_TRY(check_ctx(ctxs[i]));
    if (nrhs[i] < 1 || nrhs[i] > ctxs[i]->batch.nmax)
      return einval("batch larger than reserved (dwa_reserve_batch)");
    if (!y1[i] || !eta[i]) return einval("null field");
    if (ctxs[i]->device != ctxs[0]->device) return einval("contexts on different devices");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return einval("a context appears twice");
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = ctxs[0]->batch.stream;
  std::vector<hipStream_t> saved(nctx);
  for (int i = 0; i < nctx; ++i) {
    DWA_HIP(hipStreamSynchronize(ctxs[i]->stream), "multi entry sync");
    saved[i] = ctxs[i]->stream;
    ctxs[i]->stream = st;
  }
  auto restore = [&]() {
    for (int i = 0; i < nctx; ++i) ctxs[i]->stream = saved[i];
  };
  auto run = [&]() -> int {
    // source and Schur right-hand side of every field
    for (int i = 0; i < nctx; ++i) {
      dwa_ctx* ctx = ctxs[i];
      BatchWs& w = ctx->batch;
      const int nr = nrhs[i], Ls = ctx->Ls;
      const size_t n = field_elems(ctx), v12 = size_t(ctx->V) * 12;
      auto at = [&](int role, int f) { return static_cast<void*>(static_cast<double2*>(w.f64[role]) + f * n); };
      for (int f = 0; f < nr; ++f)
        DWA_TRY(launch_source(ctx, at(B_CHI_B, f), at(B_CHI_R, f), at(B_RHO_B, f), at(B_RHO_R, f),
                              static_cast<const double2*>(eta[i]) + f * v12));
      DWA_TRY(wall_hops(ctx, w.f64[B_CHI_B], w.f64[B_CHI_R], w.f64[B_RHO_B], w.f64[B_RHO_R], nr));
      DWA_TRY(launch_smix(ctx, DWA_F64, MIX_N, w.f64[B_T], w.f64[B_RHO_R], nullptr, 0.0, Ls, nullptr, nullptr, nr));
      HopOp prep{w.f64[B_T], w.f64[B_PHI], w.f64[B_RHO_B], nullptr, 0.5, 1.0, 0.0, MIX_GINV_IINV, 0, Ls, nullptr, nr};
      DWA_TRY(launch_hop(ctx, DWA_F64, prep, nullptr));
    }
    // solve D_bb X = PHI for every field
    const int inner = o->inner_prec;
    MultiSolve M;
    DWA_TRY(multi_solve(ctxs, nctx, nrhs, o, st, M));
    const auto& iters = M.iters;
    const auto& outer = M.outer;
    const auto& bnorm = M.bnorm;
    const auto& fp64_conv = M.fp64_conv;
    // final residuals, reconstruction and extraction
    int status = DWA_OK;
    size_t off = 0;
    for (int i = 0; i < nctx; ++i) {
      dwa_ctx* ctx = ctxs[i];
      BatchWs& w = ctx->batch;
      const int nr = nrhs[i], Ls = ctx->Ls;
      const size_t n = field_elems(ctx), v12 = size_t(ctx->V) * 12;
      std::vector<double> r2(nr);
      DWA_TRY(batch_true_residual(ctx, nr, st, r2.data()));
      DWA_TRY(launch_smix(ctx, DWA_F64, MIX_BG, w.f64[B_OPB], w.f64[B_X], nullptr, 0.0, Ls, nullptr, nullptr, nr));
      HopOp rec{w.f64[B_OPB], w.f64[B_PSI_R], w.f64[B_RHO_R], nullptr, 0.5, 1.0, 0.0, MIX_GINV_IINV, 1, Ls, nullptr, nr};
      DWA_TRY(launch_hop(ctx, DWA_F64, rec, nullptr));
      for (int f = 0; f < nr; ++f)
        DWA_TRY(launch_extract(ctx, static_cast<double2*>(y1[i]) + f * v12,
                               static_cast<const double2*>(w.f64[B_X]) + f * n,
                               static_cast<const double2*>(w.f64[B_PSI_R]) + f * n));
      for (int f = 0; f < nr; ++f) {
        const double r = bnorm[i][f] > 0.0 ? std::sqrt(r2[f]) / bnorm[i][f] : 0.0;
        // FP64: the CGLS stopping rule (recursive residual), as dwa_cgne_solve; mixed
        // precision: the FP64 residual that ends the defect correction
        const bool conv = inner == DWA_F64 ? fp64_conv[i][f] != 0 : r <= o->tol;
        if (!conv) status = DWA_ENOCONV;
        if (stats) {
          dwa_solve_stats& sf = stats[off + f];
          sf = dwa_solve_stats{};
          sf.iters = iters[i][f];
          sf.outer = outer[i][f];
          sf.converged = conv;
          sf.rel_resid = r;
        }
      }
      off += nr;
    }
    DWA_HIP(hipStreamSynchronize(st), "multi sync");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
      for (size_t k = 0; k < off; ++k) stats[k].time_ms = ms;
    return status;
  };
  const int status = run();
  if (status != DWA_OK && status != DWA_ENOCONV) (void)hipStreamSynchronize(st);
  restore();
  if (status == DWA_ENOCONV) set_error("some field of the batch did not converge");
  return status;
}

int dwa_propagator_batch(dwa_ctx* ctx, int nrhs, void* y1, const void* eta, const dwa_solve_opts* o,
                         dwa_solve_stats* stats) {
  dwa_ctx* const c[1] = {ctx};
  const int n[1] = {nrhs};
  void* const y[1] = {y1};
  const void* const e[1] = {eta};
  if (!ctx) return einval("null context");
  return dwa_propagator_multi(c, 1, n, y, e, o, stats);
}

int dwa_cgne_solve_batch(dwa_ctx* const* ctxs, int nctx, int nrhs, void* const* x_b,
                         const void* const* rhs_b, const dwa_solve_opts* o, dwa_solve_stats* stats) {
  if (!ctxs || nctx < 1 || nrhs < 1 || !x_b || !rhs_b || !o)
    return einval("null argument, nctx < 1 or nrhs < 1");
  if (!(o->tol > 0.0) || o->maxiter < 0) return einval("bad tolerance or maxiter");
  if (!valid_prec(o->inner_prec)) return einval("bad inner precision");
  if (o->mixed_mode != DWA_MIXED_RELIABLE && o->mixed_mode != DWA_MIXED_DEFECT)
    return einval("bad mixed_mode");
  if (o->warm_start) return einval("batched CGNE starts from x = 0 (warm_start must be 0)");
  for (int i = 0; i < nctx; ++i) {
    DWA_TRY(check_ctx(ctxs[i]));
    if (nrhs > ctxs[i]->batch.nmax) return einval("batch larger than reserved (dwa_reserve_batch)");
    if (!x_b[i] || !rhs_b[i]) return einval("null field");
    if (ctxs[i]->device != ctxs[0]->device) return einval("contexts on different devices");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return einval("a context appears twice");
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = ctxs[0]->batch.stream;
  std::vector<hipStream_t> saved(nctx);
  for (int i = 0; i < nctx; ++i) {
    DWA_HIP(hipStreamSynchronize(ctxs[i]->stream), "batch entry sync");
    saved[i] = ctxs[i]->stream;
    ctxs[i]->stream = st;
  }
  std::vector<int> nr(nctx, nrhs);
  auto run = [&]() -> int {
    // the right-hand sides into the batch workspace (the solve reads PHI, writes X)
    for (int i = 0; i < nctx; ++i)
      DWA_HIP(hipMemcpyAsync(ctxs[i]->batch.f64[B_PHI], rhs_b[i], dwa_field_bytes(ctxs[i], DWA_F64, nrhs),
                             hipMemcpyDeviceToDevice, st),
              "rhs copy");
    MultiSolve M;
    DWA_TRY(multi_solve(ctxs, nctx, nr.data(), o, st, M));
    int status = DWA_OK;
    for (int i = 0; i < nctx; ++i) {
      std::vector<double> r2(nrhs);
      DWA_TRY(batch_true_residual(ctxs[i], nrhs, st, r2.data()));
      DWA_HIP(hipMemcpyAsync(x_b[i], ctxs[i]->batch.f64[B_X], dwa_field_bytes(ctxs[i], DWA_F64, nrhs),
                             hipMemcpyDeviceToDevice, st),
              "solution copy");
      for (int f = 0; f < nrhs; ++f) {
        const double b = M.bnorm[i][f];
        const double r = b > 0.0 ? std::sqrt(r2[f]) / b : 0.0;
        const bool conv = o->inner_prec == DWA_F64 ? M.fp64_conv[i][f] != 0 : r <= o->tol;
        if (!conv) status = DWA_ENOCONV;
        if (stats) {
          dwa_solve_stats& sf = stats[size_t(i) * nrhs + f];
          sf = dwa_solve_stats{};
          sf.iters = M.iters[i][f];
          sf.outer = M.outer[i][f];
          sf.converged = conv;
          sf.rel_resid = r;
        }
      }
    }
    DWA_HIP(hipStreamSynchronize(st), "batch sync");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
      for (size_t k = 0; k < size_t(nctx) * nrhs; ++k) stats[k].time_ms = ms;
    return status;
  };
  const int status = run();
  if (status != DWA_OK && status != DWA_ENOCONV) (void)hipStreamSynchronize(st);
  for (int i = 0; i < nctx; ++i) ctxs[i]->stream = saved[i];
  if (status == DWA_ENOCONV) set_error("some field of the batch did not converge");
  return status;
}

// Extreme eigenvalues of a symmetric tridiagonal matrix (diagonal a[0..n), off-diagonal
// b[1..n)) by bisection on the Sturm count: the number of eigenvalues below x is the number
// of negative pivots of T - x.
static int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0) ++cnt;
  for (size_t i = 1; i < a.size(); ++i) {
    const double qq = (q == 0.0) ? 1e-300 : q;
    q = a[i] - x - b[i] * b[i] / qq;
    if (q < 0) ++cnt;
  }
  return cnt;
}

static double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, bool largest) {
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < a.size(); ++i) {  // Gershgorin interval
    const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i + 1]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const int target = largest ? int(a.size()) - 1 : 0;  // eigenvalue index (ascending)
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, mid) > target) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

int dwa_wilson_bounds(dwa_ctx* ctx, int steps, double* lmin, double* lmax) {
  DWA_TRY(check_ctx(ctx));
  if (steps < 2 || steps > 100000) return einval("steps must be in [2, 100000]");
  if (!lmin && !lmax) return einval("null outputs");
  const size_t vh = ctx->Vh, half = 12 * vh;  // one parity of a 4D field
  // 4D fields as [parity][12][Vh]: slices 0 and 1 of a workspace field (Ls >= 2)
  double2* v = static_cast<double2*>(ctx->w64[W_R]);
  double2* vp = static_cast<double2*>(ctx->w64[W_P]);
  double2* w = static_cast<double2*>(ctx->w64[W_Z]);
  double2* t = static_cast<double2*>(ctx->w64[W_Q]);
  const size_t n = 2 * half;
  // H_W = gamma_5 D_w (eq.(wilson)); out = H_W in, both parities: out_p = (4 + M5) in_p
  // - 1/2 H in_{1-p}, then gamma_5 (spins 2, 3 = components 6..11 of each parity)
  auto apply_hw = [&](double2* out, const double2* in) -> int {
    const HopOp hb{in + half, out, in, nullptr, -0.5, 4.0 + ctx->M5, 0.0, MIX_IDENTITY, 0, 1, nullptr};
    const HopOp hr{in, out + half, in + half, nullptr, -0.5, 4.0 + ctx->M5, 0.0, MIX_IDENTITY, 1, 1, nullptr};
    DWA_TRY(launch_hop(ctx, DWA_F64, hb, nullptr));
    DWA_TRY(launch_hop(ctx, DWA_F64, hr, nullptr));
    for (int par = 0; par < 2; ++par) {
      double2* lower = out + par * half + 6 * vh;
      DWA_TRY(launch_axpby(ctx, DWA_F64, lower, -1.0, lower, 0.0, 6 * vh));
    }
    return DWA_OK;
  };
  // Re <a, b> over both parities
  auto host_dot = [&](const double2* a, const double2* b, double* out) -> int {
    const void* aa[2] = {a, a + half};
    const void* bb[2] = {b, b + half};
    return host_slice_dots(ctx, aa, bb, 1, false, out);
  };
  // seeded Gaussian start vector
  {
    std::vector<double2> h(n);
    unsigned long long st = 0x9E3779B97F4A7C15ULL;
    auto unif = [&]() {  // xorshift64*, then a double in (0, 1)
      st ^= st >> 12;
      st ^= st << 25;
      st ^= st >> 27;
      return ((st * 2685821657736338717ULL) >> 11) * (1.0 / 9007199254740992.0) + 0.5 / 9007199254740992.0;
    };
    for (auto& z : h) {
      const double r = std::sqrt(-2.0 * std::log(unif())), ph = 2.0 * M_PI * unif();
      z = make_double2(r * std::cos(ph), r * std::sin(ph));
    }
    DWA_HIP(hipMemcpyAsync(v, h.data(), sizeof(double2) * n, hipMemcpyHostToDevice, ctx->stream), "start vector");
    DWA_HIP(hipStreamSynchronize(ctx->stream), "start vector sync");
  }
  double nv = 0.0;
  DWA_TRY(host_norm2(ctx, DWA_F64, v, &nv, n));
  DWA_TRY(launch_axpby(ctx, DWA_F64, v, 1.0 / std::sqrt(nv), v, 0.0, n));
  DWA_TRY(launch_zero(ctx, DWA_F64, vp, n));
  std::vector<double> al, be(1, 0.0);
  for (int j = 0; j < steps; ++j) {
    // w = H_W^2 v
    DWA_TRY(apply_hw(t, v));
    DWA_TRY(apply_hw(w, t));
    double a = 0.0;
    DWA_TRY(host_dot(v, w, &a));
    al.push_back(a);
    DWA_TRY(launch_axpby(ctx, DWA_F64, w, -a, v, 1.0, n));
    if (j > 0) DWA_TRY(launch_axpby(ctx, DWA_F64, w, -be.back(), vp, 1.0, n));
    double b2 = 0.0;
    DWA_TRY(host_norm2(ctx, DWA_F64, w, &b2, n));
    const double bn = std::sqrt(b2);
    if (!(bn > 1e-14 * std::fabs(a)) || j + 1 == steps) break;  // Krylov space exhausted
    be.push_back(bn);
    DWA_TRY(launch_axpby(ctx, DWA_F64, w, 1.0 / bn, w, 0.0, n));
    std::swap(vp, v);  // v_prev <- v
    std::swap(v, w);   // v <- w / |w|; the old v_prev becomes the next w
  }
  be.resize(al.size());
  const double emin = tridiag_eig(al, be, false), emax = tridiag_eig(al, be, true);
  if (lmin) *lmin = std::sqrt(std::max(emin, 0.0));
  if (lmax) *lmax = std::sqrt(std::max(emax, 0.0));
  return DWA_OK;
}

// Host-only access to the site-local matrices (no device needed); used to check
// the fifth-dimension algebra on the CPU.  out receives [2][Ls][Ls].
int dwa_debug_smatrix(const dwa_params* p, int kind, double* out) {
  if (!p || !out || !p->b || !p->c) return einval("null argument");
  if (kind < 0 || kind >= MIX_COUNT) return einval("bad matrix kind");
  std::vector<double> mix;
  std::string err;
  if (!build_smatrices(p->Ls, p->M5, p->m, p->alpha, p->b, p->c, mix, err)) return einval(err);
  std::memcpy(out, &mix[size_t(kind) * 2 * p->Ls * p->Ls], sizeof(double) * 2 * p->Ls * p->Ls);
  return DWA_OK;
}

}  // extern "C"
