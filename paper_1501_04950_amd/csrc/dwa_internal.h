// Internal declarations of libdwa: storage types, the context, host helpers and
// kernel launchers.  Everything here is gfx950 (CDNA4, wave64) HIP.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dwa.h"

namespace dwa {

// ----------------------------------------------------------------------------
// complex arithmetic in the compute precision R (double for FP64 fields, float
// for FP32 and BF16 storage)
template <typename R>
struct cpx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmk(R a, R b) { return cpx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.re, s * a.im}; }
// i*a and -i*a
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_i(cpx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_mi(cpx<R> a) { return {a.im, -a.re}; }
// acc += u * v, acc += conj(u) * v
template <typename R>
__host__ __device__ __forceinline__ void cmac(cpx<R>& acc, cpx<R> u, cpx<R> v) {
  acc.re = fma(u.re, v.re, acc.re);
  acc.re = fma(-u.im, v.im, acc.re);
  acc.im = fma(u.re, v.im, acc.im);
  acc.im = fma(u.im, v.re, acc.im);
}
template <typename R>
__host__ __device__ __forceinline__ void cmac_conj(cpx<R>& acc, cpx<R> u, cpx<R> v) {
  acc.re = fma(u.re, v.re, acc.re);
  acc.re = fma(u.im, v.im, acc.re);
  acc.im = fma(u.re, v.im, acc.im);
  acc.im = fma(-u.im, v.re, acc.im);
}
template <typename R>
__host__ __device__ __forceinline__ R norm2(cpx<R> a) { return a.re * a.re + a.im * a.im; }

// ----------------------------------------------------------------------------
// storage traits: how one complex number of a field is held in HBM
struct F64 {
  using real = double;
  using elem = double2;
  static constexpr int prec = DWA_F64;
};
struct F32 {
  using real = float;
  using elem = float2;
  static constexpr int prec = DWA_F32;
};
struct BF16 {  // bf16 real part in the low half, bf16 imaginary part in the high half
  using real = float;
  using elem = uint32_t;
  static constexpr int prec = DWA_BF16;
};

// Storage of the solution accumulated by a low-precision CGLS: BF16 keeps only 8
// mantissa bits, too few to sum hundreds of small corrections, so its solution is
// held in FP32 (the operator fields stay BF16).
template <typename S> struct XAcc { using type = S; };
template <> struct XAcc<BF16> { using type = F32; };
inline int xacc_prec(int prec) { return prec == DWA_BF16 ? DWA_F32 : prec; }

__host__ __device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) {  // inf or nan: keep, force a quiet nan payload
    return (u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u);
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

template <typename S>
__device__ __forceinline__ cpx<typename S::real> ld(const typename S::elem* p, size_t i);
template <>
__device__ __forceinline__ cpx<double> ld<F64>(const double2* p, size_t i) {
  double2 v = p[i];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ cpx<float> ld<F32>(const float2* p, size_t i) {
  float2 v = p[i];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ cpx<float> ld<BF16>(const uint32_t* p, size_t i) {
  uint32_t v = p[i];
  return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
}

template <typename S>
__device__ __forceinline__ void st(typename S::elem* p, size_t i, cpx<typename S::real> v);
template <>
__device__ __forceinline__ void st<F64>(double2* p, size_t i, cpx<double> v) { p[i] = make_double2(v.re, v.im); }
template <>
__device__ __forceinline__ void st<F32>(float2* p, size_t i, cpx<float> v) { p[i] = make_float2(v.re, v.im); }
// Device rounding of two floats to a packed bf16 pair (real part in the low half),
// round-to-nearest-even by the gfx950 conversion instruction.  It agrees with
// f32_to_bf16_rne on every finite input.
__device__ __forceinline__ uint32_t pack_bf16x2(float re, float im) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 b2v __attribute__((ext_vector_type(2)));
  const f2v f = {re, im};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, b2v));
}
template <>
__device__ __forceinline__ void st<BF16>(uint32_t* p, size_t i, cpx<float> v) {
  p[i] = pack_bf16x2(v.re, v.im);
}

// Load of element byte_off / sizeof(elem) from a wave-uniform base: the 32-bit
// per-lane byte offset lets the compiler address through base (scalar registers) +
// offset (one vector register), with no 64-bit address arithmetic per load.
template <typename S>
__device__ __forceinline__ cpx<typename S::real> ldb(const void* base, unsigned byte_off) {
  return ld<S>(reinterpret_cast<const typename S::elem*>(static_cast<const char*>(base) + byte_off), 0);
}
template <typename S>
__device__ __forceinline__ void stb(void* base, unsigned byte_off, cpx<typename S::real> v) {
  st<S>(reinterpret_cast<typename S::elem*>(static_cast<char*>(base) + byte_off), 0, v);
}

inline size_t elem_bytes(int prec) { return prec == DWA_F64 ? 16 : (prec == DWA_F32 ? 8 : 4); }

// ----------------------------------------------------------------------------
// site-local fifth-dimension operators.  Each is a real Ls x Ls matrix per
// chirality (index 0 = P+, spins 0,1; index 1 = P-, spins 2,3), stored [2][Ls][Ls].
enum MixKind {
  MIX_IDENTITY = 0,
  MIX_BG,          // B G           : premix of the D_bb input
  MIX_N,           // N = B I^-1    : after the first hop of D_bb
  MIX_GINV_IINV,   // G^-1 I^-1     : after the second hop of D_bb, Schur prep, reconstruction
  MIX_G5_IINVT_GINV,  // g5 I^-T G^-1 : premix of the D_bb^dag input
  MIX_NT,          // N^T           : after the first hop of D_bb^dag
  MIX_G_BT_G5,     // G B^T g5      : after the second hop of D_bb^dag
  MIX_IINV,        // I^-1 (alpha = 1 part only, used by tests)
  MIX_I_ALPHA,     // I_1 G         : the site-local block I of D_alpha (tests, eq.(redblack1))
  MIX_I_ALPHA_T,   // (I_1 G)^T     : its adjoint, per chirality
  MIX_W_I,         // W I_1 G       : I with the rows of large coefficients scaled down
  MIX_W_I_T,       // (W I_1 G)^T
  MIX_COUNT
};

// Every site-local matrix above is a product of at most three simple factors per
// chirality, so it is applied as a short program of O(Ls) sweeps over the slices:
enum StageType {
  ST_SCALE = 1,   // y_s = A_s x_s
  ST_LBI = 2,     // lower cyclic bidiagonal: y_s = A_s x_s + B_s x_{s-1}, y_0 uses B_0 x_{Ls-1}
  ST_UBI = 3,     // upper cyclic bidiagonal: y_s = A_s x_s + B_s x_{s+1}, y_{Ls-1} uses B x_0
  ST_LSOLVE = 4,  // solve a lower cyclic bidiagonal system (A = 1/d, B = e/d, C = f, W = w)
  ST_USOLVE = 5,  // solve an upper cyclic bidiagonal system
  ST_DENSE = 6    // fallback: the dense Ls x Ls matrix
};
constexpr int kMaxStages = 3;
constexpr int kLsPad = 32;  // coefficient rows are padded to 32 slices
// meta: [MIX_COUNT][2][4] = {nstages, type0, type1, type2}
// coef: [MIX_COUNT][2][kMaxStages][4][kLsPad] rows A, B, C and W (w in W[0])
struct SweepTables {
  std::vector<int> meta;
  std::vector<double> coef;
};

// Host construction (FP64) of all site-local matrices and their sweep programs (each
// checked against its dense matrix; a program that does not reproduce it to 1e-12 is
// replaced by ST_DENSE).  Returns false and a message when the site-local block I is
// singular or badly conditioned.
bool build_smatrices(int Ls, double M5, double m, double alpha, const double* b, const double* c,
                     std::vector<double>& out /* [MIX_COUNT][2][Ls][Ls] */, std::string& err,
                     SweepTables* sweeps = nullptr);

// ----------------------------------------------------------------------------
// device-side solver scalars
struct DevScalars {
  double gamma;   // |z|^2 of the current CGLS step
  double a;       // step length
  double beta;
  double qq;      // |D_bb p|^2
  double zz;      // |D_bb^dag r|^2
  double rr;      // |r|^2 (recursive residual)
  double b2;      // |rhs|^2
  double aux;     // spare
  int flags;      // bit 0: |q|^2 not positive/finite; bit 1: |z|^2 not finite
  int active;     // 0: the field is frozen (converged or stopped), set by the host
  int pad[2];
};

struct PrecFields {  // one precision's copy of the links
  void* links = nullptr;  // [2][4][9][Vh] elems, boundary phase folded
};

// FP64 workspace roles (black fields unless noted)
enum W64Role {
  W_R = 0, W_P, W_Z, W_Q, W_W, W_U, W_T /* red */, W_X, W_OPB, W_OPR /* red */,
  W_RHO_B, W_RHO_R /* red */, W_CHI_B, W_CHI_R /* red */, W_PHI, W_PSI_B, W_PSI_R /* red */,
  W_RES,
  W64_COUNT
};
// low-precision (F32 or BF16 storage) workspace roles
enum LowRole { L_R = 0, L_P, L_Z, L_Q, L_W, L_U, L_T /* red */, L_X, L_OPB, L_OPR /* red */, LOW_COUNT };

}  // namespace dwa

namespace dwa {
// FP64 roles of a batch of fields (dwa_reserve_batch): solution, right-hand side, CGLS
// vectors, residual and temporaries, and the propagator's source and prep fields
enum BatchRole {
  B_X = 0, B_PHI, B_R, B_P, B_Z, B_Q, B_W, B_U, B_T /* red */, B_RES, B_OPB, B_OPR /* red */,
  B_RHO_B, B_RHO_R, B_CHI_B, B_CHI_R, B_PSI_R, B_COUNT
};
// low-precision roles of a batch: CGLS vectors of the inner solve, its right-hand side
// and (FP32, also for BF16 fields) its accumulated solution
enum BatchLowRole { BL_R = 0, BL_P, BL_Z, BL_Q, BL_W, BL_U, BL_T /* red */, BL_RHS, BL_COUNT };
struct BatchWs {
  int nmax = 0;                   // fields reserved
  void* f64[B_COUNT] = {};        // nmax fields each
  void* lo[3][BL_COUNT] = {};     // per storage precision (index = dwa_prec; [0] unused)
  void* xacc = nullptr;           // FP32 accumulated low-precision solution, nmax fields
  DevScalars* d_scal = nullptr;   // nmax
  DevScalars* h_scal = nullptr;   // pinned mirror
  double* partials = nullptr;     // 4 banks of nmax * bank_elems
  size_t bank_elems = 0;          // per field
  double* d_coef = nullptr;       // per-field coefficient tables (4 * nmax)
  double* h_coef = nullptr;       // pinned staging for d_coef
  int* h_active = nullptr;        // pinned staging for the active flags
  hipStream_t stream = nullptr;   // capture stream of batched solves
};
}  // namespace dwa

namespace dwa {
// fused-hop tiles (sites per block) and block traversal orders
constexpr int kTileCount = 3;
constexpr int kTiles[kTileCount] = {8, 16, 32};
inline int tile_index(int ns) { return ns == 8 ? 0 : (ns == 16 ? 1 : 2); }
inline bool valid_tile(int ns) { return ns == 8 || ns == 16 || ns == 32; }
// SLAB: (t-slab, z, t in slab, y, x), each XCD a run of it; LEX: checkerboard order;
// ZDOM: XCD k owns z-planes [k Lz/8, (k+1) Lz/8), walked t-major.
enum HopOrder { ORDER_SLAB = 0, ORDER_LEX = 1, ORDER_ZDOM = 2, ORDER_COUNT = 3 };
struct HopTune {
  int ns = 16;
  int order = ORDER_SLAB;
  int nf = 1;          // fields per block when a batch is applied
  bool dense = false;  // dense fifth-dimension matrices instead of the sweeps
};
}  // namespace dwa

struct dwa_ctx {
  int dims[4];
  int Ls;
  long long V, Vh;
  double M5, m, alpha;
  std::vector<double> b, c;
  int antiperiodic_t;
  hipStream_t stream;
  hipStream_t cap_stream = nullptr;  // the context's own stream: single-field solves capture
                                     // their CG iteration into a hipGraph on it
  int device;
  bool links_set = false;

  // geometry
  int* d_nbr = nullptr;   // [2][8][Vh] neighbour cb index for an output site of parity p
  int* d_cb2lex = nullptr;  // [2][Vh]
  // fused-hop block -> chunk of sites, one table per traversal order and tile size
  int* d_blkmap[dwa::ORDER_COUNT][dwa::kTileCount] = {};
  dwa::HopTune tune[3];            // per storage precision (autotuner or default)
  size_t max_lds = 64 * 1024;      // device limit on one block's LDS
  // s-matrices (FP64 and FP32 copies), [MIX_COUNT][2][Ls][Ls]
  double* d_mix64 = nullptr;
  float* d_mix32 = nullptr;
  int* d_sweep_meta = nullptr;     // [MIX_COUNT][2][4]
  double* d_sweep64 = nullptr;     // [MIX_COUNT][2][kMaxStages][4][kLsPad]
  float* d_sweep32 = nullptr;
  std::vector<int> sweep_meta_host;
  bool dense_mix = false;          // some sweep program failed its check: dense matrices
  size_t hop_min_lds = 0;          // lower bound on a fused hop block's LDS (limits occupancy)
  std::vector<double> h_mix;
  // links per precision
  dwa::PrecFields prec[3];
  // FP64 workspace, one vector per W64Role
  void* w64[dwa::W64_COUNT] = {nullptr};
  // low-precision workspace for the inner solver (F32 or BF16 storage), one per LowRole
  void* w32[dwa::LOW_COUNT] = {nullptr};
  void* w16[dwa::LOW_COUNT] = {nullptr};
  double* d_partials = nullptr;     // reduction partials, 4 banks
  size_t partials_per_bank = 0;
  dwa::DevScalars* d_scal = nullptr;
  dwa::DevScalars* h_scal = nullptr;  // pinned
  double* d_red = nullptr;          // small result slots for standalone reductions
  dwa::BatchWs batch;               // dwa_reserve_batch
};

namespace dwa {

// Sites per block of the fused hop.  The Ls values with their own kernels (4, 8, 12, 16)
// are compiled for tiles of 8, 16 and 32 sites, and the context's tuning picks one per
// storage precision; the generic (any other Ls) and dense kernels always run 8.
inline bool hop_specialised(int Ls, bool dense) {
  return !dense && (Ls == 4 || Ls == 8 || Ls == 12 || Ls == 16);
}
// Dense fifth-dimension matrices for precision prec: forced for the context (a sweep
// program failed its check, or DWA_DENSE_MIX) or chosen by the tuning.
inline bool use_dense(const dwa_ctx* ctx, int prec) { return ctx->dense_mix || ctx->tune[prec].dense; }
inline int hop_sites_per_block(const dwa_ctx* ctx, int prec) {
  return hop_specialised(ctx->Ls, use_dense(ctx, prec)) ? ctx->tune[prec].ns : 8;
}

// kernel launchers (kernels.hip)
struct HopOp {
  const void* in;       // SoA field of the input parity
  void* out;            // SoA field of the output parity
  const void* pre;      // optional, output parity: h' = hop_coef * H in + pre_coef * pre
  const void* post;     // optional, output parity: out = M h' + post_coef * post
  double hop_coef, pre_coef, post_coef;
  int mix;              // MixKind applied to h' (MIX_IDENTITY = none)
  int parity_out;
  int nslices;          // number of 5D slices (Ls, or n for plain D_w)
  double* partials;     // optional per-block |out|^2 partial sums (grouped per field)
  int nrhs = 1;         // batch of fields, field_elems apart (partials: nblocks per field)
};

int launch_hop(dwa_ctx* ctx, int prec, const HopOp& op, int* nblocks_out);
// Batched forms: nrhs fields field_elems(ctx) apart; per-field partial sums are packed
// (field r at partials[r * nblocks ...]) and per-field coefficient tables are device
// arrays (axpby: (a, b) pairs; convert: scales).
int launch_smix(dwa_ctx* ctx, int prec, int mix, void* out, const void* in, const void* post,
                double post_coef, int nslices, double* partials, int* nblocks_out, int nrhs = 1);
int launch_pack_links(dwa_ctx* ctx, int prec, void* dst, const void* src_canon);
int launch_pack5(dwa_ctx* ctx, int prec, void* dst_soa, const void* src_canon, int parity,
                 int nslices);
int launch_unpack5(dwa_ctx* ctx, int prec, void* dst_canon, const void* src_soa, int parity,
                   int nslices);
int launch_convert(dwa_ctx* ctx, int prec_out, void* out, int prec_in, const void* in, size_t n,
                   double scale, int nrhs = 1, const double* scales = nullptr);
int launch_zero(dwa_ctx* ctx, int prec, void* p, size_t n, int nrhs = 1);
int launch_axpby(dwa_ctx* ctx, int prec, void* y, double a, const void* x, double b, size_t n,
                 int nrhs = 1, const double* ab = nullptr);
int launch_norm2(dwa_ctx* ctx, int prec, const void* x, size_t n, double* partials, int* nblocks,
                 int nrhs = 1);
int launch_sum_partials(dwa_ctx* ctx, const double* partials, int n, double* out);
// X += scale x_l, x_l = 0 (x_l in FP32 or FP64; per-field scales when given)
int launch_fold_acc(dwa_ctx* ctx, int xprec, void* X, void* xl, size_t n, double scale, int nrhs = 1,
                    const double* scales = nullptr);
// RES = PHI - Q in FP64 and per-block partial sums of |RES|^2 (nblocks per field)
int launch_residual(dwa_ctx* ctx, void* res, const void* phi, const void* q, size_t n, double* partials,
                    int* nblocks, int nrhs = 1);
// rho = D_1(ms) P (eta, 0, ..., 0) on the two wall slices: chi (the D_w part) and aux (the
// site-local part); the propagator uses ms = 1 (eq.(tosolve1))
int launch_source(dwa_ctx* ctx, void* chi_b, void* chi_r, void* aux_b, void* aux_r, const void* eta,
                  double ms = 1.0);
int launch_extract(dwa_ctx* ctx, void* y1, const void* psi_b, const void* psi_r);
int launch_check_finite(dwa_ctx* ctx, const void* canon, size_t ncomplex, int* d_flag);

// CGLS building blocks (templated on precision inside kernels.hip).  In update1, x
// has storage xacc_prec(prec); the other fields have storage prec.
// adj = true runs the updates of CGLS on D_bb^dag (premixes swapped).  With qparts
// (nq partials of |q|^2 per field) update 1 also does the finalize of a = gamma/|q|^2,
// and with zparts (nz partials of |z|^2) it takes gamma from them; with zparts update 2
// does the finalize of beta = |z|^2 / gamma.
int launch_cg_update1(dwa_ctx* ctx, int prec, void* x, void* r, void* w, const void* p,
                      const void* q, DevScalars* s, double* partials, int* nblocks,
                      bool adj = false, int nrhs = 1, const double* qparts = nullptr, int nq = 0,
                      const double* zparts = nullptr, int nz = 0);
int launch_cg_update2(dwa_ctx* ctx, int prec, void* p, void* u, const void* z,
                      DevScalars* s, bool adj = false, int nrhs = 1, const double* zparts = nullptr,
                      int nz = 0);
// one block per field: s[r] from partials_a[r * na ...] and partials_b[r * nb ...];
// which 2: CG set-up (gamma, rr = b2), which 4: rr for a host check
int launch_cg_finalize(dwa_ctx* ctx, int which, DevScalars* s, const double* partials_a, int na,
                       const double* partials_b, int nb, int nrhs = 1);
// gamma *= f for nrhs fields (per-field factors fs[k] when fs is given)
int launch_scale_gamma(dwa_ctx* ctx, DevScalars* s, double f, int nrhs = 1,
                       const double* fs = nullptr);

// gradient path (adjoint.hip), FP64 SoA fields; "lt" is g5 lambda
int launch_adj_source(dwa_ctx* ctx, void* f_b, void* f_r, const void* eta_p);
int launch_omega(dwa_ctx* ctx, void* ob, void* oc, const void* psi, const void* eta, int par);
int launch_jpsi(dwa_ctx* ctx, void* out, const void* psi);
int slice_dot_blocks(size_t per_slice);
int launch_slice_dot(dwa_ctx* ctx, const void* a, const void* b, int nslices, size_t vh, bool g5,
                     double* partials);
int launch_force(dwa_ctx* ctx, void* gU, const void* lt_b, const void* lt_r, const void* ph_b,
                 const void* ph_r);
int launch_geta(dwa_ctx* ctx, void* geta, const void* lt_b, const void* lt_r, const void* dw_b,
                const void* dw_r);

// per-precision launchers (kcommon.h), instantiated in kernels_{f64,f32,bf16}.hip
template <typename S> int launch_hop_p(dwa_ctx*, const HopOp&, int*);
template <typename S> int launch_smix_p(dwa_ctx*, int, void*, const void*, const void*, double, int,
                                        double*, int*, int);
template <typename S> int launch_update1_p(dwa_ctx*, void*, void*, void*, const void*, const void*,
                                           DevScalars*, double*, int*, bool, int, const double*, int,
                                           const double*, int);
template <typename S> int launch_update2_p(dwa_ctx*, void*, void*, const void*, DevScalars*,
                                           bool, int, const double*, int);
template <typename S> int norm2_p(dwa_ctx*, const void*, size_t, double*, int*, int);
template <typename S> int axpby_p(dwa_ctx*, void*, double, const void*, double, size_t, int,
                                  const double*);
template <typename S> int zero_p(dwa_ctx*, void*, size_t, int);
template <typename S> int pack5_p(dwa_ctx*, void*, const void*, int, int);
template <typename S> int unpack5_p(dwa_ctx*, void*, const void*, int, int);
template <typename S> int pack_links_p(dwa_ctx*, void*, const void*);
template <typename SO, typename SI> int convert_p(dwa_ctx*, void*, const void*, size_t, double, int,
                                                  const double*);

size_t field_elems(const dwa_ctx* ctx);  // Ls * 12 * Vh complex numbers
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);
// the static scratch of dwa_apply_Dbb_static (scratch.hip): per-device address lookup
// (once per device, with that device current) and its size
int scratch_init(int device);
size_t scratch_bytes();

}  // namespace dwa
