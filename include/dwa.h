/*
 * dwa.h -- C-ABI of libdwa, the MI355X (gfx950) library for the alpha-Moebius
 * domain-wall operator of H. Neff, "A better conditioned Domain Wall Operator".
 *
 * The library applies the red-black operator D_bb = 1 - I_bb^-1 D_br I_rr^-1 D_rb
 * of D_alpha(m) (Sec. 3, eq.(redblack); D_alpha(m) is the block matrix of Sec. 2,
 * eq.(mobius1), with D_w the Wilson operator of eq.(wilson)) and its adjoint,
 * solves D_bb psi_b = phi' with CG on the normal equations (Sec. 3), and returns
 * the alpha-independent 4D propagator y_1 of D_1(m) P y = D_1(1) P b
 * (Sec. 2, eq.(tosolve1); App. B, eq.(tosolve)).
 *
 * Conventions (fixed here because the paper leaves them open):
 *   - lattice extents dims = {Lx, Ly, Lz, Lt}; every extent must be even and >= 2
 *     (the red-black split needs a bipartite lattice);
 *     4D sites are lexicographic, site = x + Lx*(y + Ly*(z + Lz*t));
 *   - mu = 0,1,2,3 is x,y,z,t; U_mu(x) sits on the link x -> x+mu and multiplies
 *     psi(x+mu); the backward hop uses U_mu(x-mu)^dagger;
 *   - chiral gamma basis, gamma5 = diag(1,1,-1,-1): P+ acts on spins 0,1, P- on 2,3;
 *   - fermion fields are periodic in x,y,z and antiperiodic in t when
 *     params.antiperiodic_t is non-zero (a factor -1 on hops across t = Lt-1 <-> 0);
 *   - slices s = 0..Ls-1 stand for the paper's i_5 = 1..Ls; b[s], c[s] belong to the
 *     row (output slice) of eq.(mobius1);
 *   - "black" is the even parity (x+y+z+t even), the parity the CG runs on.
 *
 * Layouts:
 *   canonical links    complex128 [4][V][3][3]        (mu, site, row, column)
 *   canonical 4D field complex128 [V][4][3]           (site, spin, colour)
 *   canonical 5D field complex128 [Ls][V][4][3]
 *   half-lattice field ("SoA") of one parity, precision prec:
 *                      [Ls][12][Vh] complex, component = spin*3 + colour,
 *                      Vh = V/2, checkerboard index cb = site/2;
 *                      F64: 16 B per complex, F32: 8 B, BF16: 4 B (bf16 re, bf16 im).
 * Complex numbers are interleaved (re, im).
 *
 * Memory ownership: every field pointer is a device pointer owned by the caller,
 * on the device that was current when the context was created.  The library never
 * frees caller memory.  The context owns its workspace (packed links, s-matrices,
 * solver vectors, reduction buffers); it allocates in dwa_create / dwa_set_links
 * and frees in dwa_destroy.  Operator calls do not allocate.
 *
 * Streams: operator calls enqueue their work on the stream given to dwa_create (0 =
 * default stream) and return without synchronising.  Solves wait for that stream, run on
 * a stream the context owns (one CG iteration is captured into a hipGraph there and
 * replayed between the host's convergence checks), synchronise on their checks and drain
 * before returning.  A context is not thread-safe: calls
 * on one context must not overlap (they share its workspace); different contexts are
 * independent.
 *
 * Errors: every call returns a dwa_status; nothing is thrown across the ABI.
 * Argument validation happens before any HIP call and returns DWA_EINVAL.
 * dwa_strerror() maps a status to text; dwa_last_error() gives the last detail
 * message of the calling thread.
 */
#ifndef DWA_H
#define DWA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dwa_ctx dwa_ctx;

typedef enum {
  DWA_OK = 0,
  DWA_EINVAL = -1,      /* invalid argument (bad extent, Ls < 2, alpha = 0, null pointer, ...) */
  DWA_ENOMEM = -2,      /* device allocation failed */
  DWA_EHIP = -3,        /* a HIP runtime call failed (including "no device") */
  DWA_ENOCONV = -4,     /* solver reached maxiter; the best iterate and stats are returned */
  DWA_EBREAKDOWN = -5,  /* CG breakdown: |D_bb p|^2 or |D_bb^dag r|^2 is zero or not finite */
  DWA_ENAN = -6,        /* non-finite value in an input field */
  DWA_ESTATE = -7       /* call out of order (e.g. no links set yet) */
} dwa_status;

typedef enum { DWA_F64 = 0, DWA_F32 = 1, DWA_BF16 = 2 } dwa_prec;

/* Physical parameters of D_alpha(m) (Sec. 2): Wilson mass M5 enters the diagonal
 * (4 + M5) of eq.(wilson) as written; m is the quark mass; alpha the new parameter;
 * b, c are host arrays of length Ls (the Moebius coefficients of eq.(coeff)). */
typedef struct {
  int dims[4];
  int Ls;
  double M5;
  double m;
  double alpha;
  const double *b;
  const double *c;
  int antiperiodic_t;
} dwa_params;

/* Solver options.
 *   tol          stop when |phi' - D_bb x| / |phi'| <= tol (recursive residual of CGLS,
 *                confirmed by an FP64 recomputation at the end)
 *   maxiter      cap on CG iterations (inner iterations summed for mixed precision)
 *   inner_prec   DWA_F64: plain FP64 CGLS.  DWA_F32 / DWA_BF16: CGLS with fields stored
 *                in that precision and FP32 arithmetic (BF16 keeps its accumulated
 *                solution in FP32), inside an FP64 loop that recomputes the true residual
 *   delta        mixed precision: the FP64 residual is recomputed when the low-precision
 *                residual has fallen by this factor since the last recomputation (e.g. 0.3)
 *   check_every  iterations between convergence reads on the host (>= 1)
 *   warm_start   non-zero: start from the x passed in instead of 0
 *   mixed_mode   mixed precision only.  DWA_MIXED_RELIABLE (0): one low-precision CGLS
 *                keeps its search direction across FP64 residual recomputations
 *                (reliable updates).  DWA_MIXED_DEFECT (1): defect correction, a fresh
 *                low-precision CGLS per FP64 residual. */
enum { DWA_MIXED_RELIABLE = 0, DWA_MIXED_DEFECT = 1 };
typedef struct {
  double tol;
  int maxiter;
  int inner_prec;
  double delta;
  int check_every;
  int warm_start;
  int mixed_mode;
} dwa_solve_opts;

typedef struct {
  int iters;            /* CG iterations (all precisions) */
  int outer;            /* FP64 residual recomputations (mixed precision) */
  int converged;
  double rel_resid;     /* final |phi' - D_bb x| / |phi'| recomputed in FP64 */
  double time_ms;       /* wall time of the solve */
  long long n_Dbb;      /* applications of D_bb or D_bb^dag */
} dwa_solve_stats;

/* Create a context for one lattice and parameter set on the current device.
 * Validates: every extent even and >= 2, Ls in [2, 32], alpha != 0, b/c non-null
 * and finite, an FP64 half field (Ls * 12 * V/2 * 16 bytes) below 4 GiB (the kernels
 * use 32-bit byte offsets), and that the site-local matrix I of eq.(redblack) is
 * invertible.
 * stream is a hipStream_t (NULL = default stream). */
int dwa_create(dwa_ctx **ctx, const dwa_params *p, void *stream);
int dwa_destroy(dwa_ctx *ctx);

/* Upload the gauge field: U_dev is canonical complex128 [4][V][3][3] on the device.
 * The antiperiodic phase is folded into U_t(t = Lt-1) and FP32/BF16 copies are made. */
int dwa_set_links(dwa_ctx *ctx, const void *U_dev);

/* Bytes of nrhs half-lattice SoA fields of precision prec stored back to back (the
 * batched calls take nrhs fields in one buffer); 0 for a null context, a bad precision
 * or nrhs < 1. */
size_t dwa_field_bytes(const dwa_ctx *ctx, int prec, int nrhs);
/* Number of sites V and slices Ls of the context (either pointer may be NULL). */
int dwa_get_sizes(const dwa_ctx *ctx, long long *V, int *Ls);

/* Canonical 5D complex128 [Ls][V][4][3] <-> SoA half field of the given parity
 * (0 = black/even, 1 = red/odd) and precision.  Unpack writes only the sites of
 * that parity and leaves the others untouched.  Precision conversion rounds to
 * nearest even. */
int dwa_pack_spinor5(dwa_ctx *ctx, int prec, void *dst_soa, const void *src_canon5, int parity);
int dwa_unpack_spinor5(dwa_ctx *ctx, int prec, void *dst_canon5, const void *src_soa, int parity);

/* out = D_w in on n independent 4D slices (eq.(wilson)); canonical complex128
 * [n][V][4][3], FP64.  out and in must not overlap. */
int dwa_apply_Dw(dwa_ctx *ctx, void *out, const void *in, int nslices);

/* out_b = D_bb in_b (eq.(redblack)) and out_b = D_bb^dagger in_b on black SoA fields of
 * precision prec (FP64, or FP32 / BF16 storage with FP32 arithmetic).  out_b and in_b
 * must not overlap. */
int dwa_apply_Dbb(dwa_ctx *ctx, int prec, void *out_b, const void *in_b);
int dwa_apply_Dbb_dag(dwa_ctx *ctx, int prec, void *out_b, const void *in_b);

/* dwa_apply_Dbb for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same operator and
 * kernels, bitwise the same result, but its two intermediate half fields (B G in, black,
 * and the first hop's output, red) live in a static 64 MiB device array of the library
 * (one per GPU, set up by dwa_create and held until the process ends) instead of the
 * context's workspace.  The call allocates nothing.  Limit: the two fields, each rounded up
 * to 256 bytes, must fit in 64 MiB (FP64 at 8^3 x 16, L_s = 12 takes 18.9 MB; BF16 at
 * 16^3 x 32, L_s = 16 takes 101 MB and is rejected); larger lattices return DWA_EINVAL.
 * Every call on one GPU uses that GPU's array, so calls that overlap in time on one GPU
 * (other threads, other streams, other contexts) race: serialise them.  Nothing in the
 * array has to start at zero (both fields are written in full before they are read). */
int dwa_apply_Dbb_static(dwa_ctx *ctx, int prec, void *out_b, const void *in_b);

/* One launch of the fused hop kernel: out = M_kind (H in), where H is the hopping sum
 * of eq.(wilson) without its -1/2, taken from the parity 1 - parity_out to parity_out
 * on every slice, and M_kind is a fifth-dimension matrix of dwa_debug_smatrix (kinds
 * 0..6; 0 = identity runs the hop alone).  D_bb is built from two such launches
 * (kinds 2 and 3) and D_bb^dag from kinds 5 and 6.  Half fields of precision prec;
 * out and in must not overlap.  Exposed for measurement and tests. */
int dwa_apply_hop(dwa_ctx *ctx, int prec, int parity_out, int kind, void *out, const void *in);

/* Tiles and block traversal of the fused hop.  A block of the hop kernel computes ns
 * consecutive checkerboard sites on all Ls slices (ns = 8, 16 or 32; Ls = 4, 8, 12, 16
 * have kernels for all three, any other Ls and the dense fallback run 8), and blocks
 * walk the lattice in one of three orders: 0 = t-slabs (default), 1 = checkerboard
 * order, 2 = z-planes per XCD.  Only the assignment of sites to blocks changes: every
 * site's arithmetic is the same, so D_bb and every hop output are bitwise identical
 * across configurations (CG reductions group their partial sums by block, so solver
 * scalars can differ in the last bits).  The defaults are ns = 16 for FP64, 32 for
 * FP32 / BF16, order 0. */
typedef struct {
  int prec;  /* storage precision */
  int ns;    /* sites per block */
  int order; /* block traversal */
  int nf;    /* fields per block when a batch is applied */
  int dense; /* 1: dense L_s x L_s fifth-dimension matrices (generic 8-site kernel),
                0: the O(L_s) sweep programs */
  int nrhs;  /* fields the configuration was timed on (1, or a batch) */
  double us; /* average time of one hop pair of D_bb (N hop, then G^-1 I^-1 hop with the
                x term) on nrhs fields, microseconds; negative if the configuration
                cannot run here (its LDS exceeds the device limit) */
} dwa_tune_entry;

/* Autotuner: time every tile and order of precision prec on this context's lattice,
 * and the dense fifth-dimension matrices (generic 8-site kernel) against the sweep
 * programs (reps timed pairs each after a warm-up; reps <= 0 means 10), and keep the
 * fastest for all later calls on the context.  When a batch is reserved
 * (dwa_reserve_batch) it then times, with that configuration, 1, 2, 3, 4, 6 and 12
 * fields per block on a batch of up to 12 fields: a block of the batched hop stages its
 * links once and applies them to nf fields in turn.  Uses the context's own workspaces
 * (no allocation; their contents are overwritten, nothing else is touched).  entries
 * (host, may be NULL) receives up to max_entries timings; *n_entries (may be NULL) the
 * number timed. */
int dwa_autotune(dwa_ctx *ctx, int prec, int reps, dwa_tune_entry *entries, int max_entries,
                 int *n_entries);

/* Set or read the configuration used for precision prec: ns sites per block, block
 * order, nf fields per block of a batched hop (1 by default), and dense = 1 for the
 * dense fifth-dimension matrices instead of the sweep programs (0 by default; a context
 * whose sweep programs failed their check at creation always runs dense, and
 * dwa_get_tuning reports it).  The dense matrices run in the generic 8-site kernels of
 * every precision-specific launch (hop, site-local mixes, CG updates).  dwa_set_tuning
 * rejects a tile other than 8, 16, 32, an order outside 0..2, nf outside 1..64, dense
 * other than 0 / 1, a tile other than 8 where the generic kernel runs, and a
 * configuration whose LDS exceeds the device limit (DWA_EINVAL).  Output pointers of
 * dwa_get_tuning may be NULL. */
int dwa_set_tuning(dwa_ctx *ctx, int prec, int ns, int order, int nf, int dense);
int dwa_get_tuning(const dwa_ctx *ctx, int prec, int *ns, int *order, int *nf, int *dense);

/* Solve D_bb x_b = rhs_b by CG on the normal equations (Sec. 3).  x_b and rhs_b are
 * FP64 black SoA fields.  Returns DWA_OK, DWA_ENOCONV (x_b holds the last iterate) or
 * DWA_EBREAKDOWN.  stats may be NULL. */
int dwa_cgne_solve(dwa_ctx *ctx, void *x_b, const void *rhs_b, const dwa_solve_opts *opts,
                   dwa_solve_stats *stats);

/* The 4D propagator y_1 for a 4D source eta (Sec. 2 and App. B): builds
 * rho = D_1(1) P (eta, 0, ..., 0), the Schur right-hand side
 * phi' = I_bb^-1 (rho_b - D_br I_rr^-1 rho_r), solves D_bb psi_b = phi' with
 * dwa_cgne_solve, reconstructs psi_r = I_rr^-1 (rho_r - D_rb psi_b) and extracts
 * y_1 = P- psi_1 + P+ psi_Ls.  y1 and eta are canonical complex128 [V][4][3] on the
 * device.  psi5 (optional, may be NULL) receives the full 5D solution psi, canonical. */
int dwa_propagator(dwa_ctx *ctx, void *y1, const void *eta, const dwa_solve_opts *opts,
                   dwa_solve_stats *stats, void *psi5);

/* The propagator of dwa_propagator with the Schur system in one of the forms of Sec. 3,
 * for comparing their CGNE iteration counts (FP64 CGLS, every scalar read on the host, so
 * all forms run the same algorithm; opts->tol and opts->maxiter are used):
 *   form 0: eq.(redblack),  D_bb = 1 - I_bb^-1 D_br I_rr^-1 D_rb;
 *   form 1: eq.(redblack1), I_bb - D_br I_rr^-1 D_rb = I_bb D_bb, right-hand side I_bb phi';
 *   form 2: eq.(redblack1) with every row s whose coefficient max(b_s, c_s) exceeds one
 *           divided by it (the row scaling the paper describes after eq.(redblack1)).
 * Each solve stops on its own relative residual <= tol; stats->rel_resid is the residual of
 * eq.(redblack), |phi' - D_bb psi_b| / |phi'|, of the result, so the forms compare at equal
 * accuracy.  All forms have the same solution, hence the same y_1.  DWA_EINVAL for another
 * form. */
int dwa_propagator_form(dwa_ctx *ctx, int form, void *y1, const void *eta, const dwa_solve_opts *opts,
                        dwa_solve_stats *stats);

/* The 4D overlap operator through the 5D engine (App. A: D^5_OV(m) =
 * R^-1 D_DW(1)^-1 D_DW(m) R, eq.(startprop); its (1,1) block is
 * D_OV(m) = 1/2 [(1 + m) + (1 - m) gamma_5 (S - 1)/(S + 1)] with S the product of the transfer
 * matrices of the context's b_i, c_i): out = D_OV(m) in = [P^-1 D_1(1)^-1 D_1(m) P (in, 0, ..,
 * 0)]_1.  One 5D solve: rho = D_1(m) P (in, 0, ..., 0) on the wall slices, D_alpha(1) psi =
 * rho by the red-black CGNE of dwa_cgne_solve with opts (the context's alpha, mass 1:
 * well conditioned), out = P- psi_1 + P+ psi_Ls.  The context must have mass 1 (DWA_EINVAL
 * otherwise); m is the overlap mass.  out and in are canonical complex128 [V][4][3] on the
 * device and must not overlap.  Its inverse for mass m is dwa_propagator on a context of
 * mass m.  Returns like dwa_propagator. */
int dwa_overlap_apply(dwa_ctx *ctx, double m, void *out, const void *in, const dwa_solve_opts *opts,
                      dwa_solve_stats *stats);

/* Change alpha of an existing context (eq.(mobius1): alpha multiplies the P+/P- terms
 * of every row; the 4D propagator does not depend on it, Sec. 2 / eq.(tosolve1)).
 * Rebuilds the site-local matrices for the new alpha after the context's stream has
 * drained; links and workspace are kept.  DWA_EINVAL for alpha = 0, non-finite alpha
 * or a singular I, with the context unchanged. */
int dwa_set_alpha(dwa_ctx *ctx, double alpha);

/* The alpha study of Sec. 3: for each alphas[i] (i < n) solve for y_1 of eta with the
 * options opts and record the solve statistics in stats[i] (iteration counts n(alpha)
 * under the residual of eq.(redblack)).  y1 receives n canonical complex128 [V][4][3]
 * fields back to back (device, n * V * 12 * 16 bytes).  The context's alpha is
 * restored on return.  Returns the first status other than DWA_OK (DWA_ENOCONV of a
 * single alpha does not stop the sweep). */
int dwa_alpha_sweep(dwa_ctx *ctx, const double *alphas, int n, void *y1, const void *eta,
                    const dwa_solve_opts *opts, dwa_solve_stats *stats);

/* Gradients of L = Re <eta', y_1> by the adjoint-state method (no equation of the paper
 * defines them; they follow from eq.(tosolve) / eq.(tosolve1) with y_1 = E psi,
 * D_alpha(m) psi = D_1(1) P b).  One forward solve gives psi, one adjoint solve gives
 * lambda with D_alpha(m)^dag lambda = E^dag eta' (red-black: CGNE on D_bb^dag, FP64),
 * and dL = Re <lambda, d(D_1(1) P b) - (d D_alpha) psi> is evaluated for
 *   gU     device complex128 [4][V][3][3]: dL/dRe U + i dL/dIm U per link entry, the
 *          link perturbation entering the backward hop as its conjugate transpose,
 *   geta   device complex128 [V][4][3]: dL/dRe eta + i dL/dIm eta,
 *   galpha host double: dL/dalpha (zero up to rounding: y_1 does not depend on alpha),
 *   gb, gc host double [Ls]: dL/db_s, dL/dc_s,
 *   L      host double: the loss, y1 device [V][4][3]: the propagator.
 * Any output may be NULL.  eta and eta_prime are device complex128 [V][4][3].  opts
 * applies to both solves: the adjoint solve (CGLS on D_bb^dag) runs in FP64 when
 * inner_prec is DWA_F64 and otherwise in inner_prec with FP64 reliable updates
 * (mixed_mode is not used there; warm_start applies to the forward solve only);
 * stats (may be NULL) receives two entries: forward, adjoint.
 * Returns DWA_ENOCONV if either solve did not converge (outputs still written). */
int dwa_propagator_adjoint(dwa_ctx *ctx, void *gU, void *geta, double *galpha, double *gb,
                           double *gc, double *L, void *y1, const void *eta,
                           const void *eta_prime, const dwa_solve_opts *opts,
                           dwa_solve_stats *stats);

/* Zolotarev coefficients (Sec. 3: the Zolotarev row of the table and the paragraph on
 * their ordering; App. A, eq.(polar)).  Host only, no device needed.
 * With b_i = c_i = omega_i the kernel of eq.(argument) is omega_i H, H = gamma_5 D_w, and
 * eq.(polar) approximates sign(H) by (1 - r(H)) / (1 + r(H)), r(x) = prod (1 - omega_i x) /
 * (1 + omega_i x).  Returned are the omega_i minimising max |r| on [lmin, lmax], the
 * spectrum of |H| (Zolotarev's third problem: 1/omega_j = lmax dn((2j - 1) K / (2 Ls), k'),
 * k'^2 = 1 - (lmin/lmax)^2), in the order ordering = 0 increasing in i_5, 1 concave (the
 * paper's choice: smallest at i_5 = 1 and Ls, largest in the centre), 2 decreasing.
 * omega (host, Ls doubles) receives them; delta (host, may be NULL) max |r| on the
 * interval, so |1 - sign approximation| <= 2 delta / (1 - delta) there.  DWA_EINVAL
 * unless 0 < lmin < lmax is finite and 1 <= Ls <= 32. */
int dwa_zolotarev(double lmin, double lmax, int Ls, int ordering, double *omega, double *delta);

/* Spectral bounds of the Wilson kernel |H|, H = gamma_5 D_w (eq.(wilson), the context's
 * links, M5 and boundary condition), for dwa_zolotarev: `steps` Lanczos steps on
 * H^2 = D_w^dag D_w from a seeded start vector, on the GPU, and the extreme eigenvalues of
 * the Lanczos tridiagonal matrix (Sturm bisection on the host).  lmin and lmax (host, either
 * may be NULL) receive their square roots.  Ritz values lie inside the spectrum: lmax is a
 * lower bound of the largest singular value of D_w and lmin an upper bound of the smallest;
 * both converge as steps grows (exact once steps reaches the dimension 12 V).  Uses the
 * context's workspace (no allocation).  DWA_EINVAL for steps outside [2, 100000]. */
int dwa_wilson_bounds(dwa_ctx *ctx, int steps, double *lmin, double *lmax);

/* Batches of right-hand sides (the paper's solves are 12 spin-colour sources per gauge
 * field, Sec. 3).  dwa_reserve_batch allocates the workspace for up to nmax fields of
 * this context (17 FP64 and 17 low-precision half fields per entry) and a
 * stream of its own; it replaces an earlier reservation.  Batched solves allocate
 * nothing. */
int dwa_reserve_batch(dwa_ctx *ctx, int nmax);

/* out = D_bb in for nrhs black SoA fields of precision prec stored back to back (one
 * batched launch per kernel; uses the batch workspace, nrhs <= the reservation).
 * out_norm2 (host, nrhs doubles, may be NULL) receives |out|^2 per field from the
 * kernel's own partial sums (the CGNE reduction). */
int dwa_apply_Dbb_batch(dwa_ctx *ctx, int prec, int nrhs, void *out, const void *in,
                        double *out_norm2);

/* y_1 for nrhs sources at once: eta and y1 hold nrhs canonical complex128 [V][4][3]
 * fields back to back (device).  Every field takes the path of dwa_propagator; the
 * batch shares each kernel launch (the fused hop reads a chunk's links once per XCD for
 * all fields), and the CGNE iteration body is replayed from a hipGraph between host
 * convergence checks.  opts->inner_prec = DWA_F64 runs FP64 CGNE; DWA_F32 / DWA_BF16
 * run batched low-precision CGNE with FP64 reliable updates (DWA_MIXED_RELIABLE: the
 * live fields of a context are updated together, at a check where one of them has
 * reduced its residual by opts->delta) or FP64 defect correction (DWA_MIXED_DEFECT).
 * stats (may be NULL) receives nrhs entries; outer counts the FP64 updates.  nrhs must
 * not exceed the reservation.  Returns DWA_ENOCONV if any field missed the tolerance. */
int dwa_propagator_batch(dwa_ctx *ctx, int nrhs, void *y1, const void *eta,
                         const dwa_solve_opts *opts, dwa_solve_stats *stats);

/* dwa_propagator_batch over several contexts (lattices of different sizes) in one
 * solve: nrhs[i] sources of ctxs[i] in eta[i] -> y1[i]; one hipGraph holds the CGNE
 * iteration of every context that still has a live field (it is captured again when a
 * context's fields have all stopped).  All contexts must be on one device and have reserved
 * their batches; the work runs on the first context's batch stream after every
 * context's stream has drained.  stats receives sum(nrhs) entries in context order. */
int dwa_propagator_multi(dwa_ctx *const *ctxs, int nctx, const int *nrhs, void *const *y1,
                         const void *const *eta, const dwa_solve_opts *opts,
                         dwa_solve_stats *stats);

/* Batched CGNE at the Schur level (Sec. 3: CG on the normal equation of the red-black
 * operator D_bb of eq.(redblack); the paper's workload is 12 spin-colour sources per
 * gauge field, solved together here): solve D_bb x = rhs for nrhs right-hand sides of
 * each of the nctx contexts (lattices of any size, one device) in one solve.
 *   rhs_b[i]  device, nrhs FP64 black SoA fields of ctxs[i] back to back
 *             (dwa_field_bytes(ctxs[i], DWA_F64, nrhs) bytes); read only;
 *   x_b[i]    device, same layout; receives the solutions (written once, at the end).
 * Every field runs the CGLS of dwa_cgne_solve from x = 0 (opts->warm_start must be 0);
 * opts->inner_prec = DWA_F64 runs FP64 CGLS, DWA_F32 / DWA_BF16 low-precision CGLS with
 * FP64 reliable updates or defect correction (opts->mixed_mode), as in
 * dwa_propagator_multi.  One hipGraph replays the iteration of all fields between host
 * checks.  Every context must have reserved at least nrhs fields (dwa_reserve_batch); the
 * work runs on the first context's batch stream after every context's stream has drained.
 * stats (host, may be NULL) receives nctx * nrhs entries, context-major; rel_resid is the
 * FP64 |rhs - D_bb x| / |rhs|.  Returns DWA_ENOCONV if any field missed the tolerance
 * (all solutions are still written), DWA_EINVAL on a bad argument (before any device
 * work). */
int dwa_cgne_solve_batch(dwa_ctx *const *ctxs, int nctx, int nrhs, void *const *x_b,
                         const void *const *rhs_b, const dwa_solve_opts *opts,
                         dwa_solve_stats *stats);

const char *dwa_strerror(int status);
const char *dwa_last_error(void);

/* Host-only (no device needed): the real Ls x Ls fifth-dimension matrices the
 * kernels apply, per chirality, out = [2][Ls][Ls] (index 0 = P+, 1 = P-).  kind:
 * 0 identity, 1 B G, 2 N = B I_1^-1, 3 G^-1 I_1^-1, 4 g5 I_1^-T G^-1, 5 N^T,
 * 6 G B^T g5, 7 I_1^-1, 8 I_1 G (the site-local block I of D_alpha, eq.(redblack)),
 * 9 (I_1 G)^T, 10 W I_1 G, 11 (W I_1 G)^T with W = diag(1 / max(1, b_s, c_s)) (the row
 * scaling of eq.(redblack1)).
 * Here D_1 = D_w B + C slice by slice, I_1 = (4 + M5) B + C and D_alpha = D_1 G
 * with G = diag(P- + alpha P+, alpha, ..., alpha, P+ + alpha P-) (Sec. 2). */
int dwa_debug_smatrix(const dwa_params *p, int kind, double *out);

#ifdef __cplusplus
}
#endif
#endif /* DWA_H */
