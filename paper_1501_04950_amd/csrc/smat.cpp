// Host construction of the site-local fifth-dimension operators of D_alpha(m).
//
// Writing D_{s+} = b_s D_w + 1 and D_{s-} = c_s D_w - 1 (eq.(coeff)) into the rows
// of the alpha = 1 operator of eq.(mobius1) gives, slice by slice,
//   (D_1 psi)_s = D_w chi_s + omega_s,
//   chi_s   = b_s psi_s + c_s (P- psi_{s+1} + P+ psi_{s-1}),
//   omega_s = psi_s - (P- psi_{s+1} + P+ psi_{s-1}),
// with the walls closed by psi_{Ls} -> -m psi_0 and psi_{-1} -> -m psi_{Ls-1}.  So
// D_1 = D_w B + C with real Ls x Ls matrices B, C per chirality:
//   P+ : B lower bidiagonal (diag b_s, sub c_s, corner B[0][Ls-1] = -m c_0),
//        C diag 1, sub -1, corner C[0][Ls-1] = +m;
//   P- : B upper bidiagonal (diag b_s, super c_s, corner B[Ls-1][0] = -m c_{Ls-1}),
//        C diag 1, super -1, corner C[Ls-1][0] = +m.
// The column scaling of Sec. 2 (D_alpha P = D_1 P A) is the right factor G:
// D_alpha = D_1 G with G = diag(P- + alpha P+, alpha, ..., alpha, P+ + alpha P-).
// Splitting D_w = (4 + M5) - H/2 (H the hopping sum of eq.(wilson)), the site-local
// block of D_alpha is I_1 G with I_1 = (4 + M5) B + C, and the hopping block is
// -1/2 H B G.  The red-black operator of eq.(redblack) then reads
//   D_bb = 1 - 1/4 G^-1 I_1^-1 H_br N H_rb B G,       N = B I_1^-1,
//   D_bb^dag = 1 - 1/4 G B^T g5 H_br N^T H_rb g5 I_1^-T G^-1
// (the adjoint uses H_rb^dag = g5 H_br g5 and that B, N, I_1, G are real and act
// within one chirality).  This file builds every matrix these formulas need.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dwa_internal.h"

namespace dwa {

namespace {

using Mat = std::vector<double>;  // row-major n x n

Mat zeros(int n) { return Mat(size_t(n) * n, 0.0); }
Mat eye(int n) {
  Mat a = zeros(n);
  for (int i = 0; i < n; ++i) a[i * n + i] = 1.0;
  return a;
}
Mat mul(const Mat& a, const Mat& b, int n) {
  Mat c = zeros(n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double aik = a[i * n + k];
      if (aik == 0.0) continue;
      for (int j = 0; j < n; ++j) c[i * n + j] += aik * b[k * n + j];
    }
  return c;
}
Mat transpose(const Mat& a, int n) {
  Mat t = zeros(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t[j * n + i] = a[i * n + j];
  return t;
}
double norm_inf(const Mat& a, int n) {
  double best = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += std::fabs(a[i * n + j]);
    best = s > best ? s : best;
  }
  return best;
}
// Gauss-Jordan inverse with partial pivoting; false if singular.
bool inverse(const Mat& a, int n, Mat& inv) {
  Mat w = a;
  inv = eye(n);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(w[r * n + col]) > std::fabs(w[piv * n + col])) piv = r;
    if (w[piv * n + col] == 0.0 || !std::isfinite(w[piv * n + col])) return false;
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(w[piv * n + j], w[col * n + j]);
        std::swap(inv[piv * n + j], inv[col * n + j]);
      }
    double d = 1.0 / w[col * n + col];
    for (int j = 0; j < n; ++j) {
      w[col * n + j] *= d;
      inv[col * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = w[r * n + col];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        w[r * n + j] -= f * w[col * n + j];
        inv[r * n + j] -= f * inv[col * n + j];
      }
    }
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// sweep programs

namespace {

struct Stage {
  int type = 0;
  double A[kLsPad] = {0}, B[kLsPad] = {0}, C[kLsPad] = {0}, W = 0.0;
};

Stage scale_stage(const std::vector<double>& d) {
  Stage st;
  st.type = ST_SCALE;
  for (size_t s = 0; s < d.size(); ++s) st.A[s] = d[s];
  return st;
}

// a cyclic bidiagonal matrix: lower (entries [s][s-1], corner [0][Ls-1]) or upper
// (entries [s][s+1], corner [Ls-1][0])
Stage bidiag_stage(const Mat& M, int n, bool lower) {
  Stage st;
  st.type = lower ? ST_LBI : ST_UBI;
  for (int s = 0; s < n; ++s) {
    st.A[s] = M[s * n + s];
    if (lower) st.B[s] = s >= 1 ? M[s * n + (s - 1)] : M[0 * n + (n - 1)];
    else st.B[s] = s + 1 < n ? M[s * n + (s + 1)] : M[(n - 1) * n + 0];
  }
  return st;
}

// solve with a cyclic bidiagonal matrix.  Lower: y_s = (x_s - e_s y_{s-1}) / d_s with
// y_{-1} -> corner * y_{Ls-1}; writing y_s = a_s + f_s y_{Ls-1} gives a forward sweep for
// a_s, the closure y_{Ls-1} = a_{Ls-1} / (1 - f_{Ls-1}) and a second pass.  Upper mirrors
// it with y_0.
Stage solve_stage(const Mat& M, int n, bool lower) {
  Stage st;
  st.type = lower ? ST_LSOLVE : ST_USOLVE;
  std::vector<double> d(n), e(n);
  for (int s = 0; s < n; ++s) {
    d[s] = M[s * n + s];
    if (lower) e[s] = s >= 1 ? M[s * n + (s - 1)] : M[0 * n + (n - 1)];
    else e[s] = s + 1 < n ? M[s * n + (s + 1)] : M[(n - 1) * n + 0];
  }
  for (int s = 0; s < n; ++s) {
    st.A[s] = 1.0 / d[s];
    st.B[s] = e[s] / d[s];
  }
  if (lower) {
    st.C[0] = -st.B[0];
    for (int s = 1; s < n; ++s) st.C[s] = -st.B[s] * st.C[s - 1];
    st.W = 1.0 / (1.0 - st.C[n - 1]);
  } else {
    st.C[n - 1] = -st.B[n - 1];
    for (int s = n - 2; s >= 0; --s) st.C[s] = -st.B[s] * st.C[s + 1];
    st.W = 1.0 / (1.0 - st.C[0]);
  }
  return st;
}

void apply_stage_host(const Stage& st, int n, std::vector<double>& v) {
  std::vector<double> x = v;
  switch (st.type) {
    case ST_SCALE:
      for (int s = 0; s < n; ++s) v[s] = st.A[s] * x[s];
      break;
    case ST_LBI:
      for (int s = 0; s < n; ++s) v[s] = st.A[s] * x[s] + st.B[s] * x[(s + n - 1) % n];
      break;
    case ST_UBI:
      for (int s = 0; s < n; ++s) v[s] = st.A[s] * x[s] + st.B[s] * x[(s + 1) % n];
      break;
    case ST_LSOLVE: {
      v[0] = st.A[0] * x[0];
      for (int s = 1; s < n; ++s) v[s] = st.A[s] * x[s] - st.B[s] * v[s - 1];
      const double Y = st.W * v[n - 1];
      for (int s = 0; s < n - 1; ++s) v[s] += st.C[s] * Y;
      v[n - 1] = Y;
      break;
    }
    case ST_USOLVE: {
      v[n - 1] = st.A[n - 1] * x[n - 1];
      for (int s = n - 2; s >= 0; --s) v[s] = st.A[s] * x[s] - st.B[s] * v[s + 1];
      const double Y = st.W * v[0];
      for (int s = 1; s < n; ++s) v[s] += st.C[s] * Y;
      v[0] = Y;
      break;
    }
    default:
      break;
  }
}

}  // namespace

bool build_smatrices(int Ls, double M5, double m, double alpha, const double* b, const double* c,
                     std::vector<double>& out, std::string& err, SweepTables* sweeps) {
  const int n = Ls;
  // chirality 0 = P+, 1 = P-
  Mat B[2], C[2], G[2], Ginv[2];
  for (int ch = 0; ch < 2; ++ch) {
    B[ch] = zeros(n);
    C[ch] = zeros(n);
    G[ch] = zeros(n);
    Ginv[ch] = zeros(n);
    for (int s = 0; s < n; ++s) {
      B[ch][s * n + s] = b[s];
      C[ch][s * n + s] = 1.0;
    }
  }
  for (int s = 0; s < n; ++s) {
    if (s >= 1) {  // P+ couples to s-1
      B[0][s * n + (s - 1)] += c[s];
      C[0][s * n + (s - 1)] += -1.0;
    }
    if (s + 1 < n) {  // P- couples to s+1
      B[1][s * n + (s + 1)] += c[s];
      C[1][s * n + (s + 1)] += -1.0;
    }
  }
  B[0][0 * n + (n - 1)] += -m * c[0];
  C[0][0 * n + (n - 1)] += m;
  B[1][(n - 1) * n + 0] += -m * c[n - 1];
  C[1][(n - 1) * n + 0] += m;
  for (int s = 0; s < n; ++s) {
    // G+ = diag(alpha, ..., alpha, 1), G- = diag(1, alpha, ..., alpha)
    double gp = (s == n - 1) ? 1.0 : alpha;
    double gm = (s == 0) ? 1.0 : alpha;
    G[0][s * n + s] = gp;
    G[1][s * n + s] = gm;
    Ginv[0][s * n + s] = 1.0 / gp;
    Ginv[1][s * n + s] = 1.0 / gm;
  }

  out.assign(size_t(MIX_COUNT) * 2 * n * n, 0.0);
  auto put = [&](int kind, int ch, const Mat& a) {
    std::memcpy(&out[(size_t(kind) * 2 + ch) * n * n], a.data(), sizeof(double) * n * n);
  };
  for (int ch = 0; ch < 2; ++ch) {
    const double g5 = ch == 0 ? 1.0 : -1.0;
    Mat I1 = zeros(n);
    for (int k = 0; k < n * n; ++k) I1[k] = (4.0 + M5) * B[ch][k] + C[ch][k];
    Mat I1inv;
    if (!inverse(I1, n, I1inv)) {
      err = "site-local block I of D_alpha is singular";
      return false;
    }
    double cond = norm_inf(I1, n) * norm_inf(I1inv, n);
    if (!(cond < 1e14)) {
      err = "site-local block I of D_alpha is ill-conditioned (cond > 1e14)";
      return false;
    }
    Mat N = mul(B[ch], I1inv, n);
    Mat I1invT = transpose(I1inv, n);
    Mat BT = transpose(B[ch], n);
    Mat g5IinvTGinv = mul(I1invT, Ginv[ch], n);
    for (auto& v : g5IinvTGinv) v *= g5;
    Mat GBTg5 = mul(G[ch], BT, n);
    for (auto& v : GBTg5) v *= g5;
    put(MIX_IDENTITY, ch, eye(n));
    put(MIX_BG, ch, mul(B[ch], G[ch], n));
    put(MIX_N, ch, N);
    put(MIX_GINV_IINV, ch, mul(Ginv[ch], I1inv, n));
    put(MIX_G5_IINVT_GINV, ch, g5IinvTGinv);
    put(MIX_NT, ch, transpose(N, n));
    put(MIX_G_BT_G5, ch, GBTg5);
    put(MIX_IINV, ch, I1inv);
    put(MIX_I_ALPHA, ch, mul(I1, G[ch], n));
    put(MIX_I_ALPHA_T, ch, transpose(mul(I1, G[ch], n), n));
    // row scaling of eq.(redblack1) (Sec. 3): a row s whose coefficient exceeds one is
    // divided by it; the coefficient of row s is max(b_s, c_s) (b_s = c_s = omega_s for
    // Zolotarev coefficients)
    Mat Wd = zeros(n);
    for (int s = 0; s < n; ++s) Wd[s * n + s] = 1.0 / std::max(1.0, std::max(std::fabs(b[s]), std::fabs(c[s])));
    const Mat WI = mul(Wd, mul(I1, G[ch], n), n);
    put(MIX_W_I, ch, WI);
    put(MIX_W_I_T, ch, transpose(WI, n));

    if (sweeps) {
      // P+ (ch 0): B and I_1 are lower cyclic bidiagonal; P- (ch 1): upper
      const bool low = ch == 0;
      std::vector<double> g(n), ginv(n), sg(n), sginv(n);
      for (int s = 0; s < n; ++s) {
        g[s] = G[ch][s * n + s];
        ginv[s] = 1.0 / g[s];
        sg[s] = g5 * g[s];
        sginv[s] = g5 * ginv[s];
      }
      const Mat IT = transpose(I1, n);
      std::vector<std::vector<Stage>> prog(MIX_COUNT);
      prog[MIX_BG] = {scale_stage(g), bidiag_stage(B[ch], n, low)};
      prog[MIX_N] = {solve_stage(I1, n, low), bidiag_stage(B[ch], n, low)};
      prog[MIX_GINV_IINV] = {solve_stage(I1, n, low), scale_stage(ginv)};
      prog[MIX_G5_IINVT_GINV] = {scale_stage(sginv), solve_stage(IT, n, !low)};
      prog[MIX_NT] = {bidiag_stage(BT, n, !low), solve_stage(IT, n, !low)};
      prog[MIX_G_BT_G5] = {bidiag_stage(BT, n, !low), scale_stage(sg)};
      prog[MIX_IINV] = {solve_stage(I1, n, low)};
      prog[MIX_I_ALPHA] = {scale_stage(g), bidiag_stage(I1, n, low)};
      std::vector<double> wrow(n);
      for (int s = 0; s < n; ++s) wrow[s] = 1.0 / std::max(1.0, std::max(std::fabs(b[s]), std::fabs(c[s])));
      prog[MIX_I_ALPHA_T] = {bidiag_stage(IT, n, !low), scale_stage(g)};
      prog[MIX_W_I] = {scale_stage(g), bidiag_stage(I1, n, low), scale_stage(wrow)};
      prog[MIX_W_I_T] = {scale_stage(wrow), bidiag_stage(IT, n, !low), scale_stage(g)};
      if (ch == 0) {
        sweeps->meta.assign(size_t(MIX_COUNT) * 2 * 4, 0);
        sweeps->coef.assign(size_t(MIX_COUNT) * 2 * kMaxStages * 4 * kLsPad, 0.0);
      }
      // check each program against its dense matrix on a few fixed vectors
      for (int kind = 0; kind < MIX_COUNT; ++kind) {
        const double* dense = &out[(size_t(kind) * 2 + ch) * n * n];
        bool ok = true;
        for (int trial = 0; trial < 3 && ok; ++trial) {
          std::vector<double> x(n), y(n, 0.0);
          for (int s = 0; s < n; ++s) x[s] = std::sin(1.7 * (s + 1) + 0.9 * trial) + 0.3;
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) y[i] += dense[i * n + j] * x[j];
          std::vector<double> v = x;
          for (const Stage& stg : prog[kind]) apply_stage_host(stg, n, v);
          double num = 0.0, den = 0.0;
          for (int s = 0; s < n; ++s) {
            num += (v[s] - y[s]) * (v[s] - y[s]);
            den += y[s] * y[s];
          }
          ok = std::isfinite(num) && num <= 1e-24 * (den > 0 ? den : 1.0);
        }
        int* meta = &sweeps->meta[(size_t(kind) * 2 + ch) * 4];
        if (!ok) {  // dense fallback
          meta[0] = 1;
          meta[1] = ST_DENSE;
          continue;
        }
        meta[0] = (int)prog[kind].size();
        for (size_t st = 0; st < prog[kind].size(); ++st) {
          const Stage& stg = prog[kind][st];
          meta[1 + st] = stg.type;
          double* cf = &sweeps->coef[((size_t(kind) * 2 + ch) * kMaxStages + st) * 4 * kLsPad];
          for (int s = 0; s < kLsPad; ++s) {
            cf[0 * kLsPad + s] = stg.A[s];
            cf[1 * kLsPad + s] = stg.B[s];
            cf[2 * kLsPad + s] = stg.C[s];
          }
          cf[3 * kLsPad] = stg.W;
        }
      }
    }
  }
  return true;
}

}  // namespace dwa
