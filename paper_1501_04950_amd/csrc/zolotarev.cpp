// Zolotarev coefficients for the per-slice Moebius coefficients (Sec. 3: the Zolotarev
// row of the table and the ordering of the coefficients; App. A, eq.(polar)).  Host code.
//
// With b_i = c_i = omega_i the kernel of eq.(argument) is omega_i gamma_5 D_w, and eq.(polar)
// approximates sign(H), H = gamma_5 D_w, by (1 - r(H)) / (1 + r(H)) with
// r(x) = prod_i (1 - omega_i x) / (1 + omega_i x).  The omega_i that minimise max |r| over the
// spectrum [lmin, lmax] of |H| (Zolotarev's third problem) are
//     1 / omega_j = lmax dn((2j - 1) K(k') / (2 Ls), k'),  k' = sqrt(1 - (lmin / lmax)^2),
// with dn and K computed here by the arithmetic-geometric mean (the descending Landen
// sequence): a_0 = 1, b_0 = k (the complementary modulus, passed directly so that nothing
// cancels when k is small), a_n = (a + b)/2, b_n = sqrt(a b), c_n = (a - b)/2 until c_N
// vanishes; K = pi / (2 a_N); phi_N = 2^N a_N u, phi_{n-1} = (phi_n + asin(c_n sin phi_n / a_n))/2;
// dn = cos phi_0 / cos(phi_1 - phi_0).
#include <algorithm>
#include <cmath>
#include <vector>

#include "dwa_internal.h"

namespace {

struct Agm {
  std::vector<double> a, c;  // a_0 .. a_N, c_0 .. c_N (c_0 unused)
};

Agm agm(double kc) {
  Agm g;
  double a = 1.0, b = kc;
  g.a.push_back(a);
  g.c.push_back(0.0);
  for (int n = 0; n < 64; ++n) {
    const double an = 0.5 * (a + b), bn = std::sqrt(a * b), cn = 0.5 * (a - b);
    g.a.push_back(an);
    g.c.push_back(cn);
    a = an;
    b = bn;
    if (std::fabs(cn) <= 1e-17 * an) break;
  }
  return g;
}

// dn(u, k') for the modulus whose complement is kc, from the AGM sequence g of kc
double dn_from(const Agm& g, double u) {
  const int N = int(g.a.size()) - 1;
  double phi = std::ldexp(g.a[N] * u, N);
  double phi_next = phi;
  for (int n = N; n >= 1; --n) {
    phi_next = phi;
    phi = 0.5 * (phi + std::asin(g.c[n] * std::sin(phi) / g.a[n]));
  }
  return std::cos(phi) / std::cos(phi_next - phi);
}

double ratio_abs(double x, const double* om, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= (1.0 - om[i] * x) / (1.0 + om[i] * x);
  return std::fabs(r);
}

}  // namespace

extern "C" int dwa_zolotarev(double lmin, double lmax, int Ls, int ordering, double* omega,
                             double* delta) {
  if (!omega || Ls < 1 || Ls > 32 || !(lmin > 0.0) || !(lmax > lmin) || !std::isfinite(lmax) ||
      ordering < 0 || ordering > 2) {
    dwa::set_error("dwa_zolotarev: need 0 < lmin < lmax finite, 1 <= Ls <= 32, ordering 0..2, omega");
    return DWA_EINVAL;
  }
  const double k = lmin / lmax;
  const Agm g = agm(k);
  const double K = M_PI / (2.0 * g.a.back());
  std::vector<double> om(Ls);
  for (int j = 1; j <= Ls; ++j) om[j - 1] = 1.0 / (lmax * dn_from(g, (2 * j - 1) * K / (2.0 * Ls)));
  std::sort(om.begin(), om.end());
  if (ordering == 0) {
    std::copy(om.begin(), om.end(), omega);
  } else if (ordering == 2) {
    std::copy(om.rbegin(), om.rend(), omega);
  } else {  // concave: from both walls inwards, alternately front and back
    int lo = 0, hi = Ls - 1;
    for (int i = 0; i < Ls; ++i) omega[(i % 2 == 0) ? lo++ : hi--] = om[i];
  }
  if (delta) {
    double d = 0.0;
    const int n = 20001;
    for (int i = 0; i < n; ++i) {
      const double x = lmin * std::pow(lmax / lmin, double(i) / (n - 1));
      d = std::max(d, ratio_abs(x, om.data(), Ls));
    }
    *delta = d;
  }
  return DWA_OK;
}
