// Host-only FP64 pieces of the C ABI: wedges from multipoles (Sec. 2.2, eq. wedge-est with
// eq. Lbar) and the non-uniform mu edges of Sec. 3.1 (eq. nonuniform-bins).
#include <cmath>
#include <vector>

#include "../../include/pkm.h"

namespace pkm_host {

// L_l(x) by the three-term recurrence.
double legendre(int l, double x) {
  if (l == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int n = 1; n < l; ++n) {
    const double p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Mean of L_l over [a, b]: [L_{l+1} - L_{l-1}]_a^b / ((2l+1)(b-a)), and 1 for l = 0.
double lbar(int l, double a, double b) {
  if (l == 0) return 1.0;
  const double fb = legendre(l + 1, b) - legendre(l - 1, b);
  const double fa = legendre(l + 1, a) - legendre(l - 1, a);
  return (fb - fa) / ((2 * l + 1) * (b - a));
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on the recurrence).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
      const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// G(mu) = int_0^mu L_{n}(t)/t dt for odd n (the integrand is a polynomial of degree n-1, so
// a Gauss rule with n/2 + 2 points is exact).
static double g_int(int n, double mu, const std::vector<double>& gx, const std::vector<double>& gw) {
  double s = 0.0;
  for (size_t i = 0; i < gx.size(); ++i) {
    const double t = 0.5 * mu * (gx[i] + 1.0);
    s += gw[i] * legendre(n, t) / t;
  }
  return 0.5 * mu * s;
}

}  // namespace pkm_host

extern "C" pkm_status pkm_wedges(const double* poles, int32_t ell_max, int32_t n_k, const double* mu_edges,
                                 int32_t n_mu_edges, double* wedges_out) {
  if (!poles || !mu_edges || !wedges_out) return PKM_EINVAL;
  if (ell_max < 0 || ell_max % 2 || ell_max > 64 || n_k < 0 || n_mu_edges < 2) return PKM_EINVAL;
  for (int j = 0; j < n_mu_edges; ++j) {
    if (!(mu_edges[j] >= 0.0 && mu_edges[j] <= 1.0)) return PKM_EINVAL;
    if (j > 0 && !(mu_edges[j] > mu_edges[j - 1])) return PKM_EINVAL;
  }
  const int nmu = n_mu_edges - 1;
  const int nl = ell_max / 2 + 1;
  std::vector<double> lb((size_t)nl * nmu);
  for (int il = 0; il < nl; ++il)
    for (int j = 0; j < nmu; ++j) lb[(size_t)il * nmu + j] = pkm_host::lbar(2 * il, mu_edges[j], mu_edges[j + 1]);
  for (int i = 0; i < n_k; ++i)
    for (int j = 0; j < nmu; ++j) {
      double s = 0.0;
      for (int il = 0; il < nl; ++il) s += poles[(size_t)il * n_k + i] * lb[(size_t)il * nmu + j];
      wedges_out[(size_t)i * nmu + j] = s;
    }
  return PKM_OK;
}

extern "C" pkm_status pkm_nonuniform_mu_edges(int32_t ell_max, double* edges_out) {
  if (!edges_out || ell_max < 2 || ell_max % 2 || ell_max > 64) return PKM_EINVAL;
  const int n = ell_max + 1;
  std::vector<double> gx, gw;
  pkm_host::gauss_legendre(n / 2 + 2, gx, gw);
  const double g1 = pkm_host::g_int(n, 1.0, gx, gw);
  auto h = [&](double mu) { return pkm_host::g_int(n, mu, gx, gw) - g1; };
  std::vector<double> roots;
  const int grid = 20000;
  double a = 1e-9, fa = h(a);
  for (int i = 1; i <= grid && (int)roots.size() < ell_max / 2; ++i) {
    const double b = (double)i / grid * (1.0 - 1e-9);
    const double fb = h(b);
    if ((fa < 0) != (fb < 0)) {
      double lo = a, hi = b, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double fm = h(mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      roots.push_back(0.5 * (lo + hi));
    }
    a = b;
    fa = fb;
  }
  if ((int)roots.size() != ell_max / 2) return PKM_EINVAL;
  edges_out[0] = 0.0;
  for (int i = 0; i < ell_max / 2; ++i) edges_out[i + 1] = roots[i];
  edges_out[ell_max / 2 + 1] = 1.0;
  return PKM_OK;
}

extern "C" pkm_status pkm_kaiser_wedge_gamma(int32_t ell_max, const double* mu_edges, int32_t n_mu_edges, double beta,
                                             double* gamma_out) {
  if (!mu_edges || !gamma_out) return PKM_EINVAL;
  if (ell_max < 0 || ell_max % 2 || ell_max > 64 || n_mu_edges < 2 || !std::isfinite(beta)) return PKM_EINVAL;
  for (int j = 0; j < n_mu_edges; ++j) {
    if (!(mu_edges[j] >= 0.0 && mu_edges[j] <= 1.0)) return PKM_EINVAL;
    if (j > 0 && !(mu_edges[j] > mu_edges[j - 1])) return PKM_EINVAL;
  }
  const int nmu = n_mu_edges - 1;
  const int nl = ell_max / 2 + 1;
  // A_ll' = int_{-1}^{1} (dmu/2) L_l L_l' (1 + beta mu^2)^4: a polynomial of degree
  // 2 ell_max + 8, integrated exactly by ell_max + 5 Gauss points
  std::vector<double> gx, gw;
  pkm_host::gauss_legendre(ell_max + 5, gx, gw);
  std::vector<double> a((size_t)nl * nl, 0.0);
  for (size_t q = 0; q < gx.size(); ++q) {
    const double mu = gx[q], s = 1.0 + beta * mu * mu;
    const double k4 = s * s * s * s;
    for (int i = 0; i < nl; ++i) {
      const double li = pkm_host::legendre(2 * i, mu);
      for (int j = 0; j < nl; ++j) a[(size_t)i * nl + j] += 0.5 * gw[q] * li * pkm_host::legendre(2 * j, mu) * k4;
    }
  }
  // (2l+1) Lbar_l(mu_m) per wedge
  std::vector<double> lb((size_t)nl * nmu);
  for (int i = 0; i < nl; ++i)
    for (int m = 0; m < nmu; ++m) lb[(size_t)i * nmu + m] = (4 * i + 1) * pkm_host::lbar(2 * i, mu_edges[m], mu_edges[m + 1]);
  for (int m = 0; m < nmu; ++m)
    for (int n = 0; n < nmu; ++n) {
      double g = 0.0;
      for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j) g += lb[(size_t)i * nmu + m] * lb[(size_t)j * nmu + n] * a[(size_t)i * nl + j];
      gamma_out[(size_t)m * nmu + n] = g;
    }
  return PKM_OK;
}
