// Host FP64 stages of the FTLM estimator (paper Section 2.2, Eqs. 4-7, 14):
// Ritz data of each chain's tridiagonal matrix and the thermal sums.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

namespace ftlm {

// Eigenvalues and squared first eigenvector components of a symmetric
// tridiagonal matrix by the implicit QL method with Wilkinson-type shifts.
// Only the first row of the accumulated rotation product is tracked, which is
// all the FTLM weights need.  d: diagonal (n), e: off-diagonal (n-1).
namespace {
// sqrt(a^2 + b^2); the scaled std::hypot only where the squares could
// overflow or underflow
inline double pyth(double a, double b) {
  const double m = std::max(std::fabs(a), std::fabs(b));
  if (m > 1e150 || (m < 1e-150 && m > 0.0)) return std::hypot(a, b);
  return std::sqrt(a * a + b * b);
}
}  // namespace

void tridiag_ritz(const double* alpha, const double* beta, int n, double* theta, double* weight) {
  std::vector<double> d(alpha, alpha + n), e(n, 0.0), z(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) e[i] = beta[i];
  if (n > 0) z[0] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (iter > 200) fail(FTLM_ERR_INVALID_ARG, "tridiagonal QL did not converge");
      // shift from the leading 2x2 block at l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = pyth(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        double f = s * e[i];
        double b = c * e[i];
        r = pyth(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // underflow: split the problem here
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double zi1 = z[i + 1];
        z[i + 1] = s * z[i] + c * zi1;
        z[i] = c * z[i] - s * zi1;
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int k = 0; k < n; ++k) {
    theta[k] = d[idx[k]];
    weight[k] = z[idx[k]] * z[idx[k]];
  }
}

void observables(const ftlm_ritz* blocks, int nb, const double* T, int nT, double g, double* E,
                 double* C, double* chi, double* logZ) {
  double E0 = std::numeric_limits<double>::infinity();
  for (int b = 0; b < nb; ++b) {
    const ftlm_ritz& B = blocks[b];
    if (B.D == 0) continue;
    for (int r = 0; r < B.R; ++r)
      for (int k = 0; k < B.nsteps[r]; ++k) E0 = std::min(E0, B.theta[(size_t)r * B.ld + k]);
  }
  if (!std::isfinite(E0)) fail(FTLM_ERR_INVALID_ARG, "no Ritz values in the given blocks");
  // temperatures are independent: one thread per range of them
  parallel_for(nT, 4, [&](int64_t t) {
    const double beta = 1.0 / T[t];
    double Z = 0, H1 = 0, H2 = 0, num = 0, den = 0;
    for (int b = 0; b < nb; ++b) {
      const ftlm_ritz& B = blocks[b];
      if (B.D == 0 || B.R == 0) continue;
      const double mult = B.two_M == 0 ? 1.0 : 2.0;
      double z = 0, h1 = 0, h2 = 0;
      for (int r = 0; r < B.R; ++r)
        for (int k = 0; k < B.nsteps[r]; ++k) {
          double sh = B.theta[(size_t)r * B.ld + k] - E0;
          double bz = std::exp(-beta * sh) * B.weight[(size_t)r * B.ld + k];
          z += bz;
          h1 += bz * sh;
          h2 += bz * sh * sh;
        }
      const double zblock = double(B.d_gamma) * double(B.D) / double(B.R) * z;  // d_Gamma Z_{M,Gamma}
      Z += mult * zblock;
      const double fac = mult * double(B.d_gamma) * double(B.D) / double(B.R);
      H1 += fac * h1;
      H2 += fac * h2;
      const double M = 0.5 * B.two_M;
      num += mult * M * M * zblock;
      den += mult * zblock;
    }
    const double e1 = H1 / Z, e2 = H2 / Z;
    if (E) E[t] = E0 + e1;
    if (C) C[t] = beta * beta * (e2 - e1 * e1);
    if (chi) chi[t] = g * g * beta * num / den;
    if (logZ) logZ[t] = std::log(Z) - beta * E0;
  });
}

// KPM thermal sums (see ftlm.h): Jackson-damped chain-averaged moments ->
// Gauss-Chebyshev node weights per block -> shifted Boltzmann sums.
void kpm_observables(const ftlm_kpm_block* blocks, int nb, const double* T, int nT, double g, int n_nodes, double* E,
                     double* C, double* chi, double* logZ) {
  struct Nodes {
    double fac, M2;  // mult * d_Gamma * D, M^2
    std::vector<double> e, w;
  };
  std::vector<Nodes> all;
  int maxM = 0;
  for (int b = 0; b < nb; ++b) maxM = std::max(maxM, blocks[b].n_moments);
  const int K = n_nodes > 0 ? n_nodes : 2 * maxM;
  if (K <= 0) fail(FTLM_ERR_INVALID_ARG, "no moments");
  double E0 = std::numeric_limits<double>::infinity();
  for (int b = 0; b < nb; ++b) {
    const ftlm_kpm_block& B = blocks[b];
    if (B.D == 0 || B.R <= 0 || B.n_moments <= 0) continue;
    if (!B.moments || !(B.half_width > 0)) fail(FTLM_ERR_INVALID_ARG, "bad KPM block");
    const int M = B.n_moments;
    std::vector<double> c(M, 0.0);
    for (int r = 0; r < B.R; ++r)
      for (int n = 0; n < M; ++n) c[n] += B.moments[(size_t)r * M + n];
    const double pq = M_PI / (M + 1);
    for (int n = 0; n < M; ++n) {
      const double gj = ((M - n + 1) * std::cos(pq * n) + std::sin(pq * n) / std::tan(pq)) / (M + 1);
      c[n] *= gj / B.R;  // Jackson kernel times the chain average
    }
    Nodes nd;
    nd.fac = (B.two_M == 0 ? 1.0 : 2.0) * (double)B.d_gamma * (double)B.D;
    nd.M2 = 0.25 * B.two_M * B.two_M;
    nd.e.resize(K);
    nd.w.resize(K);
    for (int k = 0; k < K; ++k) {
      const double th = M_PI * (k + 0.5) / K;
      double s = c[0];
      for (int n = 1; n < M; ++n) s += 2.0 * c[n] * std::cos(n * th);
      nd.w[k] = s / K;
      nd.e[k] = B.center + B.half_width * std::cos(th);
      E0 = std::min(E0, nd.e[k]);
    }
    all.push_back(std::move(nd));
  }
  if (all.empty()) fail(FTLM_ERR_INVALID_ARG, "no moments in the given blocks");
  parallel_for(nT, 4, [&](int64_t t) {
    const double beta = 1.0 / T[t];
    double Z = 0, H1 = 0, H2 = 0, num = 0;
    for (const Nodes& nd : all) {
      double z = 0, h1 = 0, h2 = 0;
      for (size_t k = 0; k < nd.e.size(); ++k) {
        const double sh = nd.e[k] - E0;
        const double bz = std::exp(-beta * sh) * nd.w[k];
        z += bz;
        h1 += bz * sh;
        h2 += bz * sh * sh;
      }
      Z += nd.fac * z;
      H1 += nd.fac * h1;
      H2 += nd.fac * h2;
      num += nd.fac * nd.M2 * z;
    }
    const double e1 = H1 / Z, e2 = H2 / Z;
    if (E) E[t] = E0 + e1;
    if (C) C[t] = beta * beta * (e2 - e1 * e1);
    if (chi) chi[t] = g * g * beta * num / Z;
    if (logZ) logZ[t] = std::log(Z) - beta * E0;
  });
}

}  // namespace ftlm
