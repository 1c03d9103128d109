// Site-permutation group closure and real irreps (paper Section 3).
//
// Closure uses Dimino's algorithm: each new generator extends the current
// subgroup H by the right cosets H x reached by right-multiplying coset
// representatives with the generators seen so far.  Elements are then sorted
// lexicographically by permutation image.
//
// Irreps: the eigenspaces of a generic real symmetric element
// S = A + A^T, A = sum_g c_g R(g), of the right regular algebra are invariant
// under the left regular representation; restricted to one eigenspace Q the
// left action rho(g) = Q^T L(g) Q is a real representation that is
// irreducible over the reals.  With <chi, chi> = 1 it is an irrep of real
// type (indicator +1) in real orthogonal form.  With <chi, chi> = 2 and
// indicator 0 it is a conjugate pair Gamma, Gamma* of complex type in real
// form (dimension 2 d_Gamma); it is kept as one real irrep of kind 2, whose
// blocks are the real forms of the complex Gamma blocks (the paper keeps a
// complex-arithmetic path for these; here everything stays real).  With
// <chi, chi> = 4 and indicator -2 it is the realification (dimension 2 d_Gamma)
// of a quaternionic irrep Gamma, kept as one real irrep of kind 4: its real
// commutant is the quaternions, whose non-identity units are antisymmetric,
// so each row again satisfies (dim/|G|) sum_g rho_am rho_am' = delta_mm', and
// its row block is the real form of the Gamma block (trace weight dim / 4).
#include "group.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <string>
#include <unordered_map>
#include <unordered_set>

#include "common.h"

namespace ftlm {

namespace {

using Perm = std::string;  // byte string of images (N <= 64)

Perm compose(const Perm& g, const Perm& h) {  // (g h)[k] = g[h[k]]
  Perm r(h.size(), 0);
  for (size_t k = 0; k < h.size(); ++k) r[k] = g[(unsigned char)h[k]];
  return r;
}

uint64_t splitmix_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

Group build_group(int N, const int32_t* gens, int ngens) {
  if (N <= 0 || N > 64) fail(FTLM_ERR_INVALID_ARG, "N must be in 1..64");
  if (ngens < 0 || (ngens > 0 && !gens)) fail(FTLM_ERR_INVALID_ARG, "bad generator array");
  std::vector<Perm> gen;
  for (int i = 0; i < ngens; ++i) {
    Perm p(N, 0);
    std::vector<char> seen(N, 0);
    for (int k = 0; k < N; ++k) {
      int v = gens[(size_t)i * N + k];
      if (v < 0 || v >= N || seen[v]) fail(FTLM_ERR_NOT_A_PERMUTATION, "generator " + std::to_string(i) + " is not a permutation");
      seen[v] = 1;
      p[k] = (char)v;
    }
    gen.push_back(p);
  }
  Perm e(N, 0);
  for (int k = 0; k < N; ++k) e[k] = (char)k;
  std::vector<Perm> elems{e};
  std::unordered_set<Perm> have{e};
  std::vector<Perm> used;
  const size_t limit = 65535;
  for (const Perm& s : gen) {
    if (have.count(s)) continue;
    std::vector<Perm> H = elems;  // current subgroup
    used.push_back(s);
    std::vector<Perm> reps{s};
    auto add_coset = [&](const Perm& x) {
      for (const Perm& h : H) {
        Perm y = compose(h, x);
        if (have.insert(y).second) elems.push_back(y);
      }
      if (elems.size() > limit) fail(FTLM_ERR_GROUP_TOO_LARGE, "group order exceeds 65535");
    };
    add_coset(s);
    for (size_t i = 0; i < reps.size(); ++i) {
      for (const Perm& t : used) {
        Perm x = compose(reps[i], t);
        if (!have.count(x)) {
          reps.push_back(x);
          add_coset(x);
        }
      }
    }
  }
  std::sort(elems.begin(), elems.end(), [](const Perm& a, const Perm& b) {
    for (size_t k = 0; k < a.size(); ++k)
      if (a[k] != b[k]) return (unsigned char)a[k] < (unsigned char)b[k];
    return false;
  });
  Group G;
  G.N = N;
  G.order = (int)elems.size();
  const int n = G.order;
  std::unordered_map<Perm, int> index;
  index.reserve(n * 2);
  for (int i = 0; i < n; ++i) index[elems[i]] = i;
  G.perms.resize((size_t)n * N);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < N; ++k) G.perms[(size_t)i * N + k] = (unsigned char)elems[i][k];
  for (const Perm& g : gen) G.gen_idx.push_back(index.at(g));
  G.mul.resize((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) G.mul[(size_t)a * n + b] = (uint16_t)index.at(compose(elems[a], elems[b]));
  G.inv.resize(n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (G.mul[(size_t)a * n + b] == 0) { G.inv[a] = (uint16_t)b; break; }
  G.elem_order.resize(n);
  for (int a = 0; a < n; ++a) {
    int k = 1, x = a;
    while (x != 0) { x = G.idx_mul(x, a); ++k; }
    G.elem_order[a] = k;
  }
  // conjugacy classes, canonical order (element order, size, smallest member)
  std::vector<int> cls(n, -1);
  std::vector<std::vector<int32_t>> raw;
  for (int a = 0; a < n; ++a) {
    if (cls[a] >= 0) continue;
    std::vector<int32_t> mem;
    for (int x = 0; x < n; ++x) mem.push_back(G.idx_mul(G.idx_mul(x, a), G.inv[x]));
    std::sort(mem.begin(), mem.end());
    mem.erase(std::unique(mem.begin(), mem.end()), mem.end());
    for (int m : mem) cls[m] = (int)raw.size();
    raw.push_back(mem);
  }
  std::vector<int> ord(raw.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) {
    auto kx = std::make_tuple(G.elem_order[raw[x][0]], raw[x].size(), raw[x][0]);
    auto ky = std::make_tuple(G.elem_order[raw[y][0]], raw[y].size(), raw[y][0]);
    return kx < ky;
  });
  G.class_of.assign(n, 0);
  for (size_t ci = 0; ci < ord.size(); ++ci) {
    G.classes.push_back(raw[ord[ci]]);
    for (int m : raw[ord[ci]]) G.class_of[m] = (int)ci;
  }
  return G;
}

// Symmetric eigenproblem A = V diag(w) V^T (w ascending, eigenvectors in the
// columns of V; A is overwritten): Householder reduction to tridiagonal form
// with the reflections accumulated into V, then implicit QL iterations with
// Wilkinson-type shifts whose rotations are applied to the rows of V
// (Golub and Van Loan, Matrix Computations, Sections 8.3.1 and 8.3.3).
std::vector<double> sym_eigh(std::vector<double>& A, int n, std::vector<double>& V) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    // reflection H = I - beta u u^T on rows / columns k+1..n-1 zeroing a(k+2.., k)
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += a(i, k) * a(i, k);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double al = a(k + 1, k) > 0 ? -xn : xn;
    for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
    v[k + 1] -= al;
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // p = beta A v, q = p - (beta v^T p / 2) v, A -= v q^T + q v^T
    double vp = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
      p[i] = beta * s;
      vp += v[i] * p[i];
    }
    const double K = 0.5 * beta * vp;
    for (int i = k + 1; i < n; ++i) q[i] = p[i] - K * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) a(i, j) -= v[i] * q[j] + q[i] * v[j];
    a(k + 1, k) = a(k, k + 1) = al;
    for (int i = k + 2; i < n; ++i) a(i, k) = a(k, i) = 0.0;
    // V <- V H
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += V[(size_t)r * n + j] * v[j];
      s *= beta;
      for (int j = k + 1; j < n; ++j) V[(size_t)r * n + j] -= s * v[j];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m)
        if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
      if (m == l) break;
      if (iter > 200) fail(FTLM_ERR_IRREPS_FAILED, "symmetric QL did not converge");
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::sqrt(g * g + 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::sqrt(f * f + g * g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          double* row = &V[(size_t)k * n];
          const double x1 = row[i + 1];
          row[i + 1] = s * row[i] + c * x1;
          row[i] = c * row[i] - s * x1;
        }
      }
      if (split) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  std::vector<double> ws(n), Vs((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    ws[j] = d[idx[j]];
    for (int i = 0; i < n; ++i) Vs[(size_t)i * n + j] = V[(size_t)i * n + idx[j]];
  }
  V.swap(Vs);
  return ws;
}

double verify_irreps(const Group& G, const std::vector<const Irrep*>& irs) {
  const int n = G.order;
  // homomorphism and orthogonality, one group element a per task (the
  // largest residual does not depend on the split)
  std::vector<double> worst_a(n, 0.0);
  parallel_for(n, 8, [&](int64_t a) {
    double worst = 0.0;
    for (const Irrep* ir : irs) {
      const int d = ir->dim;
      const double* r = ir->rho.data();
      // orthogonality rho(a)^T rho(a) = 1
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          double s = 0;
          for (int k = 0; k < d; ++k) s += r[((size_t)a * d + k) * d + i] * r[((size_t)a * d + k) * d + j];
          worst = std::max(worst, std::fabs(s - (i == j ? 1.0 : 0.0)));
        }
      for (int b = 0; b < n; ++b) {
        const double* ab = r + (size_t)G.idx_mul((int)a, b) * d * d;
        for (int i = 0; i < d; ++i)
          for (int j = 0; j < d; ++j) {
            double s = 0;
            for (int k = 0; k < d; ++k) s += r[((size_t)a * d + i) * d + k] * r[((size_t)b * d + k) * d + j];
            worst = std::max(worst, std::fabs(s - ab[i * d + j]));
          }
      }
    }
    worst_a[a] = worst;
  });
  double worst = 0.0;
  for (double w : worst_a) worst = std::max(worst, w);
  // great orthogonality (d_A/|G|) sum_g rho_A(g)_ij rho_B(g)_kl = delta_AB delta_ik delta_jl
  for (size_t x = 0; x < irs.size(); ++x)
    for (size_t y = x; y < irs.size(); ++y) {
      const Irrep& A = *irs[x];
      const Irrep& B = *irs[y];
      for (int i = 0; i < A.dim; ++i)
        for (int j = 0; j < A.dim; ++j)
          for (int k = 0; k < B.dim; ++k)
            for (int l = 0; l < B.dim; ++l) {
              // a realified irrep (kind 2 or 4) satisfies the relation within
              // one row (i == k), which is what the block construction uses
              if (x == y && A.kind >= 2 && i != k) continue;
              double s = 0;
              for (int g = 0; g < n; ++g)
                s += A.rho[((size_t)g * A.dim + i) * A.dim + j] * B.rho[((size_t)g * B.dim + k) * B.dim + l];
              s *= double(A.dim) / n;
              double ref = (x == y && i == k && j == l) ? 1.0 : 0.0;
              worst = std::max(worst, std::fabs(s - ref));
            }
    }
  return worst;
}

void compute_irreps(Group& G) {
  const int n = G.order;
  G.irreps_computed = false;
  G.irreps.clear();
  if (n > 1024) return;
  const int nclass = (int)G.classes.size();
  std::vector<int> rep_of_class(nclass);
  for (int c = 0; c < nclass; ++c) rep_of_class[c] = G.classes[c][0];

  for (int attempt = 0; attempt < 4; ++attempt) {
    uint64_t st = 0x1234ABCDull + 7919ull * attempt;
    std::vector<double> c(n);
    for (int g = 0; g < n; ++g) c[g] = (double)(splitmix_next(st) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    std::vector<double> S((size_t)n * n);
    for (int x = 0; x < n; ++x)
      for (int y = 0; y < n; ++y)
        S[(size_t)x * n + y] = c[G.idx_mul(G.inv[x], y)] + c[G.idx_mul(G.inv[y], x)];
    std::vector<double> Q;
    std::vector<double> w = sym_eigh(S, n, Q);
    double spread = w.back() - w.front();
    double tol = 1e-7 * std::max(1.0, spread);
    std::vector<std::pair<int, int>> clusters;
    int start = 0;
    for (int i = 1; i <= n; ++i)
      if (i == n || w[i] - w[i - 1] > tol) { clusters.push_back({start, i}); start = i; }

    bool complete = true;
    std::map<std::vector<long long>, Irrep> found;
    std::vector<double> chi(n);
    for (auto [a, b] : clusters) {
      const int m = b - a;
      // chi(g) = sum_i sum_x Q[x][a+i] Q[g^-1 x][a+i]
      for (int g = 0; g < n; ++g) {
        int gi = G.inv[g];
        double s = 0;
        for (int x = 0; x < n; ++x) {
          const double* qx = &Q[(size_t)x * n + a];
          const double* qy = &Q[(size_t)G.idx_mul(gi, x) * n + a];
          for (int i = 0; i < m; ++i) s += qx[i] * qy[i];
        }
        chi[g] = s;
      }
      double nrm = 0;
      for (int g = 0; g < n; ++g) nrm += chi[g] * chi[g];
      double nu = 0;
      for (int g = 0; g < n; ++g) nu += chi[G.idx_mul(g, g)];
      nu /= n;
      // <chi, chi> = 1: real type; 2 with indicator 0: a complex pair; 4 with
      // indicator -2: a realified quaternionic irrep (both irreducible over
      // the reals); anything else (a degenerate split) is left out
      int kind = 0;
      if (std::fabs(nrm / n - 1.0) < 1e-6 && std::fabs(nu - 1.0) < 1e-6) kind = 1;
      if (std::fabs(nrm / n - 2.0) < 1e-6 && std::fabs(nu) < 1e-6 && m % 2 == 0) kind = 2;
      if (std::fabs(nrm / n - 4.0) < 1e-6 && std::fabs(nu + 2.0) < 1e-6 && m % 4 == 0) kind = 4;
      if (!kind) { complete = false; continue; }
      std::vector<long long> key(nclass);
      for (int cc = 0; cc < nclass; ++cc) key[cc] = std::llround(chi[rep_of_class[cc]] * 1e6);
      if (found.count(key)) continue;
      Irrep ir;
      ir.dim = m;
      ir.kind = kind;
      ir.rho.assign((size_t)n * m * m, 0.0);
      for (int g = 0; g < n; ++g) {
        int gi = G.inv[g];
        double* rg = &ir.rho[(size_t)g * m * m];
        for (int x = 0; x < n; ++x) {
          const double* qx = &Q[(size_t)x * n + a];
          const double* qy = &Q[(size_t)G.idx_mul(gi, x) * n + a];
          for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) rg[i * m + j] += qx[i] * qy[j];
        }
      }
      ir.chars.resize(nclass);
      for (int cc = 0; cc < nclass; ++cc) ir.chars[cc] = chi[rep_of_class[cc]];
      // reported: the Frobenius-Schur indicator of the complex irrep (+1, 0, -1)
      ir.indicator = kind == 4 ? -1 : (int)std::lround(nu);
      found.emplace(key, std::move(ir));
    }
    std::vector<Irrep> irs;
    for (auto& kv : found) irs.push_back(std::move(kv.second));
    std::sort(irs.begin(), irs.end(), [&](const Irrep& x, const Irrep& y) {
      if (x.dim != y.dim) return x.dim < y.dim;
      for (int cc = 0; cc < nclass; ++cc) {
        long long a = std::llround(x.chars[cc] * 1e9), b = std::llround(y.chars[cc] * 1e9);
        if (a != b) return a > b;
      }
      return false;
    });
    // sum over complex irreps of d^2: a realified pair holds two of dimension
    // dim / 2, a realified quaternionic irrep one of dimension dim / 2
    int sumsq = 0;
    for (auto& ir : irs) sumsq += ir.dim * ir.weight();
    std::vector<const Irrep*> ptrs;
    for (auto& ir : irs) ptrs.push_back(&ir);
    double res = verify_irreps(G, ptrs);
    if (res > 1e-9) continue;  // retry with another random element
    if (complete && sumsq != n) continue;
    G.irreps = std::move(irs);
    G.all_real = complete && sumsq == n;
    G.max_residual = res;
    G.irreps_computed = true;
    return;
  }
  fail(FTLM_ERR_IRREPS_FAILED, "irrep construction did not pass verification");
}

}  // namespace ftlm

namespace ftlm {

namespace {

// Subgroup generated by the given elements (closure under right
// multiplication by the generators), as a membership mask.
std::vector<char> generated(const Group& G, const std::vector<int>& gens) {
  std::vector<char> in(G.order, 0);
  std::vector<int> list{0};
  in[0] = 1;
  for (size_t i = 0; i < list.size(); ++i)
    for (int s : gens) {
      const int y = G.idx_mul(list[i], s);
      if (!in[y]) {
        in[y] = 1;
        list.push_back(y);
      }
    }
  return in;
}

}  // namespace

namespace {
Factorization factor_group_uncached(const Group& G, int max_plain);
}

Factorization factor_group(const Group& G, int max_plain) {
  std::lock_guard<std::mutex> lk(G.fac_mu);
  auto it = G.fac_cache.find(max_plain);
  if (it == G.fac_cache.end())
    it = G.fac_cache.emplace(max_plain, std::make_shared<const Factorization>(factor_group_uncached(G, max_plain))).first;
  return *it->second;
}

namespace {
Factorization factor_group_uncached(const Group& G, int max_plain) {
  const int n = G.order;
  std::vector<char> best;
  int best_h = 1;
  if (n > max_plain) {
    long best_cost = (long)n + 1;
    auto consider = [&](const std::vector<int>& gens) {
      std::vector<char> in = generated(G, gens);
      int h = 0;
      for (char c : in) h += c;
      const long cost = (long)h + n / h;
      if (cost < best_cost || (cost == best_cost && h < best_h)) {
        best_cost = cost;
        best_h = h;
        best = std::move(in);
      }
    };
    const int ng = std::min<int>((int)G.gen_idx.size(), 10);
    for (int m = 1; m < (1 << ng); ++m) {
      std::vector<int> gs;
      for (int k = 0; k < ng; ++k)
        if ((m >> k) & 1) gs.push_back(G.gen_idx[k]);
      consider(gs);
    }
    for (int g = 1; g < n; ++g) consider({g});
    std::vector<int> reps;
    for (const auto& c : G.classes) reps.push_back(c[0]);
    if (reps.size() > 64) reps.clear();  // pairs only while they stay cheap
    for (size_t i = 0; i < reps.size(); ++i)
      for (size_t j = i + 1; j < reps.size(); ++j) consider({reps[i], reps[j]});
  }
  Factorization f;
  if (best.empty()) {
    best.assign(n, 0);
    best[0] = 1;
    best_h = 1;
  }
  for (int g = 0; g < n; ++g)
    if (best[g]) f.H.push_back(g);  // ascending, so H[0] = identity
  // left cosets t H, each represented by its smallest element
  std::vector<char> covered(n, 0);
  for (int g = 0; g < n; ++g) {
    if (covered[g]) continue;
    f.T.push_back(g);
    for (int h : f.H) covered[G.idx_mul(g, h)] = 1;
  }
  const int nH = (int)f.H.size(), nT = (int)f.T.size();
  if ((long)nH * nT != n) fail(FTLM_ERR_INVALID_ARG, "internal: coset decomposition does not cover the group");
  f.gidx.resize((size_t)nT * nH);
  for (int t = 0; t < nT; ++t)
    for (int h = 0; h < nH; ++h) f.gidx[(size_t)t * nH + h] = (uint16_t)G.idx_mul(f.T[t], f.H[h]);
  return f;
}
}  // namespace

}  // namespace ftlm
