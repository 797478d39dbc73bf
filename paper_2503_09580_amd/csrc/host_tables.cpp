// Host-side FP64 precomputation of the plan (Algorithm 1, precomputation):
// the g-quadrature (Sec. 2.3 eq. (13), Jacobi-Gauss-Radau as in Sec. 4.1),
// the radial kernel-mode tables and phi_j = iDFT[s_j] (eq. (24)).
#include "host_tables.h"

#include <cmath>
#include <vector>

namespace lincoll {

namespace {

// Eigenvalues d[] and first eigenvector components z[] of the symmetric
// tridiagonal matrix diag(d) + offdiag(e) (e[i] couples i, i+1; e has n
// entries, the last unused), by implicit QL iteration with Wilkinson-type
// shifts (Bowdler, Martin, Reinsch and Wilkinson, Numer. Math. 1968).
// Only the first row of the accumulated rotations is kept, which is all the
// Golub-Welsch weights need.
bool tridiag_ql(int n, double* d, double* e, double* z) {
  for (int k = 0; k < n; ++k) z[k] = (k == 0) ? 1.0 : 0.0;
  if (n > 0) e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-17 * dd) break;
      }
      if (m == l) break;
      if (++iter > 200) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool underflow = false;
      for (; i >= l; --i) {
        const double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          underflow = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        const double zf = z[i + 1];
        z[i + 1] = s * z[i] + c * zf;
        z[i] = c * z[i] - s * zf;
      }
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

// n-point Gauss-Jacobi rule for (1-x)^a (1+x)^b by Golub-Welsch.
bool gauss_jacobi(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> d(n), e(n), z(n);
  const double mu0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) / std::tgamma(a + b + 2.0);
  for (int k = 0; k < n; ++k) {
    const double s = 2.0 * k + a + b;
    d[k] = (k == 0 && std::fabs(a + b) < 1e-300) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / (s * (s + 2.0));
    if (k + 1 < n) {
      const double kk = k + 1.0, t = 2.0 * kk + a + b;
      const double beta = 4.0 * kk * (kk + a) * (kk + b) * (kk + a + b) / (t * t * (t + 1.0) * (t - 1.0));
      e[k] = std::sqrt(beta);
    }
  }
  if (!tridiag_ql(n, d.data(), e.data(), z.data())) return false;
  // sort ascending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && d[idx[j]] < d[idx[j - 1]]; --j) std::swap(idx[j], idx[j - 1]);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    x[i] = d[idx[i]];
    w[i] = mu0 * z[idx[i]] * z[idx[i]];
  }
  return true;
}

// n-point Gauss-Radau rule for (1+x)^b with the node -1 fixed: the free nodes
// are the (n-1)-point Gauss-Jacobi nodes for (1+x)^(b+1), their weights
// divided by (1 + x_i); the fixed node carries the remaining mass.
bool gauss_jacobi_radau(int n, double b, std::vector<double>& x, std::vector<double>& w) {
  const double mu0 = std::pow(2.0, b + 1.0) / (b + 1.0);
  x.assign(1, -1.0);
  w.assign(1, mu0);
  if (n == 1) return true;
  std::vector<double> xi, wi;
  if (!gauss_jacobi(n - 1, 0.0, b + 1.0, xi, wi)) return false;
  double sum = 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double lam = wi[i] / (1.0 + xi[i]);
    x.push_back(xi[i]);
    w.push_back(lam);
    sum += lam;
  }
  w[0] = mu0 - sum;
  return true;
}

double sinc(double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; }

// cos(2 pi m / n) with exact reduction of the integer argument.
double cos2pi(long long m, int n) {
  m %= n;
  if (m < 0) m += n;
  return std::cos(2.0 * M_PI * (double)m / (double)n);
}

}  // namespace

bool build_tables(const TableParams& tp, HostTables& t) {
  const int n = tp.n, N = n / 2, P = N + 1, Q = 3 * N * N + 1, J = tp.J;
  t.n = n;
  t.J = J;
  t.Q = Q;
  std::vector<double> x, lam;
  double beta;
  if (tp.quad_rule == 0) {
    beta = 4.0 - 2.0 * tp.omega;
  } else {
    beta = 2.0;
  }
  if (!gauss_jacobi_radau(J, beta, x, lam)) return false;
  t.g.resize(J);
  t.W.resize(J);
  for (int j = 0; j < J; ++j) {
    t.g[j] = 0.5 * tp.R * (1.0 + x[j]);
    if (tp.quad_rule == 0) {
      t.W[j] = tp.C * std::pow(0.5 * tp.R, beta + 1.0) * lam[j];
    } else {
      t.W[j] = std::pow(0.5 * tp.R, 3.0) * lam[j] * tp.C * std::pow(t.g[j], 2.0 * (1.0 - tp.omega));
    }
  }
  // radial tables indexed by q = |k|^2
  t.Phi.assign((size_t)J * Q, 0.0);
  t.Omega.assign(Q, 0.0);
  for (int q = 0; q < Q; ++q) {
    const double kk = std::sqrt((double)q);
    double om = 0.0;
    for (int j = 0; j < J; ++j) {
      t.Phi[(size_t)j * Q + q] = 4.0 * M_PI * M_PI * t.W[j] * sinc(M_PI * t.g[j] * kk / (2.0 * tp.L));
      om += t.W[j] * sinc(M_PI * t.g[j] * kk / tp.L);
    }
    t.Omega[q] = 16.0 * M_PI * M_PI * om;
  }
  // phi_j = iDFT[sigma_j] on the octant |d| in [0, N]^3.  sigma_j is s_j with
  // its Nyquist entries doubled (eq. (24) sums over -N..N); folding the
  // even sum over k in -N..N-1 onto |k| gives the weight 1 at k = 0 and 2
  // elsewhere (the doubled -N included).
  std::vector<double> A((size_t)P * P);   // A[d][k]
  for (int d = 0; d < P; ++d)
    for (int k = 0; k < P; ++k) A[(size_t)d * P + k] = (k == 0 ? 1.0 : 2.0) * cos2pi((long long)k * d, n);
  t.phi.assign((size_t)J * P * P * P, 0.0);
  std::vector<double> s((size_t)P * P * P), u1((size_t)P * P * P), u2((size_t)P * P * P);
  const double inv_n3 = 1.0 / ((double)n * n * n);
  for (int j = 0; j < J; ++j) {
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b)
        for (int c = 0; c < P; ++c)
          s[((size_t)a * P + b) * P + c] = sinc(M_PI * t.g[j] * std::sqrt((double)(a * a + b * b + c * c)) / (2.0 * tp.L));
    // transform along the first index, then the second, then the third
    for (int d = 0; d < P; ++d)
      for (int b = 0; b < P; ++b)
        for (int c = 0; c < P; ++c) {
          double acc = 0.0;
          for (int k = 0; k < P; ++k) acc += A[(size_t)d * P + k] * s[((size_t)k * P + b) * P + c];
          u1[((size_t)d * P + b) * P + c] = acc;
        }
    for (int a = 0; a < P; ++a)
      for (int d = 0; d < P; ++d)
        for (int c = 0; c < P; ++c) {
          double acc = 0.0;
          for (int k = 0; k < P; ++k) acc += A[(size_t)d * P + k] * u1[((size_t)a * P + k) * P + c];
          u2[((size_t)a * P + d) * P + c] = acc;
        }
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b)
        for (int d = 0; d < P; ++d) {
          double acc = 0.0;
          for (int k = 0; k < P; ++k) acc += A[(size_t)d * P + k] * u2[((size_t)a * P + b) * P + k];
          t.phi[(size_t)j * P * P * P + ((size_t)a * P + b) * P + d] = acc * inv_n3;
        }
  }
  // K_j = DFT[G phi_j] folded onto the octant: the real-space kernel has no
  // doubled entries, so the weight is 1 at d = 0 and d = N, 2 elsewhere.
  t.Cdct.assign((size_t)P * P, 0.0);   // Cdct[k][d]
  for (int k = 0; k < P; ++k)
    for (int d = 0; d < P; ++d) t.Cdct[(size_t)k * P + d] = ((d == 0 || d == N) ? 1.0 : 2.0) * cos2pi((long long)k * d, n);
  return true;
}

// Hemisphere product rule for the binary operator (Sec. 2.3, eq. (14)): the
// positive nodes mu_i of the n_polar-point Gauss-Legendre rule on [-1, 1]
// (polar cosines) with their weights; combined with n_azimuth equispaced
// azimuths and weights w_i / n_azimuth the rule sums to 1 over S^2_+.
bool hemisphere_polar(int n_polar, std::vector<double>& mu, std::vector<double>& w) {
  std::vector<double> x, wx;
  if (n_polar < 2 || n_polar % 2 || !gauss_jacobi(n_polar, 0.0, 0.0, x, wx)) return false;
  mu.clear();
  w.clear();
  for (int i = 0; i < n_polar; ++i)
    if (x[i] > 0.0) {
      mu.push_back(x[i]);
      w.push_back(wx[i]);
    }
  return (int)mu.size() == n_polar / 2;
}

}  // namespace lincoll
