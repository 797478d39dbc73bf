// Driver for the host-sanitizer test (tests/test_host_sanitizers.py): builds
// the plan tables of every supported size and both quadrature rules, small
// and large node counts, and every hemisphere rule, with the host code
// compiled under AddressSanitizer and UndefinedBehaviorSanitizer.  Checks a
// few invariants so that the calls are not optimised away; exits non-zero on
// a failed check (the sanitizers abort on their own findings).
#include <cmath>
#include <cstdio>
#include <vector>

#include "../paper_2503_09580_amd/csrc/host_tables.h"

using namespace lincoll;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

int main() {
  const int ns[] = {8, 16, 32, 64};
  const double omegas[] = {0.5, 0.74, 1.0};
  for (int n : ns)
    for (double om : omegas)
      for (int rule = 0; rule <= 1; ++rule)
        for (int J : {1, 3, n / 2 + 1, 2 * n}) {
          TableParams tp{n, 8.0, om, 1.0 / (4.0 * M_PI), 4.0 * 8.0 / (3.0 + std::sqrt(2.0)), J, rule};
          HostTables t;
          CHECK(build_tables(tp, t));
          const int P = n / 2 + 1, Q = 3 * (n / 2) * (n / 2) + 1;
          CHECK(t.J == J && t.Q == Q);
          CHECK((int)t.g.size() == J && (int)t.W.size() == J);
          CHECK((int)t.Phi.size() == J * Q && (int)t.Omega.size() == Q);
          CHECK((int)t.phi.size() == J * P * P * P && (int)t.Cdct.size() == P * P);
          double ws = 0.0;
          for (int j = 0; j < J; ++j) {
            // rule 1 multiplies B(g_j) in, which is 0 at the fixed node g = 0
            CHECK(std::isfinite(t.g[j]) && std::isfinite(t.W[j]) && t.W[j] >= 0.0);
            ws += t.W[j];
          }
          CHECK(ws > 0.0 || (rule == 1 && J == 1));
          for (double v : t.Phi) CHECK(std::isfinite(v));
          for (double v : t.Omega) CHECK(std::isfinite(v));
          for (double v : t.phi) CHECK(std::isfinite(v));
        }
  for (int np = 2; np <= 64; np += 2) {
    std::vector<double> mu, w;
    CHECK(hemisphere_polar(np, mu, w));
    CHECK((int)mu.size() == np / 2 && (int)w.size() == np / 2);
    double s = 0.0;
    for (int i = 0; i < np / 2; ++i) {
      CHECK(mu[i] > 0.0 && mu[i] < 1.0);
      s += w[i];
    }
    CHECK(std::fabs(s - 1.0) < 1e-12);   // positive half of a rule of total weight 2
  }
  std::vector<double> mu, w;
  CHECK(!hemisphere_polar(3, mu, w));     // odd orders are rejected
  std::printf("host tables: %s\n", fails ? "FAILED" : "ok");
  return fails ? 1 : 0;
}
