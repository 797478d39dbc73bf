// The in-register FFT building blocks of csrc/fft.h, compiled for the host,
// against the DFT's definition X[k] = sum_j x[j] exp(-+ 2 pi i j k / N)
// summed in long double: every transform (fft: decimation in time up to 32
// points and radix-4 decimation in frequency at 64; fft_dit and fft_r4 at
// every size), forward and inverse, in float and double, and the real-pair
// packing (split_real_pair with its scale arguments, join_real_pair).
// Bound: 2 log2(N) unit roundoffs of the largest output.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "fft.h"

using namespace lincoll;
using cld = std::complex<long double>;

static int failures = 0;

template <typename T>
static double eps() { return std::is_same<T, float>::value ? 0x1p-24 : 0x1p-53; }

static void direct(const cld* x, cld* X, int n, bool inv) {
  const long double pi = acosl(-1.0L);
  for (int k = 0; k < n; ++k) {
    X[k] = 0;
    for (int j = 0; j < n; ++j) {
      const long double a = (inv ? 2 : -2) * pi * ((long)j * k % n) / n;
      X[k] += x[j] * cld(cosl(a), sinl(a));
    }
  }
}

static void report(const char* what, int n, const char* type, bool inv, double err, double bound) {
  const bool ok = err <= bound;
  if (!ok) ++failures;
  printf("%-16s N=%2d %-6s %s  rel err %.2e  bound %.2e  %s\n", what, n, type, inv ? "inv" : "fwd", err, bound,
         ok ? "ok" : "FAIL");
}

// which: 0 fft, 1 fft_dit, 2 fft_r4
template <int N, bool INV, typename T>
static void check_transform(int which, std::mt19937& g) {
  std::normal_distribution<double> nd;
  T re[N], im[N];
  cld x[N], X[N];
  for (int i = 0; i < N; ++i) {
    re[i] = T(nd(g));
    im[i] = T(nd(g));
    x[i] = cld(re[i], im[i]);
  }
  if (which == 0) fft<N, INV>(re, im);
  else if (which == 1) fft_dit<N, INV>(re, im);
  else fft_r4<N, INV>(re, im);
  direct(x, X, N, INV);
  double err = 0, mx = 0;
  for (int k = 0; k < N; ++k) {
    err = std::fmax(err, double(std::abs(X[k] - cld(re[k], im[k]))));
    mx = std::fmax(mx, double(std::abs(X[k])));
  }
  static const char* names[] = {"fft", "fft_dit", "fft_r4"};
  report(names[which], N, std::is_same<T, float>::value ? "float" : "double", INV, err / mx,
         2 * ilog2(N) * eps<T>());
}

// Two real sequences a, b as z = a + i b: forward, split into A, B (scaled by
// 2 ha and 2 hb), then join and inverse back to N (a + i b).
template <int N, typename T>
static void check_real_pair(std::mt19937& g) {
  std::normal_distribution<double> nd;
  T zr[N], zi[N];
  cld a[N], b[N], A[N], B[N];
  for (int i = 0; i < N; ++i) {
    zr[i] = T(nd(g));
    zi[i] = T(nd(g));
    a[i] = zr[i];
    b[i] = zi[i];
  }
  direct(a, A, N, false);
  direct(b, B, N, false);
  const T ha = T(0.375), hb = T(-1.25);   // exact in binary: scales 0.75 and -2.5
  fft<N, false>(zr, zi);
  T Ar[N / 2 + 1], Ai[N / 2 + 1], Br[N / 2 + 1], Bi[N / 2 + 1];
  split_real_pair<N>(zr, zi, Ar, Ai, Br, Bi, ha, hb);
  double err = 0, mx = 0;
  for (int k = 0; k <= N / 2; ++k) {
    err = std::fmax(err, double(std::abs(A[k] * (long double)(2 * ha) - cld(Ar[k], Ai[k]))));
    err = std::fmax(err, double(std::abs(B[k] * (long double)(2 * hb) - cld(Br[k], Bi[k]))));
    mx = std::fmax(mx, double(std::abs(A[k] * (long double)(2 * ha))));
    mx = std::fmax(mx, double(std::abs(B[k] * (long double)(2 * hb))));
  }
  const char* type = std::is_same<T, float>::value ? "float" : "double";
  report("split_real_pair", N, type, false, err / mx, (2 * ilog2(N) + 2) * eps<T>());
  // join the unscaled spectra and transform back
  for (int k = 0; k <= N / 2; ++k) {
    Ar[k] = T(A[k].real()), Ai[k] = T(A[k].imag()), Br[k] = T(B[k].real()), Bi[k] = T(B[k].imag());
  }
  T wr[N], wi[N];
  join_real_pair<N>(Ar, Ai, Br, Bi, wr, wi);
  fft<N, true>(wr, wi);
  err = 0, mx = 0;
  for (int i = 0; i < N; ++i) {
    const cld want = cld(a[i].real() * N, b[i].real() * N);
    err = std::fmax(err, double(std::abs(want - cld(wr[i], wi[i]))));
    mx = std::fmax(mx, double(std::abs(want)));
  }
  report("join_real_pair", N, type, true, err / mx, (2 * ilog2(N) + 2) * eps<T>());
}

template <int N>
static void run(std::mt19937& g) {
  for (int which = 0; which < 3; ++which) {
    check_transform<N, false, float>(which, g);
    check_transform<N, true, float>(which, g);
    check_transform<N, false, double>(which, g);
    check_transform<N, true, double>(which, g);
  }
  if constexpr (N >= 4) {
    check_real_pair<N, float>(g);
    check_real_pair<N, double>(g);
  }
}

int main() {
  std::mt19937 g(20250312);
  run<2>(g);
  run<4>(g);
  run<8>(g);
  run<16>(g);
  run<32>(g);
  run<64>(g);
  printf(failures ? "fft host check: %d FAILED\n" : "fft host check: ok\n", failures);
  return failures ? 1 : 0;
}
