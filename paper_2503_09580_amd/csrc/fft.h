// In-register FFT building blocks for gfx950 (one thread owns a whole
// length-N complex sequence; N a power of two <= 64).  Every index is a
// compile-time constant after expansion, so the sequence stays in VGPRs and
// the bit-reversal is a register renaming.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "twiddles.h"

namespace lincoll {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

constexpr int bitrev(int i, int n) {
  int r = 0;
  for (int b = 1; b < n; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// (re + i im) *= exp(-+ 2 pi i E / N)   (minus: forward, plus: inverse)
template <int N, int E, bool INV, typename T>
__device__ __forceinline__ void twiddle(T& re, T& im) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return;
  } else if constexpr (2 * e == N) {
    re = -re;
    im = -im;
  } else if constexpr (4 * e == N) {
    const T r = re;
    if constexpr (!INV) { re = im; im = -r; } else { re = -im; im = r; }
  } else if constexpr (4 * e == 3 * N) {
    const T r = re;
    if constexpr (!INV) { re = -im; im = r; } else { re = im; im = -r; }
  } else {
    constexpr int k = e * (64 / N);
    const T c = static_cast<T>(TWC[k]);
    const T s = INV ? static_cast<T>(TWS[k]) : -static_cast<T>(TWS[k]);
    const T r = re * c - im * s;
    im = re * s + im * c;
    re = r;
  }
}

// Unnormalised DFT of length N in place, natural order in and out:
//   X[k] = sum_j x[j] exp(-+ 2 pi i j k / N),
// by decimation in frequency with radix-4 steps: each step is two radix-2 DIF
// stages (spans S and S/2) done at once, leaving the same in-place layout, so
// the output is bit-reversed exactly as after radix-2 stages.  For the four
// values a, b, c, d at k, k + S/4, k + S/2, k + 3S/4 (w = exp(-+2 pi i / S)):
//   k        <- (a + c) + (b + d)
//   k +  S/4 <- ((a + c) - (b + d)) w^2k
//   k +  S/2 <- ((a - c) -+ i (b - d)) w^k
//   k + 3S/4 <- ((a - c) +- i (b - d)) w^3k
// which needs three twiddles where the two radix-2 stages need four.  An odd
// number of stages ends with one radix-2 stage of span 2 (no twiddles).
template <int N, bool INV, typename T>
__device__ __forceinline__ void fft_r4(T (&re)[N], T (&im)[N]) {
  static_assert(N >= 2 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two <= 64");
  constexpr int LOG = ilog2(N);
  static_for<0, LOG / 2>([&](auto st) {
    constexpr int span = N >> (2 * st);
    constexpr int q = span / 4;
    static_for<0, N / span>([&](auto g) {
      static_for<0, q>([&](auto k) {
        constexpr int i0 = g * span + k, i1 = i0 + q, i2 = i0 + 2 * q, i3 = i0 + 3 * q;
        const T t0r = re[i0] + re[i2], t0i = im[i0] + im[i2];
        const T t1r = re[i0] - re[i2], t1i = im[i0] - im[i2];
        const T t2r = re[i1] + re[i3], t2i = im[i1] + im[i3];
        const T dr = re[i1] - re[i3], di = im[i1] - im[i3];
        // t3 = -i (b - d) forward, +i (b - d) inverse
        const T t3r = INV ? -di : di, t3i = INV ? dr : -dr;
        re[i0] = t0r + t2r;
        im[i0] = t0i + t2i;
        T xr = t0r - t2r, xi = t0i - t2i;
        twiddle<span, 2 * k, INV>(xr, xi);
        re[i1] = xr;
        im[i1] = xi;
        xr = t1r + t3r;
        xi = t1i + t3i;
        twiddle<span, k, INV>(xr, xi);
        re[i2] = xr;
        im[i2] = xi;
        xr = t1r - t3r;
        xi = t1i - t3i;
        twiddle<span, 3 * k, INV>(xr, xi);
        re[i3] = xr;
        im[i3] = xi;
      });
    });
  });
  if constexpr (LOG % 2 == 1) {
    static_for<0, N / 2>([&](auto g) {
      constexpr int i0 = 2 * g, i1 = i0 + 1;
      const T ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
      re[i0] = ar + br;
      im[i0] = ai + bi;
      re[i1] = ar - br;
      im[i1] = ai - bi;
    });
  }
  T tr[N], ti[N];
  static_for<0, N>([&](auto i) {
    constexpr int r = bitrev(i, N);
    tr[r] = re[i];
    ti[r] = im[i];
  });
  static_for<0, N>([&](auto i) {
    re[i] = tr[i];
    im[i] = ti[i];
  });
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One decimation-in-time butterfly (a, b) <- (a + w b, a - w b) with
// w = exp(-+ 2 pi i E / S) = c + i s.  Where |c| >= |s|, w b = c u with
// u = b (1 + i s/c), so u takes two FMAs and each output component one more:
// six instructions where a product followed by the sum and difference takes
// eight (the FMA-based butterfly of Linzer and Feig, 1993; Goedecker, 1997).
// Where |s| > |c|, w = s (c/s + i) is used the same way, so the factor
// multiplying b never exceeds 1 in magnitude.
template <int S, int E, bool INV, typename T>
__device__ __forceinline__ void dit_butterfly(T& ar, T& ai, T& br, T& bi) {
  constexpr int e = ((E % S) + S) % S;
  if constexpr (e == 0) {
    const T xr = ar, xi = ai;
    ar = xr + br;
    ai = xi + bi;
    br = xr - br;
    bi = xi - bi;
  } else if constexpr (4 * e == S) {
    // w = -i (forward) or +i (inverse)
    const T tr = INV ? -bi : bi, ti = INV ? br : -br;
    const T xr = ar, xi = ai;
    ar = xr + tr;
    ai = xi + ti;
    br = xr - tr;
    bi = xi - ti;
  } else {
    constexpr int k = e * (64 / S);
    const double c = TWC[k], s = INV ? TWS[k] : -TWS[k];
    constexpr int m = e % (S / 2);   // angle modulo pi, in units of 2 pi / S
    const T xr = ar, xi = ai;
    T ur, ui, f;
    if constexpr (8 * m <= S || 8 * m >= 3 * S) {
      const T t = static_cast<T>(s / c);
      f = static_cast<T>(c);
      ur = fma_t(-t, bi, br);
      ui = fma_t(t, br, bi);
    } else {
      const T t = static_cast<T>(c / s);
      f = static_cast<T>(s);
      ur = fma_t(t, br, -bi);
      ui = fma_t(t, bi, br);
    }
    ar = fma_t(f, ur, xr);
    ai = fma_t(f, ui, xi);
    br = fma_t(-f, ur, xr);
    bi = fma_t(-f, ui, xi);
  }
}

// The same transform by radix-2 decimation in time: the input is taken in
// bit-reversed order (a register renaming) and the stages run from span 2 up
// to N, each twiddled butterfly in six FMAs (dit_butterfly).  A 32-point
// transform takes 34 twiddled and 46 plain butterflies, 388 instructions,
// against 432 with radix-4 frequency decimation.
template <int N, bool INV, typename T>
__device__ __forceinline__ void fft_dit(T (&re)[N], T (&im)[N]) {
  static_assert(N >= 2 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two <= 64");
  T tr[N], ti[N];
  static_for<0, N>([&](auto i) {
    constexpr int r = bitrev(i, N);
    tr[r] = re[i];
    ti[r] = im[i];
  });
  static_for<0, N>([&](auto i) {
    re[i] = tr[i];
    im[i] = ti[i];
  });
  static_for<1, ilog2(N) + 1>([&](auto s) {
    constexpr int span = 1 << s;
    constexpr int half = span / 2;
    static_for<0, N / span>([&](auto g) {
      static_for<0, half>([&](auto k) {
        constexpr int i0 = g * span + k;
        constexpr int i1 = i0 + half;
        dit_butterfly<span, k, INV>(re[i0], im[i0], re[i1], im[i1]);
      });
    });
  });
}

// The transform every kernel calls: decimation in time up to 32 points
// (the fewest instructions, and in the fused kernel also the fewest spills);
// at 64 points radix-4 frequency decimation compiles to fewer instructions
// in the staged kernels.
template <int N, bool INV, typename T>
__device__ __forceinline__ void fft(T (&re)[N], T (&im)[N]) {
  if constexpr (N <= 32)
    fft_dit<N, INV>(re, im);
  else
    fft_r4<N, INV>(re, im);
}

// Two real length-N sequences a, b packed as z = a + i b, transformed
// forward: returns the half spectra A[k], B[k], k = 0..N/2, times ha / (1/2)
// and hb / (1/2) (the defaults give A and B themselves; a caller that scales
// a or b by a constant passes it here, where it costs no extra multiply).
template <int N, typename T>
__device__ __forceinline__ void split_real_pair(const T (&zr)[N], const T (&zi)[N], T (&Ar)[N / 2 + 1],
                                                T (&Ai)[N / 2 + 1], T (&Br)[N / 2 + 1], T (&Bi)[N / 2 + 1],
                                                T ha = T(0.5), T hb = T(0.5)) {
  static_for<0, N / 2 + 1>([&](auto k) {
    constexpr int m = (N - k) % N;
    const T pr = zr[k], pi = zi[k], qr = zr[m], qi = -zi[m];   // Z(k), conj Z(N-k)
    Ar[k] = ha * (pr + qr);
    Ai[k] = ha * (pi + qi);
    // (Z - conj Z') / (2i)
    Br[k] = hb * (pi - qi);
    Bi[k] = -hb * (pr - qr);
  });
}

// Inverse of the above packing: from Hermitian half spectra A, B build
// Z = A + i B on all N bins (imaginary parts of the bins 0 and N/2 are
// dropped, as a real inverse transform does).
template <int N, typename T>
__device__ __forceinline__ void join_real_pair(const T (&Ar)[N / 2 + 1], const T (&Ai)[N / 2 + 1],
                                               const T (&Br)[N / 2 + 1], const T (&Bi)[N / 2 + 1], T (&zr)[N],
                                               T (&zi)[N]) {
  zr[0] = Ar[0];
  zi[0] = Br[0];
  zr[N / 2] = Ar[N / 2];
  zi[N / 2] = Br[N / 2];
  static_for<1, N / 2>([&](auto k) {
    zr[k] = Ar[k] - Bi[k];
    zi[k] = Ai[k] + Br[k];
    zr[N - k] = Ar[k] + Bi[k];
    zi[N - k] = Br[k] - Ai[k];
  });
}

}  // namespace lincoll
