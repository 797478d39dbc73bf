// The binary collision operator Q(f, f) by the spectral method of Sec. 2.3,
// eq. (14), with a product quadrature on the hemisphere, FP64 (the residual
// of the steady-state Newton iteration, Sec. 5.2, needs it; Q itself is not
// the fast linearized method).
//
// With F = DFT[f] (unnormalised, natural index order, frequencies read as
// signed p in -n/2..n/2-1) and a_jm(p) = pi g_j (sigma_m . p) / (2L), the
// point values of eq. (14) are
//   Q(v) = 16 pi^2 / n^3 Re iDFT_u[ sum_j W_j s_j(|k|) DFT_u[S_j] ](v)
//          - f(v) Re iDFT_u[ Omega_u DFT_u[f] ](v)          (Omega_u = Omega / n^3)
//   S_j  = sum_m w_m c_jm d_jm,   c_jm, d_jm = iDFT[F exp(+-i a_jm(p))]
// (the cos*cos + sin*sin bracket of eq. (14) is A_c^2 + A_s^2 = c d with
// A_c, A_s the inverse transforms of F cos a and F sin a), s_j the sinc
// factor of the kernel modes and Omega the loss table of the linearized
// operator.  The phase exp(i a) factorises over the axes, so for one g-node
// and one polar cosine mu_i the transform along z, G_+- = iDFT_z[F
// exp(+-i alpha mu_i p_z)], serves all azimuths; per azimuth only the
// in-plane transforms remain.
//
// Layouts: f and the result [cell][x][y][z]; every complex work volume is
// [cell][plane][a][b] with the plane index the z (or k_z) axis.
#include <hip/hip_runtime.h>

#include "fft.h"
#include "internal.h"

namespace lincoll {

namespace {

template <int NN>
__device__ __forceinline__ int sgn_idx(int k) { return k < NN / 2 ? k : k - NN; }

template <int NN>
__device__ __forceinline__ int fold_q(int k) { return k <= NN / 2 ? k : NN - k; }

// ---- column transforms along the plane axis --------------------------------
// MODE 0: forward transform of the real f along z (columns contiguous in f),
//         out[plane = kz][e].
// MODE 1: inverse along kz of F exp(sign i alpha mu p_z), scaled by 1/n^3,
//         out[plane = z][e] (G+- for one g-node and one polar cosine).
// MODE 2: forward along z of S_j (in-plane already transformed); adds
//         W_j s_j(|k|) * result into Qk[plane = kz][e] (stores at the first node).
// MODE 3: inverse along kz; out real part to res[cell][e][z] (physical).
// MODE 4: inverse along kz; final combine into out[cell][e][z]:
//         16 pi^2 / n^3 Re(q) - f * V   (V from MODE 3).
template <int NN, int MODE>
__global__ void __launch_bounds__(128) k_qc_col(const double2* __restrict__ in, double2* __restrict__ cout,
                                                 const double* __restrict__ f, double* __restrict__ res,
                                                 const double* __restrict__ V, const double* __restrict__ Ws,
                                                 int Q, int j, double alpha, double mu, int sign, int first,
                                                 int batch) {
  constexpr int NP = NN * NN;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * NP) return;
  const int cell = (int)(gid / NP), e = (int)(gid % NP);
  double vr[NN], vi[NN];
  if constexpr (MODE == 0) {
    const double* src = f + ((size_t)cell * NP + e) * NN;
    static_for<0, NN>([&](auto z) {
      vr[z] = src[z];
      vi[z] = 0.0;
    });
  } else {
    const double2* src = in + (size_t)cell * NN * NP + e;
    static_for<0, NN>([&](auto p) {
      const double2 v = src[(size_t)p * NP];
      vr[p] = v.x;
      vi[p] = v.y;
    });
  }
  if constexpr (MODE == 1) {
    constexpr double s3 = 1.0 / ((double)NN * NN * NN);
    static_for<0, NN>([&](auto p) {
      double sn, cs;
      sincos(sign * alpha * mu * sgn_idx<NN>(p), &sn, &cs);
      const double r = vr[p] * cs - vi[p] * sn, i = vr[p] * sn + vi[p] * cs;
      vr[p] = r * s3;
      vi[p] = i * s3;
    });
  }
  constexpr bool INV = MODE == 1 || MODE == 3 || MODE == 4;
  fft<NN, INV>(vr, vi);
  if constexpr (MODE == 0 || MODE == 1) {
    double2* dst = cout + (size_t)cell * NN * NP + e;
    static_for<0, NN>([&](auto p) { dst[(size_t)p * NP] = double2{vr[p], vi[p]}; });
  } else if constexpr (MODE == 2) {
    const int f1 = fold_q<NN>(e / NN), f2 = fold_q<NN>(e % NN);
    const double* w = Ws + (size_t)j * Q;
    double2* dst = cout + (size_t)cell * NN * NP + e;
    static_for<0, NN>([&](auto p) {
      constexpr int fz = p <= NN / 2 ? p : NN - p;
      const double m = w[f1 * f1 + f2 * f2 + fz * fz];
      double2 o{0.0, 0.0};
      if (!first) o = dst[(size_t)p * NP];
      dst[(size_t)p * NP] = double2{o.x + m * vr[p], o.y + m * vi[p]};
    });
  } else if constexpr (MODE == 3) {
    double* dst = res + ((size_t)cell * NP + e) * NN;
    static_for<0, NN>([&](auto z) { dst[z] = vr[z]; });
  } else {
    constexpr double g = 16.0 * M_PI * M_PI / ((double)NN * NN * NN);
    const size_t o = ((size_t)cell * NP + e) * NN;
    static_for<0, NN>([&](auto z) { res[o + z] = g * vr[z] - f[o + z] * V[o + z]; });
  }
}

// ---- in-plane transforms of contiguous NN x NN planes ------------------------
// thread a of a plane holds column a ([k1][a], k1 = 0..NN-1).
// MODE 0: forward, plain.
// MODE 1: forward of S_j, plain (alias of 0, kept for clarity of the launches).
// MODE 2: inverse after multiplying by the loss table Omega_u(|k|^2) (plane = kz).
// MODE 3: inverse, plain.
// MODE 4: inverse after multiplying by exp(sign i alpha (sx p1 + sy p2)); stores c.
// MODE 5: as 4 with the conjugate phase, then S (+)= w c d (c read from cin).
template <int NN, int MODE>
__global__ void __launch_bounds__(64) k_qc_plane(const double2* __restrict__ in, double2* __restrict__ out,
                                                  const double2* __restrict__ cin, const double* __restrict__ tab,
                                                  double alpha, double sx, double sy, int sign, double w,
                                                  int first, int nplanes) {
  constexpr int NP = NN * NN, PPB = 64 / NN, LD = NN + 1;
  constexpr bool INV = MODE >= 2;
  __shared__ double2 lds[PPB * NN * LD];
  const int lp = threadIdx.x / NN, a = threadIdx.x % NN;
  const long pid = (long)blockIdx.x * PPB + lp;
  const bool active = pid < nplanes;
  double2* sm = lds + lp * NN * LD;
  double vr[NN], vi[NN];
  if (active) {
    const double2* src = in + (size_t)pid * NP + a;
    static_for<0, NN>([&](auto k1) {
      const double2 v = src[(size_t)k1 * NN];
      vr[k1] = v.x;
      vi[k1] = v.y;
    });
    if constexpr (MODE == 2) {
      const int kz = fold_q<NN>((int)(pid % NN)), fa = fold_q<NN>(a);
      static_for<0, NN>([&](auto k1) {
        constexpr int f1 = k1 <= NN / 2 ? k1 : NN - k1;
        const double m = tab[f1 * f1 + fa * fa + kz * kz];
        vr[k1] *= m;
        vi[k1] *= m;
      });
    }
    if constexpr (MODE == 4 || MODE == 5) {
      const double s = MODE == 4 ? sign : -sign;
      const double pb = alpha * sy * sgn_idx<NN>(a);
      static_for<0, NN>([&](auto k1) {
        double sn, cs;
        sincos(s * (alpha * sx * sgn_idx<NN>(k1) + pb), &sn, &cs);
        const double r = vr[k1] * cs - vi[k1] * sn, i = vr[k1] * sn + vi[k1] * cs;
        vr[k1] = r;
        vi[k1] = i;
      });
    }
  } else {
    static_for<0, NN>([&](auto k1) { vr[k1] = 0.0; vi[k1] = 0.0; });
  }
  fft<NN, INV>(vr, vi);
  static_for<0, NN>([&](auto k1) { sm[k1 * LD + a] = double2{vr[k1], vi[k1]}; });
  __syncthreads();
  static_for<0, NN>([&](auto k2) {
    const double2 v = sm[a * LD + k2];
    vr[k2] = v.x;
    vi[k2] = v.y;
  });
  fft<NN, INV>(vr, vi);
  __syncthreads();
  static_for<0, NN>([&](auto k2) { sm[a * LD + k2] = double2{vr[k2], vi[k2]}; });
  __syncthreads();
  static_for<0, NN>([&](auto k1) {
    const double2 v = sm[k1 * LD + a];
    vr[k1] = v.x;
    vi[k1] = v.y;
  });
  if (!active) return;
  double2* dst = out + (size_t)pid * NP + a;
  if constexpr (MODE == 5) {
    const double2* c = cin + (size_t)pid * NP + a;
    static_for<0, NN>([&](auto k1) {
      const double2 cv = c[(size_t)k1 * NN];
      const double pr = cv.x * vr[k1] - cv.y * vi[k1], pi = cv.x * vi[k1] + cv.y * vr[k1];
      double2 o{0.0, 0.0};
      if (!first) o = dst[(size_t)k1 * NN];
      dst[(size_t)k1 * NN] = double2{o.x + w * pr, o.y + w * pi};
    });
  } else {
    static_for<0, NN>([&](auto k1) { dst[(size_t)k1 * NN] = double2{vr[k1], vi[k1]}; });
  }
}

template <int NN>
hipError_t quadcoll_n(const QuadCtx& c) {
  constexpr int NP = NN * NN;
  const int B = c.batch, nplanes = B * NN;
  const dim3 gc((unsigned)(((long)B * NP + 127) / 128)), gp((unsigned)((nplanes + 64 / NN - 1) / (64 / NN)));
  double2 *Fk = c.Fk, *Gp = c.Gp, *Gm = c.Gm, *C = c.C, *S = c.S, *Qk = c.Qk;
  hipStream_t s = c.stream;
  // F = DFT3[f]: along z, then in-plane
  k_qc_col<NN, 0><<<gc, 128, 0, s>>>(nullptr, Fk, c.f, nullptr, nullptr, nullptr, 0, 0, 0, 0, 0, 0, B);
  k_qc_plane<NN, 0><<<gp, 64, 0, s>>>(Fk, Fk, nullptr, nullptr, 0, 0, 0, 0, 0, 0, nplanes);
  // loss: V = Re iDFT_u[Omega_u F] (into the output buffer's shadow V)
  k_qc_plane<NN, 2><<<gp, 64, 0, s>>>(Fk, C, nullptr, c.Om64, 0, 0, 0, 0, 0, 0, nplanes);
  k_qc_col<NN, 3><<<gc, 128, 0, s>>>(C, nullptr, nullptr, c.V, nullptr, nullptr, 0, 0, 0, 0, 0, 0, B);
  for (int j = 0; j < c.J; ++j) {
    const double alpha = M_PI * c.g[j] / (2.0 * c.L);
    for (int i = 0; i < c.npolar; ++i) {
      const double mu = c.mu[i], st = c.st[i];
      k_qc_col<NN, 1><<<gc, 128, 0, s>>>(Fk, Gp, nullptr, nullptr, nullptr, nullptr, 0, 0, alpha, mu, +1, 0, B);
      k_qc_col<NN, 1><<<gc, 128, 0, s>>>(Fk, Gm, nullptr, nullptr, nullptr, nullptr, 0, 0, alpha, mu, -1, 0, B);
      for (int m = 0; m < c.nazim; ++m) {
        const double phi = 2.0 * M_PI * m / c.nazim;
        const double sx = st * cos(phi), sy = st * sin(phi), w = c.wpolar[i] / c.nazim;
        k_qc_plane<NN, 4><<<gp, 64, 0, s>>>(Gp, C, nullptr, nullptr, alpha, sx, sy, +1, 0, 0, nplanes);
        k_qc_plane<NN, 5><<<gp, 64, 0, s>>>(Gm, S, C, nullptr, alpha, sx, sy, +1, w, i == 0 && m == 0, nplanes);
      }
    }
    // Qk (+)= W_j s_j DFT3[S_j]
    k_qc_plane<NN, 1><<<gp, 64, 0, s>>>(S, S, nullptr, nullptr, 0, 0, 0, 0, 0, 0, nplanes);
    k_qc_col<NN, 2><<<gc, 128, 0, s>>>(S, Qk, nullptr, nullptr, nullptr, c.Ws, c.Q, j, 0, 0, 0, j == 0, B);
  }
  // Q = 16 pi^2 / n^3 Re iDFT_u[Qk] - f V
  k_qc_plane<NN, 3><<<gp, 64, 0, s>>>(Qk, Qk, nullptr, nullptr, 0, 0, 0, 0, 0, 0, nplanes);
  k_qc_col<NN, 4><<<gc, 128, 0, s>>>(Qk, nullptr, c.f, c.out, c.V, nullptr, 0, 0, 0, 0, 0, 0, B);
  return hipGetLastError();
}

}  // namespace

bool quadcoll_supported(int n) { return n == 8 || n == 16 || n == 32; }

hipError_t quadcoll_apply_fp64(const QuadCtx& c) {
  switch (c.n) {
    case 8: return quadcoll_n<8>(c);
    case 16: return quadcoll_n<16>(c);
    case 32: return quadcoll_n<32>(c);
  }
  return hipErrorInvalidValue;
}

}  // namespace lincoll
