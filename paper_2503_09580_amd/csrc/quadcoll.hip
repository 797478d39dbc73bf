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
// in-plane transforms remain, and one kernel runs the whole azimuth loop of a
// plane pair with S accumulated in registers (k_qc_azim).
//
// Layouts: f and the result [cell][x][y][z]; every complex work volume is
// [cell][plane][a][b] with the plane index the z (or k_z) axis.
#include <hip/hip_runtime.h>

#include <cmath>

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
// MODE 1: inverse along kz of F exp(+i alpha mu p_z) and of F exp(-i alpha mu p_z),
//         scaled by 1/n^3, into cout and cout2 [plane = z][e] (G+ and G- for one
//         g-node and one polar cosine; the second read of F comes from L2).
// MODE 2: forward along z of S_j (in-plane already transformed); adds
//         W_j s_j(|k|) * result into Qk[plane = kz][e] (stores at the first node).
// MODE 3: inverse along kz; out real part to res[cell][e][z] (physical).
// MODE 4: inverse along kz; final combine into out[cell][e][z]:
//         16 pi^2 / n^3 Re(q) - f * V   (V from MODE 3).
// exp(i alpha mu p_z) for the MODE 1 pass, p_z = signed index of the plane:
// the same for every column, so it travels as a kernel argument (uniform
// across the wave) rather than being evaluated per thread.
struct ZPhase {
  double2 e[32];
};

template <int NN, int MODE>
__global__ void __launch_bounds__(128) k_qc_col(const double2* __restrict__ in, double2* __restrict__ cout,
                                                 double2* __restrict__ cout2, const double* __restrict__ f,
                                                 double* __restrict__ res, const double* __restrict__ V,
                                                 const double* __restrict__ Ws, int Q, int j, ZPhase zp,
                                                 int first, int batch) {
  constexpr int NP = NN * NN;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * NP) return;
  const int cell = (int)(gid / NP), e = (int)(gid % NP);
  double vr[NN], vi[NN];
  if constexpr (MODE == 1) {
    const double2* src = in + (size_t)cell * NN * NP + e;
    constexpr double s3 = 1.0 / ((double)NN * NN * NN);
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const double sign = pass == 0 ? 1.0 : -1.0;
      static_for<0, NN>([&](auto p) {
        const double2 v = src[(size_t)p * NP];
        const double cs = zp.e[p].x, sn = sign * zp.e[p].y;
        vr[p] = (v.x * cs - v.y * sn) * s3;
        vi[p] = (v.x * sn + v.y * cs) * s3;
      });
      fft<NN, true>(vr, vi);
      double2* dst = (pass == 0 ? cout : cout2) + (size_t)cell * NN * NP + e;
      static_for<0, NN>([&](auto p) { dst[(size_t)p * NP] = double2{vr[p], vi[p]}; });
    }
    return;
  }
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
  constexpr bool INV = MODE == 3 || MODE == 4;
  fft<NN, INV>(vr, vi);
  if constexpr (MODE == 0) {
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
// MODE 4: inverse after multiplying by a full table tab[kz][kx][ky] (the
//         hemisphere-estimated loss weight of the second mass fix, eq. (16)).
template <int NN, int MODE>
__global__ void __launch_bounds__(64) k_qc_plane(const double2* __restrict__ in, double2* __restrict__ out,
                                                  const double* __restrict__ tab, int nplanes) {
  constexpr int NP = NN * NN, PPB = 64 / NN, LD = NN + 1;
  constexpr bool INV = MODE >= 2;
  __shared__ double2 lds[PPB * NN * LD];
  static_assert(MODE >= 0 && MODE <= 4, "k_qc_plane mode");
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
    if constexpr (MODE == 4) {
      // element [k1][a] of plane kz is (kx, ky) = (k1, a)
      const double* t3 = tab + (size_t)(pid % NN) * NP + a;
      static_for<0, NN>([&](auto k1) {
        const double m = t3[(size_t)k1 * NN];
        vr[k1] *= m;
        vi[k1] *= m;
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
  static_for<0, NN>([&](auto k1) { dst[(size_t)k1 * NN] = double2{vr[k1], vi[k1]}; });
}

// All azimuths of one (g-node, polar cosine) for one plane (cell, z) per
// workgroup of 2 NN threads:
//   S (+)= sum_m w Re(c_m d_m),  c_m, d_m = iDFT_xy[G+- exp(+-i alpha (sx_m p1 + sy_m p2))]
// with sx_m, sy_m = sin(polar) (cos, sin)(2 pi m / nazim) and w the polar weight
// over nazim.  G+- stay in L2 across the azimuth loop and S is written once,
// so the HBM traffic of the loop is that of G+- and S alone.  Only Re S is
// kept: S enters Q through Re iDFT[s_j DFT S] with s_j real and even in the
// signed frequencies, which maps i Im S to a purely imaginary field.
// Lanes [0, NN) transform c and lanes [NN, 2 NN) transform d at the same time
// (lane a: column a, then row a).
// Azimuths m and nazim - m have the same sx and opposite sy.  The factor
// exp(+-i alpha sy p2) is constant along the first transform axis, so the
// first-axis transform of G+- exp(+-i alpha sx p1) is done once for the pair
// (through LDS) and the sy phase is applied after the transpose, once per
// azimuth: nazim/2 + 1 first-axis transforms instead of nazim.
// The product pairs lane a (c) with lane a + NN (d).  At NN = 32 these are the
// two halves of the wave, and v_permlane32_swap of registers x2 and x2 + 16
// leaves c[x2] d[x2] in the low half and c[x2 + 16] d[x2 + 16] in the high
// half: a VALU exchange, with identical code in both halves.  Below NN = 32
// the exchange is a shuffle, and the d lanes multiply their second-axis input
// by (-1)^p2, which shifts their output by NN/2 along x2, so that every lane
// keeps registers [0, NN/2) and sends [NN/2, NN) to its partner.  Either way
// lane a accumulates S[a][x2 < NN/2] and lane a + NN S[a][x2 >= NN/2].
// Phase tables of one g-node for k_qc_azim, one block of 2 NN threads per
// (polar cosine i, azimuth pair m): exp(i alpha sx p1) and its conjugate
// (lanes [0, NN), p1 = lane) and exp(i alpha sy p2) and its conjugate
// (lanes [NN, 2 NN), p2 = lane - NN), with (sx, sy) = sin(polar) (cos, sin)
// of azimuth m.  Layout [i][m][4][NN].
struct PolarSines {
  double v[32];
};

template <int NN>
__global__ void __launch_bounds__(2 * NN) k_qc_phases(double2* __restrict__ tab, double alpha, PolarSines st,
                                                       int nazim, int npair) {
  const int i = blockIdx.x / npair, m = blockIdx.x % npair;
  const int half = threadIdx.x / NN, a = threadIdx.x % NN;
  const double ph = 2.0 * M_PI * m / nazim;
  const double sc = half == 0 ? st.v[i] * cos(ph) : st.v[i] * sin(ph);
  double sn, cs;
  sincos(alpha * sc * sgn_idx<NN>(a), &sn, &cs);
  double2* t = tab + (size_t)blockIdx.x * 4 * NN;
  t[2 * half * NN + a] = double2{cs, sn};
  t[(2 * half + 1) * NN + a] = double2{cs, -sn};
}

__device__ __forceinline__ void swap_wave_halves(double& x, double& y) {
  // lanes 32..63 of x <-> lanes 0..31 of y
  const unsigned long long xb = __builtin_bit_cast(unsigned long long, x);
  const unsigned long long yb = __builtin_bit_cast(unsigned long long, y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
  y = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}

template <int NN>
__global__ void __launch_bounds__(2 * NN) k_qc_azim(const double2* __restrict__ Gp, const double2* __restrict__ Gm,
                                                     double2* __restrict__ S, const double2* __restrict__ tab,
                                                     double w, int nazim, int first) {
  constexpr int NP = NN * NN, LD = NN + 1, H = NN / 2;
  constexpr bool SWAP = NN == 32;      // c and d on the two halves of one wave
  __shared__ double2 Ub[2][NN * LD];   // first-axis transforms of c and d, transposed
  // exp(i alpha sx p1) and its conjugate, exp(i alpha sy p2) and its
  // conjugate, for the current pair (from the k_qc_phases tables): each lane
  // picks a table instead of multiplying by a sign
  __shared__ double2 E[4][NN];
  const int half = threadIdx.x / NN, a = threadIdx.x % NN;
  const long pid = blockIdx.x;
  double2* ub = Ub[half];
  const double2* src = (half == 0 ? Gp : Gm) + pid * NP + a;
  const double dsign = SWAP || half == 0 ? 1.0 : -1.0;   // shuffle form, d: (-1)^p2 on the odd p2
  double sacc[H], vr[NN], vi[NN];
  static_for<0, H>([&](auto x) { sacc[x] = 0.0; });
  // the 4 NN table entries of a pair, two per lane; the next pair's are
  // loaded while the current one is processed
  double2* Ef = &E[0][0];
  const int npair = nazim / 2 + 1;
  double2 t0 = tab[threadIdx.x], t1 = tab[threadIdx.x + 2 * NN];
  for (int m = 0; 2 * m <= nazim; ++m) {
    const bool pair = m > 0 && 2 * m < nazim;      // azimuth nazim - m shares sx
    Ef[threadIdx.x] = t0;
    Ef[threadIdx.x + 2 * NN] = t1;
    if (m + 1 < npair) {
      t0 = tab[(size_t)(m + 1) * 4 * NN + threadIdx.x];
      t1 = tab[(size_t)(m + 1) * 4 * NN + threadIdx.x + 2 * NN];
    }
    __syncthreads();
    const double2* e1 = E[half];   // c: exp(+i alpha sx p1), d: its conjugate
    static_for<0, NN>([&](auto k1) {
      const double2 v = src[(size_t)k1 * NN];
      const double2 e = e1[k1];
      vr[k1] = v.x * e.x - v.y * e.y;
      vi[k1] = v.x * e.y + v.y * e.x;
    });
    fft<NN, true>(vr, vi);
    static_for<0, NN>([&](auto k1) { ub[k1 * LD + a] = double2{vr[k1], vi[k1]}; });
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < (pair ? 2 : 1); ++t) {
      // read the row and the phases again for the second azimuth rather than
      // keeping 2 NN complex values live across the loop
      asm volatile("" ::: "memory");
      // the sy phase: c exp(+i ..) at azimuth m and exp(-i ..) at nazim - m, d the reverse
      const double2* e2 = E[2 + (half ^ t)];
      static_for<0, NN>([&](auto k2) {
        const double2 v = ub[a * LD + k2];
        const double2 e = e2[k2];
        double er = e.x, ei = e.y;
        if constexpr (!SWAP && k2 % 2 == 1) {
          er *= dsign;
          ei *= dsign;
        }
        vr[k2] = v.x * er - v.y * ei;
        vi[k2] = v.x * ei + v.y * er;
      });
      fft<NN, true>(vr, vi);
      if constexpr (SWAP) {
        static_for<0, H>([&](auto k) {
          double xr = vr[k], yr = vr[H + k], xi = vi[k], yi = vi[H + k];
          swap_wave_halves(xr, yr);
          swap_wave_halves(xi, yi);
          sacc[k] = fma(xr, yr, sacc[k]);
          sacc[k] = fma(-xi, yi, sacc[k]);
        });
      } else {
        static_for<0, H>([&](auto k) {
          const double rr = __shfl_xor(vr[H + k], NN, 2 * NN), ri = __shfl_xor(vi[H + k], NN, 2 * NN);
          sacc[k] = fma(vr[k], rr, sacc[k]);
          sacc[k] = fma(-vi[k], ri, sacc[k]);
        });
      }
    }
    __syncthreads();   // ub and E are rewritten for the next pair
  }
  // S[x1 = a][x2 = half H + k] (times the weight, constant over the loop) ->
  // LDS, then column-wise coalesced stores
  static_for<0, H>([&](auto k) { Ub[0][a * LD + half * H + k] = double2{w * sacc[k], 0.0}; });
  __syncthreads();
  double2* dst = S + pid * NP + a;
  static_for<0, H>([&](auto r) {
    const int x1 = half * H + r;
    const double v = Ub[0][x1 * LD + a].x;
    dst[(size_t)x1 * NN] = first ? double2{v, 0.0} : double2{dst[(size_t)x1 * NN].x + v, 0.0};
  });
}

// Loss weight of the second mass fix (eq. (16)): the sinc of the loss term
// replaced by its estimate on the hemisphere rule,
//   tab[kz][kx][ky] = 16 pi^2 / n^3 sum_j W_j sum_m w_m cos(pi g_j sigma_m . p / L)
// with p the signed frequency of (kx, ky, kz); gw = [J][2] (g_j, W_j),
// rule = [nsph][4] (sigma_m, w_m).
template <int NN>
__global__ void __launch_bounds__(256) k_qc_sph_table(double* __restrict__ tab, const double* __restrict__ gw,
                                                       int J, const double* __restrict__ rule, int nsph, double L) {
  constexpr int NP = NN * NN;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NN * NP) return;
  const double pz = sgn_idx<NN>(i / NP), px = sgn_idx<NN>((i / NN) % NN), py = sgn_idx<NN>(i % NN);
  double acc = 0.0;
  for (int j = 0; j < J; ++j) {
    const double a = M_PI * gw[2 * j] / L;
    double sj = 0.0;
    for (int m = 0; m < nsph; ++m) {
      const double* r = rule + 4 * m;
      sj += r[3] * cos(a * (r[0] * px + r[1] * py + r[2] * pz));
    }
    acc += gw[2 * j + 1] * sj;
  }
  tab[i] = 16.0 * M_PI * M_PI / ((double)NN * NP) * acc;
}

// First mass fix (eq. (15)): Q^_0 = 0, i.e. the per-cell mean of the point
// values removed.  One block per cell, FP64 sums in a fixed order.
template <int NN>
__global__ void __launch_bounds__(256) k_qc_remove_mean(double* __restrict__ q) {
  constexpr int N3 = NN * NN * NN;
  __shared__ double red[256];
  double* qc = q + (size_t)blockIdx.x * N3;
  double s = 0.0;
  for (int i = threadIdx.x; i < N3; i += 256) s += qc[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = red[0] / N3;
  for (int i = threadIdx.x; i < N3; i += 256) qc[i] -= mean;
}

template <int NN>
hipError_t quadcoll_n(const QuadCtx& c) {
  constexpr int NP = NN * NN;
  const int B = c.batch, nplanes = B * NN;
  const dim3 gc((unsigned)(((long)B * NP + 127) / 128)), gp((unsigned)((nplanes + 64 / NN - 1) / (64 / NN)));
  double2 *Fk = c.Fk, *Gp = c.Gp, *Gm = c.Gm, *C = c.C, *S = c.S, *Qk = c.Qk;
  hipStream_t s = c.stream;
  // F = DFT3[f]: along z, then in-plane
  k_qc_col<NN, 0><<<gc, 128, 0, s>>>(nullptr, Fk, nullptr, c.f, nullptr, nullptr, nullptr, 0, 0, ZPhase{}, 0, B);
  k_qc_plane<NN, 0><<<gp, 64, 0, s>>>(Fk, Fk, nullptr, nplanes);
  // loss: V = Re iDFT_u[Omega_u F] (into the output buffer's shadow V); with
  // the second mass fix the weight is the hemisphere estimate of eq. (16)
  if (c.fix == 2) {
    if (!c.Osph) return hipErrorInvalidValue;
    k_qc_plane<NN, 4><<<gp, 64, 0, s>>>(Fk, C, c.Osph, nplanes);
  } else {
    k_qc_plane<NN, 2><<<gp, 64, 0, s>>>(Fk, C, c.Om64, nplanes);
  }
  k_qc_col<NN, 3><<<gc, 128, 0, s>>>(C, nullptr, nullptr, nullptr, c.V, nullptr, nullptr, 0, 0, ZPhase{}, 0, B);
  if (c.npolar < 1 || c.npolar > 32 || c.nazim < 1 || !c.phase) return hipErrorInvalidValue;
  const int npair = c.nazim / 2 + 1;
  PolarSines sines{};
  for (int i = 0; i < c.npolar; ++i) sines.v[i] = c.st[i];
  for (int j = 0; j < c.J; ++j) {
    const double alpha = M_PI * c.g[j] / (2.0 * c.L);
    k_qc_phases<NN><<<c.npolar * npair, 2 * NN, 0, s>>>(c.phase, alpha, sines, c.nazim, npair);
    for (int i = 0; i < c.npolar; ++i) {
      ZPhase zp{};
      for (int p = 0; p < NN; ++p) {
        const double a = alpha * c.mu[i] * (p < NN / 2 ? p : p - NN);
        zp.e[p] = double2{std::cos(a), std::sin(a)};
      }
      k_qc_col<NN, 1><<<gc, 128, 0, s>>>(Fk, Gp, Gm, nullptr, nullptr, nullptr, nullptr, 0, 0, zp, 0, B);
      k_qc_azim<NN><<<nplanes, 2 * NN, 0, s>>>(Gp, Gm, S, c.phase + (size_t)i * npair * 4 * NN,
                                                 c.wpolar[i] / c.nazim, c.nazim, i == 0);
    }
    // Qk (+)= W_j s_j DFT3[S_j]
    k_qc_plane<NN, 1><<<gp, 64, 0, s>>>(S, S, nullptr, nplanes);
    k_qc_col<NN, 2><<<gc, 128, 0, s>>>(S, Qk, nullptr, nullptr, nullptr, nullptr, c.Ws, c.Q, j, ZPhase{}, j == 0, B);
  }
  // Q = 16 pi^2 / n^3 Re iDFT_u[Qk] - f V
  k_qc_plane<NN, 3><<<gp, 64, 0, s>>>(Qk, Qk, nullptr, nplanes);
  k_qc_col<NN, 4><<<gc, 128, 0, s>>>(Qk, nullptr, nullptr, c.f, c.out, c.V, nullptr, 0, 0, ZPhase{}, 0, B);
  if (c.fix == 1) k_qc_remove_mean<NN><<<B, 256, 0, s>>>(c.out);
  return hipGetLastError();
}

template <int NN>
hipError_t sph_table_n(double* tab, const double* gw, int J, const double* rule, int nsph, double L, hipStream_t s) {
  k_qc_sph_table<NN><<<(NN * NN * NN + 255) / 256, 256, 0, s>>>(tab, gw, J, rule, nsph, L);
  return hipGetLastError();
}

}  // namespace

bool quadcoll_supported(int n) { return n == 8 || n == 16 || n == 32; }

hipError_t quadcoll_sph_table(int n, double* tab, const double* gw, int J, const double* rule, int nsph, double L,
                              hipStream_t s) {
  switch (n) {
    case 8: return sph_table_n<8>(tab, gw, J, rule, nsph, L, s);
    case 16: return sph_table_n<16>(tab, gw, J, rule, nsph, L, s);
    case 32: return sph_table_n<32>(tab, gw, J, rule, nsph, L, s);
  }
  return hipErrorInvalidValue;
}

hipError_t quadcoll_apply_fp64(const QuadCtx& c) {
  switch (c.n) {
    case 8: return quadcoll_n<8>(c);
    case 16: return quadcoll_n<16>(c);
    case 32: return quadcoll_n<32>(c);
  }
  return hipErrorInvalidValue;
}

}  // namespace lincoll
