// Staged (batched, multi-kernel) evaluation of the linearized operator:
// every step of Algorithm 1 as its own batched launch over all cells.
// Works for every supported (n, dtype); the fused kernel replaces it where
// one cell fits on one compute unit.
//
// Layout: real volumes [cell][x][y][z] (z fastest); spectra are half spectra
// along z stored as planes [cell][kz][kx][ky], kz = 0..n/2, complex
// interleaved.  Forward transforms are unnormalised; 1/n^3 is folded into the
// mode tables (K_j, Phi_j, Omega).  Frequencies use the natural FFT index
// K in [0, n) with |k| = min(K, n-K): every spectral factor depends on |k|
// only, so the phase origin of the grid cancels in each transform pair.
#include <type_traits>

#include "fft.h"
#include "internal.h"

namespace lincoll {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

// Arrays in device memory hold the storage type TS (float or double); every
// transform and product runs in registers of the compute type TC.  The FP32
// path uses TS = float, TC = double: on gfx950 without packed FP32 math a
// double FMA issues at the same rate as a float FMA, so the extra precision
// costs only conversions and registers, while the round-off that the
// division r = h/M amplifies (Sec. 3.3) drops to the FP32 storage rounding.

template <int NN>
__device__ __forceinline__ int fold(int K) { return K <= NN / 2 ? K : NN - K; }

// ---------------------------------------------------------------- z stage
// Prologue (Algorithm 1, first loop and the FFTs of r and f): per pair of
// columns (x, y) and (x, y + n/2) the real sequences r = chi h / M and h along
// z; the two r columns share one complex transform and the two h columns
// another (r and h are never packed together: r is large where M is small,
// and its round-off would swamp the much smaller h).
// MODE 1: M itself for the setup of nu (into H).
template <typename TS, typename T, int NN, int MODE>
__global__ void __launch_bounds__(256) k_z_fwd(const TS* __restrict__ h, double2* __restrict__ R,
                                                typename V2<TS>::t* __restrict__ H, const TS* __restrict__ fac,
                                                const TS* __restrict__ pref, const uint32_t* __restrict__ mask,
                                                int Bc, int batch) {
  using C = typename V2<TS>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, HALF = NP / 2, MW = (NN + 31) / 32;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * HALF) return;
  const int cell = (int)(gid / HALF), c = (int)(gid % HALF);
  const int x = c / (NN / 2), y1 = c % (NN / 2), y2 = y1 + NN / 2;
  const int col1 = x * NN + y1;
  const int cc = Bc > 1 ? cell : 0;
  const TS* f = fac + (size_t)cc * 6 * NN;
  const T mx = T(pref[2 * cc]) * T(f[x]);
  const T m1 = mx * T(f[NN + y1]), m2 = mx * T(f[NN + y2]);
  T ar[NN], ai[NN];
  T Ar[P], Ai[P], Br[P], Bi[P];
  const size_t b1 = (size_t)cell * P * NP + col1, b2 = b1 + NN / 2;
  if constexpr (MODE == 0) {
    const TS* h1 = h + ((size_t)cell * NP + col1) * NN;
    const TS* h2 = h1 + (size_t)(NN / 2) * NN;
    const uint32_t* mk1 = mask + ((size_t)cc * NP + col1) * MW;
    const uint32_t* mk2 = mk1 + (NN / 2) * MW;
    uint32_t k1[MW], k2[MW];
    static_for<0, MW>([&](auto w) { k1[w] = mk1[w]; k2[w] = mk2[w]; });
    static_for<0, NN>([&](auto z) {
      const T ez = T(f[2 * NN + z]);
      const T v1 = T(h1[z]), v2 = T(h2[z]);
      ar[z] = ((k1[z / 32] >> (z % 32)) & 1u) ? v1 / (m1 * ez) : T(0);
      ai[z] = ((k2[z / 32] >> (z % 32)) & 1u) ? v2 / (m2 * ez) : T(0);
    });
    fft<NN, false>(ar, ai);
    split_real_pair<NN>(ar, ai, Ar, Ai, Br, Bi);
    static_for<0, P>([&](auto k) {
      R[b1 + (size_t)k * NP] = double2{double(Ar[k]), double(Ai[k])};
      R[b2 + (size_t)k * NP] = double2{double(Br[k]), double(Bi[k])};
    });
    // h columns again (read back rather than kept live next to r)
    T hr[NN], hi[NN];
    static_for<0, NN>([&](auto z) {
      hr[z] = T(h1[z]);
      hi[z] = T(h2[z]);
    });
    fft<NN, false>(hr, hi);
    split_real_pair<NN>(hr, hi, Ar, Ai, Br, Bi);
    static_for<0, P>([&](auto k) {
      H[b1 + (size_t)k * NP] = C{TS(Ar[k]), TS(Ai[k])};
      H[b2 + (size_t)k * NP] = C{TS(Br[k]), TS(Bi[k])};
    });
  } else {
    static_for<0, NN>([&](auto z) {
      const T ez = T(f[2 * NN + z]);
      ar[z] = m1 * ez;
      ai[z] = m2 * ez;
    });
    fft<NN, false>(ar, ai);
    split_real_pair<NN>(ar, ai, Ar, Ai, Br, Bi);
    static_for<0, P>([&](auto k) {
      H[b1 + (size_t)k * NP] = C{TS(Ar[k]), TS(Ai[k])};
      H[b2 + (size_t)k * NP] = C{TS(Br[k]), TS(Bi[k])};
    });
  }
}

// Gain loop, physical-space step (Algorithm 1: psi <- M^h psi between the
// inverse and forward transforms): per pair of columns (x, y) and
// (x, y + n/2), inverse real transform along z, multiply by M^h, forward
// real transform, in place on W.
template <typename TS, typename T, int NN, typename TW>
__global__ void __launch_bounds__(256) k_z_mid(const typename V2<TW>::t* __restrict__ W, typename V2<TS>::t* __restrict__ Wq,
                                                const TS* __restrict__ fac, const TS* __restrict__ pref, int Bc,
                                                int batch) {
  using C = typename V2<TS>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, HALF = NP / 2;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * HALF) return;
  const int cell = (int)(gid / HALF), c = (int)(gid % HALF);
  const int x = c / (NN / 2), y1 = c % (NN / 2), y2 = y1 + NN / 2;
  const int cc = Bc > 1 ? cell : 0;
  const TS* f = fac + (size_t)cc * 6 * NN + 3 * NN;    // M^h factors
  const T ph = T(pref[2 * cc + 1]) * T(f[x]);
  const T m1 = ph * T(f[NN + y1]), m2 = ph * T(f[NN + y2]);
  const size_t b1 = (size_t)cell * P * NP + (size_t)x * NN + y1;
  const size_t b2 = b1 + NN / 2;
  T Ar[P], Ai[P], Br[P], Bi[P];
  static_for<0, P>([&](auto k) {
    const auto a = W[b1 + (size_t)k * NP];
    const auto b = W[b2 + (size_t)k * NP];
    Ar[k] = T(a.x); Ai[k] = T(a.y); Br[k] = T(b.x); Bi[k] = T(b.y);
  });
  T zr[NN], zi[NN];
  join_real_pair<NN>(Ar, Ai, Br, Bi, zr, zi);
  fft<NN, true>(zr, zi);
  static_for<0, NN>([&](auto z) {
    const T ez = T(f[2 * NN + z]);
    zr[z] *= m1 * ez;
    zi[z] *= m2 * ez;
  });
  fft<NN, false>(zr, zi);
  split_real_pair<NN>(zr, zi, Ar, Ai, Br, Bi);
  static_for<0, P>([&](auto k) {
    Wq[b1 + (size_t)k * NP] = C{TS(Ar[k]), TS(Ai[k])};
    Wq[b2 + (size_t)k * NP] = C{TS(Br[k]), TS(Bi[k])};
  });
}

// Epilogue (Algorithm 1, last three lines): per pair of columns, inverse
// real transforms along z of L+^ (two columns packed) and of (Omega H^) (two
// columns packed), then L = L+ - M U - nu h.
// MODE 1 (setup): nu <- inverse of H only.
template <typename TS, typename T, int NN, int MODE>
__global__ void __launch_bounds__(256) k_z_inv(const typename V2<TS>::t* __restrict__ Lp,
                                                const typename V2<TS>::t* __restrict__ H, const TS* __restrict__ h,
                                                const TS* __restrict__ nu, TS* __restrict__ out,
                                                const TS* __restrict__ fac, const TS* __restrict__ pref, int Bc,
                                                int batch, double2* __restrict__ park) {
  using C = typename V2<TS>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, HALF = NP / 2;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * HALF) return;
  const int cell = (int)(gid / HALF), c = (int)(gid % HALF);
  const int x = c / (NN / 2), y1 = c % (NN / 2), y2 = y1 + NN / 2;
  const int col1 = x * NN + y1, col2 = col1 + NN / 2;
  const int cc = Bc > 1 ? cell : 0;
  const size_t b1 = (size_t)cell * P * NP + col1, b2 = b1 + NN / 2;
  T Ar[P], Ai[P], Br[P], Bi[P];
  // n = 64: two 64-point double pencils do not fit one thread's registers;
  // L+ is transformed first and parked in double (this thread's own slots of
  // a free work buffer), then combined with the loss pencil.
  constexpr bool PARK = MODE == 0 && NN == 64;
  if constexpr (PARK) {
    T lr[NN], li[NN];
    static_for<0, P>([&](auto k) {
      const C a = Lp[b1 + (size_t)k * NP];
      const C b = Lp[b2 + (size_t)k * NP];
      Ar[k] = T(a.x); Ai[k] = T(a.y); Br[k] = T(b.x); Bi[k] = T(b.y);
    });
    join_real_pair<NN>(Ar, Ai, Br, Bi, lr, li);
    fft<NN, true>(lr, li);
    double2* pk = park + (size_t)gid * NN;
    static_for<0, NN>([&](auto z) { pk[z] = double2{double(lr[z]), double(li[z])}; });
  }
  T ur[NN], ui[NN];
  static_for<0, P>([&](auto k) {
    const C a = H[b1 + (size_t)k * NP];
    const C b = H[b2 + (size_t)k * NP];
    Ar[k] = T(a.x); Ai[k] = T(a.y); Br[k] = T(b.x); Bi[k] = T(b.y);
  });
  join_real_pair<NN>(Ar, Ai, Br, Bi, ur, ui);
  fft<NN, true>(ur, ui);                       // U on column 1 (re), column 2 (im)
  TS* o1 = out + ((size_t)cell * NP + col1) * NN;
  TS* o2 = o1 + (size_t)(NN / 2) * NN;
  if constexpr (MODE == 0) {
    T lr[NN], li[NN];
    if constexpr (!PARK) {
      static_for<0, P>([&](auto k) {
        const C a = Lp[b1 + (size_t)k * NP];
        const C b = Lp[b2 + (size_t)k * NP];
        Ar[k] = T(a.x); Ai[k] = T(a.y); Br[k] = T(b.x); Bi[k] = T(b.y);
      });
      join_real_pair<NN>(Ar, Ai, Br, Bi, lr, li);
      fft<NN, true>(lr, li);                   // L+ on column 1 (re), column 2 (im)
    }
    const TS* f = fac + (size_t)cc * 6 * NN;
    const T mx = T(pref[2 * cc]) * T(f[x]);
    const T m1 = mx * T(f[NN + y1]), m2 = mx * T(f[NN + y2]);
    const TS* h1 = h + ((size_t)cell * NP + col1) * NN;
    const TS* h2 = h1 + (size_t)(NN / 2) * NN;
    const TS* n1 = nu + ((size_t)cc * NP + col1) * NN;
    const TS* n2 = n1 + (size_t)(NN / 2) * NN;
    const double2* pk = park + (size_t)gid * NN;
    static_for<0, NN>([&](auto z) {
      const T ez = T(f[2 * NN + z]);
      T l1, l2;
      if constexpr (PARK) {
        const double2 v = pk[z];   // parked L+ (read element by element)
        l1 = T(v.x);
        l2 = T(v.y);
      } else {
        l1 = lr[z];
        l2 = li[z];
      }
      o1[z] = TS(l1 - (m1 * ez) * ur[z] - T(n1[z]) * T(h1[z]));
      o2[z] = TS(l2 - (m2 * ez) * ui[z] - T(n2[z]) * T(h2[z]));
    });
  } else {
    static_for<0, NN>([&](auto z) {
      o1[z] = TS(ur[z]);
      o2[z] = TS(ui[z]);
    });
  }
  (void)col2;
}

// ------------------------------------------------------------- xy stage
// 2-D transform over (x, y) of each kz plane, one plane per NN lanes.
// PRE 1: multiply by K_j(|kx|,|ky|,kz) before an inverse transform.
// POST 1: multiply by a radial table t(|k|^2) after a forward transform.
// POST 2: as 1 and accumulate into out (store when first).
// TPB: threads per block (64, or 32 for the half tile at n <= 32), one plane
// per NN threads.
template <typename TI, typename TO, typename TS, typename T, int NN, bool INV, int PRE, int POST, int TPB = 64>
__global__ void __launch_bounds__(TPB) k_plane(const typename V2<TI>::t* in, typename V2<TO>::t* out,
                                                const double* __restrict__ Kh, const TS* __restrict__ table, int J,
                                                int j, int Bc, int nplanes, int first) {
  using CI = typename V2<TI>::t;
  using C = typename V2<TO>::t;
  static_assert(TPB % NN == 0, "a block holds whole planes");
  constexpr int P = NN / 2 + 1, NP = NN * NN, PPB = TPB / NN, LD = NN + 1;
  // The transposes go through LDS in compute precision, one component at a
  // time: half the footprint of a complex tile, so that LDS does not limit the
  // blocks per CU below what the registers allow (at n = 64 a complex double
  // tile would leave two single-wave blocks per CU).
  __shared__ T lds[PPB * NN * LD];
  const int lp = threadIdx.x / NN, a = threadIdx.x % NN;
  const long pid = (long)blockIdx.x * PPB + lp;
  const bool active = pid < nplanes;
  const int cell = (int)(pid / P), kz = (int)(pid % P);
  const int cc = Bc > 1 ? cell : 0;
  T* sm = lds + lp * NN * LD;
  // (k1, a) -> (a, k2) when FWD, (a, k2) -> (k1, a) otherwise; w is one
  // component of this lane's pencil
  auto transpose = [&](T(&w)[NN], bool fwd) {
    static_for<0, NN>([&](auto k) { sm[fwd ? k * LD + a : a * LD + k] = w[k]; });
    __syncthreads();
    static_for<0, NN>([&](auto k) { w[k] = sm[fwd ? a * LD + k : k * LD + a]; });
    __syncthreads();
  };
  T vr[NN], vi[NN];
  // column a of the plane: element [k1][a], k1 = 0..NN-1
  if (active) {
    const CI* src = in + (size_t)pid * NP + a;
    static_for<0, NN>([&](auto k1) {
      const CI v = src[(size_t)k1 * NN];
      vr[k1] = T(v.x);
      vi[k1] = T(v.y);
    });
    if constexpr (PRE == 1) {
      const double* K = Kh + ((size_t)cc * J + j) * kh_stride(NN) + (size_t)kz * P * P + fold<NN>(a);
      static_for<0, NN>([&](auto k1) {
        const T kv = T(K[fold<NN>(k1) * P]);
        vr[k1] *= kv;
        vi[k1] *= kv;
      });
    }
  } else {
    static_for<0, NN>([&](auto k1) { vr[k1] = T(0); vi[k1] = T(0); });
  }
  fft<NN, INV>(vr, vi);                    // along the first in-plane axis
  transpose(vr, true);
  transpose(vi, true);
  fft<NN, INV>(vr, vi);                    // along the second in-plane axis
  transpose(vr, false);
  transpose(vi, false);
  if (!active) return;
  C* dst = out + (size_t)pid * NP + a;
  if constexpr (POST >= 1) {
    const TS* tj = table + (size_t)j * phi_stride(NN);
    const int fa = fold<NN>(a);
    const int qb = fa * fa + kz * kz;
    static_for<0, NN>([&](auto k1) {
      const int f1 = fold<NN>(k1);
      const T t = T(tj[qb + f1 * f1]);
      vr[k1] *= t;
      vi[k1] *= t;
    });
  }
  if constexpr (POST == 2) {
    if (!first) {
      static_for<0, NN>([&](auto k1) {
        const C o = dst[(size_t)k1 * NN];
        vr[k1] += T(o.x);
        vi[k1] += T(o.y);
      });
    }
  }
  static_for<0, NN>([&](auto k1) { dst[(size_t)k1 * NN] = C{TO(vr[k1]), TO(vi[k1])}; });
}

// ----------------------------------------------------------- launchers
// Tile of the staged path (lincoll_set_option / the launch tuner): c.zblk
// threads per block of the z-pass kernels, TPB threads per block (planes per
// block TPB / NN) of the in-plane kernels.  Neither changes the arithmetic:
// every tile gives bitwise the same result.
template <typename TS, typename T, int NN, int TPB>
static hipError_t apply_n_tile(const ApplyCtx& c) {
  using Cx = typename V2<TS>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, PPB = TPB / NN;
  const int B = c.batch;
  const TS* fac = static_cast<const TS*>(c.fac);
  const TS* pref = static_cast<const TS*>(c.pref);
  const double* Kh = static_cast<const double*>(c.Kh);
  const TS* Phi = static_cast<const TS*>(c.Phi);
  const TS* Om = static_cast<const TS*>(c.Om);
  // r-derived spectra are transformed in double for every dtype; R is stored
  // in double, W as below; H, W after the product and L+ use TS.
  double2* R = static_cast<double2*>(c.R);
  double2* W = static_cast<double2*>(c.W);
  // W between the in-plane and z passes of a node stays in double: rounding
  // this partially transformed r-derived spectrum to float (like storing the
  // kernel modes K_j in float) raised the largest element-wise FP32 error to
  // about 1.8e-5 of max |L| on per-cell Maxwellian inputs at n = 16.
  using TW = double;
  using CW = typename V2<TW>::t;
  CW* WS = static_cast<CW*>(c.W);
  Cx* H = static_cast<Cx*>(c.H);
  Cx* Wq = static_cast<Cx*>(c.Wq);
  Cx* Lp = static_cast<Cx*>(c.Lp);
  const long ncol = (long)B * NP;
  const int nplanes = B * P;
  const int zb = c.zblk;
  const dim3 gz2((unsigned)((ncol / 2 + zb - 1) / zb));
  const dim3 gp((unsigned)((nplanes + PPB - 1) / PPB));
  k_z_fwd<TS, T, NN, 0><<<gz2, zb, 0, c.stream>>>(static_cast<const TS*>(c.h), R, H, fac, pref, c.mask, c.Bc, B);
  k_plane<double, double, TS, T, NN, false, 0, 0, TPB><<<gp, TPB, 0, c.stream>>>(R, R, nullptr, nullptr, c.J, 0,
                                                                                 c.Bc, nplanes, 1);
  // Transforms of h-derived data and of the products with M^h (the loss
  // spectrum, the gain node passes, the final inverses) compute in the storage
  // precision; only the r-derived passes keep T.
  using TF = TS;
  k_plane<TS, TS, TS, TF, NN, false, 0, 1, TPB><<<gp, TPB, 0, c.stream>>>(H, H, nullptr, Om, c.J, 0, c.Bc, nplanes,
                                                                           1);
  for (int j = 0; j < c.J; ++j) {
    k_plane<double, TW, TS, T, NN, true, 1, 0, TPB><<<gp, TPB, 0, c.stream>>>(R, WS, Kh, nullptr, c.J, j, c.Bc,
                                                                              nplanes, 1);
    k_z_mid<TS, T, NN, TW><<<gz2, zb, 0, c.stream>>>(WS, Wq, fac, pref, c.Bc, B);
    if constexpr (std::is_same<TS, float>::value && (NN == 32 || NN == 64)) {
      if (c.dtype == 2) {   // BF16x3: the forward in-plane DFT stages on the matrix cores
        hipError_t e = plane_fwd_bf16x3(NN, reinterpret_cast<const float2*>(Wq), reinterpret_cast<float2*>(Lp), Phi,
                                        j, nplanes, j == 0, c.cus, c.stream);
        if (e) return e;
        continue;
      }
    }
    k_plane<TS, TS, TS, TF, NN, false, 0, 2, TPB><<<gp, TPB, 0, c.stream>>>(Wq, Lp, nullptr, Phi, c.J, j, c.Bc,
                                                                            nplanes, j == 0);
  }
  k_plane<TS, TS, TS, TF, NN, true, 0, 0, TPB><<<gp, TPB, 0, c.stream>>>(Lp, Lp, nullptr, nullptr, c.J, 0, c.Bc,
                                                                         nplanes, 1);
  k_plane<TS, TS, TS, TF, NN, true, 0, 0, TPB><<<gp, TPB, 0, c.stream>>>(H, H, nullptr, nullptr, c.J, 0, c.Bc,
                                                                         nplanes, 1);
  k_z_inv<TS, T, NN, 0><<<gz2, zb, 0, c.stream>>>(Lp, H, static_cast<const TS*>(c.h), static_cast<const TS*>(c.nu),
                                                static_cast<TS*>(c.out), fac, pref, c.Bc, B, W);
  return hipGetLastError();
}

template <typename TS, typename T, int NN>
static hipError_t apply_n(const ApplyCtx& c) {
  if (c.zblk != 64 && c.zblk != 128 && c.zblk != 256) return hipErrorInvalidValue;
  if constexpr (NN <= 32) {
    if (c.plane_tile == 1) return apply_n_tile<TS, T, NN, 32>(c);
  }
  return apply_n_tile<TS, T, NN, 64>(c);
}

bool staged_supported(int n, int dtype) {
  if (dtype == 2) return n == 32 || n == 64;   // the BF16x3 matrix-core stage exists for these
  return n == 8 || n == 16 || n == 32 || n == 64;
}

hipError_t staged_apply(const ApplyCtx& c) {
  if (c.dtype == 0) {
    switch (c.n) {
      case 8: return apply_n<double, double, 8>(c);
      case 16: return apply_n<double, double, 16>(c);
      case 32: return apply_n<double, double, 32>(c);
      case 64: return apply_n<double, double, 64>(c);
    }
  } else {
    switch (c.n) {
      case 8: return apply_n<float, double, 8>(c);
      case 16: return apply_n<float, double, 16>(c);
      case 32: return apply_n<float, double, 32>(c);
      case 64: return apply_n<float, double, 64>(c);
    }
  }
  return hipErrorInvalidValue;
}

// nu = iDFT[Omega DFT[M]] for a chunk of cells, FP64 (used by the setup).
template <int NN>
hipError_t nu_chunk(const double* fac64, const double* pref64, const double* Om64, double2* planes, double* nu64,
                    int ncell, hipStream_t s) {
  constexpr int P = NN / 2 + 1, NP = NN * NN, PPB = 64 / NN;
  const long ncol = (long)ncell * NP;
  const int nplanes = ncell * P;
  const dim3 gz2((unsigned)((ncol / 2 + 127) / 128)), gp((unsigned)((nplanes + PPB - 1) / PPB));
  k_z_fwd<double, double, NN, 1><<<gz2, 128, 0, s>>>(nullptr, nullptr, planes, fac64, pref64, nullptr, ncell, ncell);
  k_plane<double, double, double, double, NN, false, 0, 1><<<gp, 64, 0, s>>>(planes, planes, nullptr, Om64, 0, 0,
                                                                             ncell, nplanes, 1);
  k_plane<double, double, double, double, NN, true, 0, 0><<<gp, 64, 0, s>>>(planes, planes, nullptr, nullptr, 0, 0,
                                                                            ncell, nplanes, 1);
  k_z_inv<double, double, NN, 1><<<gz2, 128, 0, s>>>(nullptr, planes, nullptr, nullptr, nu64, nullptr, nullptr, ncell, ncell,
                                                    nullptr);
  return hipGetLastError();
}

hipError_t nu_chunk_dispatch(int n, const double* fac64, const double* pref64, const double* Om64, double2* planes,
                             double* nu64, int ncell, hipStream_t s) {
  switch (n) {
    case 8: return nu_chunk<8>(fac64, pref64, Om64, planes, nu64, ncell, s);
    case 16: return nu_chunk<16>(fac64, pref64, Om64, planes, nu64, ncell, s);
    case 32: return nu_chunk<32>(fac64, pref64, Om64, planes, nu64, ncell, s);
    case 64: return nu_chunk<64>(fac64, pref64, Om64, planes, nu64, ncell, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lincoll
