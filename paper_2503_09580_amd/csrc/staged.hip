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
#include "fft.h"
#include "internal.h"

namespace lincoll {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

template <int NN>
__device__ __forceinline__ int fold(int K) { return K <= NN / 2 ? K : NN - K; }

// ---------------------------------------------------------------- z stage
// Prologue (Algorithm 1, first loop and the FFTs of r and f): per column
// (cell, x, y) the two real sequences r = chi h / M and h along z, packed as
// one complex transform, split into the half spectra R and H.
// MODE 1: the same for the single sequence M (setup of nu), into H.
template <typename T, int NN, int MODE>
__global__ void __launch_bounds__(128) k_z_fwd(const T* __restrict__ h, typename V2<T>::t* __restrict__ R,
                                                typename V2<T>::t* __restrict__ H, const T* __restrict__ fac,
                                                const T* __restrict__ pref, const uint32_t* __restrict__ mask,
                                                int Bc, int batch) {
  using C = typename V2<T>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, MW = (NN + 31) / 32;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * NP) return;
  const int cell = (int)(gid / NP), col = (int)(gid % NP);
  const int x = col / NN, y = col % NN;
  const int cc = Bc > 1 ? cell : 0;
  const T* f = fac + (size_t)cc * 6 * NN;
  const T mxy = pref[2 * cc] * f[x] * f[NN + y];
  T zr[NN], zi[NN];
  if constexpr (MODE == 0) {
    const T* hc = h + ((size_t)cell * NP + col) * NN;
    const uint32_t* mk = mask + ((size_t)cc * NP + col) * MW;
    uint32_t bits[MW];
    static_for<0, MW>([&](auto w) { bits[w] = mk[w]; });
    static_for<0, NN>([&](auto z) {
      const T hv = hc[z];
      const T M = mxy * f[2 * NN + z];
      const bool keep = (bits[z / 32] >> (z % 32)) & 1u;
      zr[z] = keep ? hv / M : T(0);
      zi[z] = hv;
    });
  } else {
    static_for<0, NN>([&](auto z) {
      zr[z] = mxy * f[2 * NN + z];
      zi[z] = T(0);
    });
  }
  fft<NN, false>(zr, zi);
  T Ar[P], Ai[P], Br[P], Bi[P];
  split_real_pair<NN>(zr, zi, Ar, Ai, Br, Bi);
  const size_t base = (size_t)cell * P * NP + col;
  static_for<0, P>([&](auto k) {
    if constexpr (MODE == 0) {
      R[base + (size_t)k * NP] = C{Ar[k], Ai[k]};
      H[base + (size_t)k * NP] = C{Br[k], Bi[k]};
    } else {
      H[base + (size_t)k * NP] = C{Ar[k], Ai[k]};
    }
  });
}

// Gain loop, physical-space step (Algorithm 1: psi <- M^h psi between the
// inverse and forward transforms): per pair of columns (x, y) and
// (x, y + n/2), inverse real transform along z, multiply by M^h, forward
// real transform, in place on W.
template <typename T, int NN>
__global__ void __launch_bounds__(128) k_z_mid(typename V2<T>::t* __restrict__ W, const T* __restrict__ fac,
                                                const T* __restrict__ pref, int Bc, int batch) {
  using C = typename V2<T>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, HALF = NP / 2;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * HALF) return;
  const int cell = (int)(gid / HALF), c = (int)(gid % HALF);
  const int x = c / (NN / 2), y1 = c % (NN / 2), y2 = y1 + NN / 2;
  const int cc = Bc > 1 ? cell : 0;
  const T* f = fac + (size_t)cc * 6 * NN + 3 * NN;     // M^h factors
  const T ph = pref[2 * cc + 1] * f[x];
  const T m1 = ph * f[NN + y1], m2 = ph * f[NN + y2];
  const size_t b1 = (size_t)cell * P * NP + (size_t)x * NN + y1;
  const size_t b2 = b1 + NN / 2;
  T Ar[P], Ai[P], Br[P], Bi[P];
  static_for<0, P>([&](auto k) {
    const C a = W[b1 + (size_t)k * NP];
    const C b = W[b2 + (size_t)k * NP];
    Ar[k] = a.x; Ai[k] = a.y; Br[k] = b.x; Bi[k] = b.y;
  });
  T zr[NN], zi[NN];
  join_real_pair<NN>(Ar, Ai, Br, Bi, zr, zi);
  fft<NN, true>(zr, zi);
  static_for<0, NN>([&](auto z) {
    const T ez = f[2 * NN + z];
    zr[z] *= m1 * ez;
    zi[z] *= m2 * ez;
  });
  fft<NN, false>(zr, zi);
  split_real_pair<NN>(zr, zi, Ar, Ai, Br, Bi);
  static_for<0, P>([&](auto k) {
    W[b1 + (size_t)k * NP] = C{Ar[k], Ai[k]};
    W[b2 + (size_t)k * NP] = C{Br[k], Bi[k]};
  });
}

// Epilogue (Algorithm 1, last three lines): per column, inverse real
// transforms of L+^ and (Omega H^) along z packed as one complex transform,
// then L = L+ - M U - nu h.  MODE 1 (setup): nu <- inverse of H only.
template <typename T, int NN, int MODE>
__global__ void __launch_bounds__(128) k_z_inv(const typename V2<T>::t* __restrict__ Lp,
                                                const typename V2<T>::t* __restrict__ H, const T* __restrict__ h,
                                                const T* __restrict__ nu, T* __restrict__ out,
                                                const T* __restrict__ fac, const T* __restrict__ pref, int Bc,
                                                int batch) {
  using C = typename V2<T>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)batch * NP) return;
  const int cell = (int)(gid / NP), col = (int)(gid % NP);
  const int x = col / NN, y = col % NN;
  const int cc = Bc > 1 ? cell : 0;
  const size_t base = (size_t)cell * P * NP + col;
  T Ar[P], Ai[P], Br[P], Bi[P];
  static_for<0, P>([&](auto k) {
    const C b = H[base + (size_t)k * NP];
    Br[k] = b.x; Bi[k] = b.y;
    if constexpr (MODE == 0) {
      const C a = Lp[base + (size_t)k * NP];
      Ar[k] = a.x; Ai[k] = a.y;
    } else {
      Ar[k] = T(0); Ai[k] = T(0);
    }
  });
  T zr[NN], zi[NN];
  join_real_pair<NN>(Ar, Ai, Br, Bi, zr, zi);
  fft<NN, true>(zr, zi);
  T* oc = out + ((size_t)cell * NP + col) * NN;
  if constexpr (MODE == 0) {
    const T* f = fac + (size_t)cc * 6 * NN;
    const T mxy = pref[2 * cc] * f[x] * f[NN + y];
    const T* hc = h + ((size_t)cell * NP + col) * NN;
    const T* nc = nu + ((size_t)cc * NP + col) * NN;
    static_for<0, NN>([&](auto z) {
      const T M = mxy * f[2 * NN + z];
      oc[z] = zr[z] - M * zi[z] - nc[z] * hc[z];
    });
  } else {
    static_for<0, NN>([&](auto z) { oc[z] = zi[z]; });
  }
}

// ------------------------------------------------------------- xy stage
// 2-D transform over (x, y) of each kz plane, one plane per NN lanes.
// PRE 1: multiply by K_j(|kx|,|ky|,kz) before an inverse transform.
// POST 1: multiply by a radial table t(|k|^2) after a forward transform.
// POST 2: as 1 and accumulate into out (store when first).
template <typename T, int NN, bool INV, int PRE, int POST>
__global__ void __launch_bounds__(64) k_plane(const typename V2<T>::t* in, typename V2<T>::t* out,
                                               const T* __restrict__ Kh, const T* __restrict__ table, int J,
                                               int j, int Bc, int nplanes, int first) {
  using C = typename V2<T>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, PPB = 64 / NN, LD = NN + 1;
  __shared__ C lds[PPB * NN * LD];
  const int lp = threadIdx.x / NN, a = threadIdx.x % NN;
  const long pid = (long)blockIdx.x * PPB + lp;
  const bool active = pid < nplanes;
  const int cell = (int)(pid / P), kz = (int)(pid % P);
  const int cc = Bc > 1 ? cell : 0;
  C* sm = lds + lp * NN * LD;
  T vr[NN], vi[NN];
  // column a of the plane: element [k1][a], k1 = 0..NN-1
  if (active) {
    const C* src = in + (size_t)pid * NP + a;
    static_for<0, NN>([&](auto k1) {
      const C v = src[(size_t)k1 * NN];
      vr[k1] = v.x;
      vi[k1] = v.y;
    });
    if constexpr (PRE == 1) {
      const T* K = Kh + ((size_t)cc * J + j) * P * P * P + (size_t)kz * P * P + fold<NN>(a);
      static_for<0, NN>([&](auto k1) {
        const T kv = K[fold<NN>(k1) * P];
        vr[k1] *= kv;
        vi[k1] *= kv;
      });
    }
  } else {
    static_for<0, NN>([&](auto k1) { vr[k1] = T(0); vi[k1] = T(0); });
  }
  fft<NN, INV>(vr, vi);                    // along the first in-plane axis
  static_for<0, NN>([&](auto k1) { sm[k1 * LD + a] = C{vr[k1], vi[k1]}; });
  __syncthreads();
  static_for<0, NN>([&](auto k2) {
    const C v = sm[a * LD + k2];
    vr[k2] = v.x;
    vi[k2] = v.y;
  });
  fft<NN, INV>(vr, vi);                    // along the second in-plane axis
  __syncthreads();
  static_for<0, NN>([&](auto k2) { sm[a * LD + k2] = C{vr[k2], vi[k2]}; });
  __syncthreads();
  static_for<0, NN>([&](auto k1) {
    const C v = sm[k1 * LD + a];
    vr[k1] = v.x;
    vi[k1] = v.y;
  });
  if (!active) return;
  C* dst = out + (size_t)pid * NP + a;
  if constexpr (POST >= 1) {
    const T* tj = table + (size_t)j * (3 * (NN / 2) * (NN / 2) + 1);
    const int fa = fold<NN>(a);
    const int qb = fa * fa + kz * kz;
    static_for<0, NN>([&](auto k1) {
      const int f1 = fold<NN>(k1);
      const T t = tj[qb + f1 * f1];
      vr[k1] *= t;
      vi[k1] *= t;
    });
  }
  if constexpr (POST == 2) {
    if (!first) {
      static_for<0, NN>([&](auto k1) {
        const C o = dst[(size_t)k1 * NN];
        vr[k1] += o.x;
        vi[k1] += o.y;
      });
    }
  }
  static_for<0, NN>([&](auto k1) { dst[(size_t)k1 * NN] = C{vr[k1], vi[k1]}; });
}

// ----------------------------------------------------------- launchers
template <typename T, int NN>
static hipError_t apply_n(const ApplyCtx& c) {
  using Cx = typename V2<T>::t;
  constexpr int P = NN / 2 + 1, NP = NN * NN, PPB = 64 / NN;
  const int B = c.batch;
  const T* fac = static_cast<const T*>(c.fac);
  const T* pref = static_cast<const T*>(c.pref);
  const T* Kh = static_cast<const T*>(c.Kh);
  const T* Phi = static_cast<const T*>(c.Phi);
  const T* Om = static_cast<const T*>(c.Om);
  Cx* R = static_cast<Cx*>(c.R);
  Cx* H = static_cast<Cx*>(c.H);
  Cx* W = static_cast<Cx*>(c.W);
  Cx* Lp = static_cast<Cx*>(c.Lp);
  const long ncol = (long)B * NP;
  const int nplanes = B * P;
  const dim3 gz((unsigned)((ncol + 127) / 128)), gz2((unsigned)((ncol / 2 + 127) / 128));
  const dim3 gp((unsigned)((nplanes + PPB - 1) / PPB));
  k_z_fwd<T, NN, 0><<<gz, 128, 0, c.stream>>>(static_cast<const T*>(c.h), R, H, fac, pref, c.mask, c.Bc, B);
  k_plane<T, NN, false, 0, 0><<<gp, 64, 0, c.stream>>>(R, R, nullptr, nullptr, c.J, 0, c.Bc, nplanes, 1);
  k_plane<T, NN, false, 0, 1><<<gp, 64, 0, c.stream>>>(H, H, nullptr, Om, c.J, 0, c.Bc, nplanes, 1);
  for (int j = 0; j < c.J; ++j) {
    k_plane<T, NN, true, 1, 0><<<gp, 64, 0, c.stream>>>(R, W, Kh, nullptr, c.J, j, c.Bc, nplanes, 1);
    k_z_mid<T, NN><<<gz2, 128, 0, c.stream>>>(W, fac, pref, c.Bc, B);
    k_plane<T, NN, false, 0, 2><<<gp, 64, 0, c.stream>>>(W, Lp, nullptr, Phi, c.J, j, c.Bc, nplanes, j == 0);
  }
  k_plane<T, NN, true, 0, 0><<<gp, 64, 0, c.stream>>>(Lp, Lp, nullptr, nullptr, c.J, 0, c.Bc, nplanes, 1);
  k_plane<T, NN, true, 0, 0><<<gp, 64, 0, c.stream>>>(H, H, nullptr, nullptr, c.J, 0, c.Bc, nplanes, 1);
  k_z_inv<T, NN, 0><<<gz, 128, 0, c.stream>>>(Lp, H, static_cast<const T*>(c.h), static_cast<const T*>(c.nu),
                                             static_cast<T*>(c.out), fac, pref, c.Bc, B);
  return hipGetLastError();
}

bool staged_supported(int n, int dtype) {
  if (dtype == 0) return n == 8 || n == 16 || n == 32;
  return n == 8 || n == 16 || n == 32 || n == 64;
}

hipError_t staged_apply(const ApplyCtx& c) {
  if (c.dtype == 0) {
    switch (c.n) {
      case 8: return apply_n<double, 8>(c);
      case 16: return apply_n<double, 16>(c);
      case 32: return apply_n<double, 32>(c);
    }
  } else {
    switch (c.n) {
      case 8: return apply_n<float, 8>(c);
      case 16: return apply_n<float, 16>(c);
      case 32: return apply_n<float, 32>(c);
      case 64: return apply_n<float, 64>(c);
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
  const dim3 gz((unsigned)((ncol + 127) / 128)), gp((unsigned)((nplanes + PPB - 1) / PPB));
  k_z_fwd<double, NN, 1><<<gz, 128, 0, s>>>(nullptr, nullptr, planes, fac64, pref64, nullptr, ncell, ncell);
  k_plane<double, NN, false, 0, 1><<<gp, 64, 0, s>>>(planes, planes, nullptr, Om64, 0, 0, ncell, nplanes, 1);
  k_plane<double, NN, true, 0, 0><<<gp, 64, 0, s>>>(planes, planes, nullptr, nullptr, 0, 0, ncell, nplanes, 1);
  k_z_inv<double, NN, 1><<<gz, 128, 0, s>>>(nullptr, planes, nullptr, nullptr, nu64, nullptr, nullptr, ncell, ncell);
  return hipGetLastError();
}

hipError_t nu_chunk_dispatch(int n, const double* fac64, const double* pref64, const double* Om64, double2* planes,
                             double* nu64, int ncell, hipStream_t s) {
  switch (n) {
    case 8: return nu_chunk<8>(fac64, pref64, Om64, planes, nu64, ncell, s);
    case 16: return nu_chunk<16>(fac64, pref64, Om64, planes, nu64, ncell, s);
    case 32: return nu_chunk<32>(fac64, pref64, Om64, planes, nu64, ncell, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lincoll
