// Fused persistent kernel: one workgroup per cell (looping over cells) runs
// all of Algorithm 1 on chip; only the FP64 spectrum of r streams from a
// per-workgroup scratch slot, once per quadrature node.  For batches too
// small to fill the chip, k_fused_split runs the same body with each cell's
// quadrature nodes partitioned over several workgroups (and the loss term in
// a work item of its own where the chip has room); k_fused_sum adds the
// partial gain sums and k_fused_finish applies the last inverse transform.
//
// Grid-of-pencils layout for n = NN points per axis (N = NN/2, KP = N packed
// z-planes, NN*N threads).  The real transform along z packs the real bins
// kz = 0 and kz = N of each column into one complex value, so every spectral
// array is KP planes of NN x NN complex values.
//   Y role: thread t = (kp, a) = (t / NN, t % NN) owns the pencil along ky of
//           plane kp at kx = a.
//   X role: thread t = (kp, b) owns the pencil along x (or kx) at y (ky) = b.
//   Z role: thread t = (x, yp) = (t / N, t % N) owns the columns (x, yp) and
//           (x, yp + N) along z.
// A wave holds whole planes in the Y and X roles (64 / NN planes), so the
// Y <-> X transposes are local to a wave's own LDS region and need no
// workgroup barrier; only X <-> Z exchanges synchronise the workgroup.
//
// Precision (FP32 at the HBM boundary): everything that acts on r-derived data
// (the forward transform of r = chi h / M, its stored spectrum, the kernel
// modes K_j, the inverse transforms giving psi_j) is double, including the
// LDS exchanges between axis passes, which move one component at a time.  r
// is large where M is small (Sec. 3.3): a float rounding anywhere on that
// path (of K_j, or of partially transformed values between passes) spreads
// that size over the box and cost up to 1.8e-5 of max |L| element-wise.
// After the product with M^h everything runs in float.  F64 plans run the
// same kernel with that second half (and h, L, nu and the radial tables) in
// double.
//
// LDS: one float2 volume for the exchanges (double data in two rounds), the
// radial table of the node, the 1-D Maxwellian factors and (n = 32) two
// chunks of each thread's L+^ accumulator.  The kernel modes K_j of a node are needed
// only in the Y role, where each wave handles its own planes: each wave
// copies its planes of K_j (and, wave 0, the Nyquist plane kz = N) into its
// own region of the exchange volume, which no other wave touches between the
// end of one node's forward transform and the start of the next node's
// X -> Z exchange.
#include <mutex>

#include "fft.h"
#include "internal.h"

namespace lincoll {

// Slots of lincoll_apply_noalloc: the persistent workgroups' scratch (the
// spectrum of r and the L+ accumulator) in a file-scope device array instead
// of plan memory, so that the entry point allocates nothing.  Each device the
// library runs on holds its own copy until the process ends.  96 MiB holds
// 256 F32 slots at n = 32 (one per compute unit of an MI355X) or 1024 at
// n = 16; 192 and 1536 F64 slots.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

template <int NN>
struct Cfg {
  static constexpr int N = NN / 2;
  static constexpr int KP = N;                 // packed planes
  static constexpr int T = NN * N;             // threads
  static constexpr int P = N + 1;
  static constexpr int P3 = P * P * P;
  static constexpr int Q = 3 * N * N + 1;
  static constexpr int MW = (NN + 31) / 32;
  static constexpr int LD = NN + 1;            // padded LDS row
  static constexpr int LDS_BYTES = KP * NN * LD * 8;   // one float2 volume
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copy count floats from global memory into LDS with the direct load-to-LDS
// path (no registers involved): wave w moves 64-float chunks w, w + nw, ...
// Completion is tracked by vmcnt; the caller waits for it and synchronises the
// workgroup before the data is read.
__device__ __forceinline__ void lds_dma(const float* src, float* dst, int count, int t, int nthreads) {
  const int wave = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64, nw = nthreads / 64;
  for (int c = wave; c * 64 < count; c += nw) {
    const int q = c * 64 + lane;
    if (q < count)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + q),
                                       (__attribute__((address_space(3))) void*)(dst + c * 64), 4, 0, 0);
  }
}

// ---- z stage: two real columns <-> their packed half spectra ------------------
// forward: a, b real (as zr, zi) -> v[k] (column a) and v[N + k] (column b),
// k < N; bin 0 holds (A(0), A(N)), bins 1..N-1 the complex A(k).  The
// spectra come out scaled by ga and gb.
template <int NN, typename T>
__device__ __forceinline__ void z_forward(T (&zr)[NN], T (&zi)[NN], T (&vr)[NN], T (&vi)[NN], T ga = T(1),
                                          T gb = T(1)) {
  constexpr int N = NN / 2;
  fft<NN, false>(zr, zi);
  T Ar[N + 1], Ai[N + 1], Br[N + 1], Bi[N + 1];
  split_real_pair<NN>(zr, zi, Ar, Ai, Br, Bi, T(0.5) * ga, T(0.5) * gb);
  vr[0] = Ar[0];
  vi[0] = Ar[N];
  vr[N] = Br[0];
  vi[N] = Br[N];
  static_for<1, N>([&](auto k) {
    vr[k] = Ar[k];
    vi[k] = Ai[k];
    vr[N + k] = Br[k];
    vi[N + k] = Bi[k];
  });
}

template <int NN, typename T>
__device__ __forceinline__ void z_inverse(const T (&vr)[NN], const T (&vi)[NN], T (&zr)[NN], T (&zi)[NN]) {
  constexpr int N = NN / 2;
  T Ar[N + 1], Ai[N + 1], Br[N + 1], Bi[N + 1];
  Ar[0] = vr[0]; Ai[0] = T(0); Ar[N] = vi[0]; Ai[N] = T(0);
  Br[0] = vr[N]; Bi[0] = T(0); Br[N] = vi[N]; Bi[N] = T(0);
  static_for<1, N>([&](auto k) {
    Ar[k] = vr[k]; Ai[k] = vi[k];
    Br[k] = vr[N + k]; Bi[k] = vi[N + k];
  });
  join_real_pair<NN>(Ar, Ai, Br, Bi, zr, zi);
  fft<NN, true>(zr, zi);
}

// Wave-private copy of K_j: wave w's planes kp = w*PW .. w*PW+PW-1 of the
// octant [P][P][P] (and, wave 0 only, plane N after them) into the start of
// the wave's own region of the exchange volume, as double.  Completion is
// tracked by vmcnt; the wave waits for it before reading.
template <int NN>
__device__ __forceinline__ void k_slice_dma(const double* Kj, float2* lds, int t) {
  constexpr int N = NN / 2, P = N + 1, PP = P * P, PW = 64 / NN, LD = NN + 1;
  const int wave = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64;
  float* dst = reinterpret_cast<float*>(lds + wave * PW * NN * LD);
  auto copy = [&](const float* src, float* d, int count) {
    for (int c = 0; c * 64 < count; ++c) {
      const int q = c * 64 + lane;
      if (q < count)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + q),
                                         (__attribute__((address_space(3))) void*)(d + c * 64), 4, 0, 0);
    }
  };
  copy(reinterpret_cast<const float*>(Kj + (size_t)wave * PW * PP), dst, PW * PP * 2);
  if (wave == 0) copy(reinterpret_cast<const float*>(Kj + (size_t)N * PP), dst + PW * PP * 2, PP * 2);
}

// ---- transposes through LDS (float2 storage) ----------------------------------
// Within plane kp: thread (kp, i) holds v[j] = element (i, j); afterwards it
// holds v[j] = element (j, i).  Plane kp lives in the region of the wave that
// owns it, so a wave-level fence suffices.
template <int NN, typename T>
__device__ __forceinline__ void transpose_plane(T (&vr)[NN], T (&vi)[NN], float2* lds, int t) {
  constexpr int LD = NN + 1;
  const int kp = t / NN, i = t % NN;
  float2* pl = lds + kp * NN * LD;
  static_for<0, NN>([&](auto j) { pl[i * LD + j] = float2{float(vr[j]), float(vi[j])}; });
  wave_lds_sync();
  static_for<0, NN>([&](auto j) {
    const float2 v = pl[j * LD + i];
    vr[j] = T(v.x);
    vi[j] = T(v.y);
  });
  wave_lds_sync();
}

// X role (kp, y) holding v[x] -> Z role (x, yp) holding v[k] = (k, x, yp),
// v[N + k] = (k, x, yp + N).  Writes go to the writer's own plane region.
template <int NN, typename T>
__device__ __forceinline__ void x_to_z(T (&vr)[NN], T (&vi)[NN], float2* lds, int t) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  static_for<0, NN>([&](auto xx) { lds[(kp * NN + xx) * LD + y] = float2{float(vr[xx]), float(vi[xx])}; });
  __syncthreads();
  static_for<0, KP>([&](auto k) {
    const float2 a = lds[(k * NN + x) * LD + yp];
    const float2 b = lds[(k * NN + x) * LD + yp + N];
    vr[k] = T(a.x); vi[k] = T(a.y);
    vr[N + k] = T(b.x); vi[N + k] = T(b.y);
  });
}

// Z role -> X role.  Reads come from the reader's own plane region.
template <int NN, typename T>
__device__ __forceinline__ void z_to_x(T (&vr)[NN], T (&vi)[NN], float2* lds, int t) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  __syncthreads();
  static_for<0, KP>([&](auto k) {
    lds[(k * NN + x) * LD + yp] = float2{float(vr[k]), float(vi[k])};
    lds[(k * NN + x) * LD + yp + N] = float2{float(vr[N + k]), float(vi[N + k])};
  });
  __syncthreads();
  static_for<0, NN>([&](auto xx) {
    const float2 a = lds[(kp * NN + xx) * LD + y];
    vr[xx] = T(a.x);
    vi[xx] = T(a.y);
  });
}

// The same three exchanges in double for r-derived data: the volume holds
// one double per complex slot, so the real and the imaginary parts go in two
// rounds.
template <int NN>
__device__ __forceinline__ void transpose_plane_d(double (&vr)[NN], double (&vi)[NN], float2* lds, int t) {
  constexpr int LD = NN + 1;
  const int kp = t / NN, i = t % NN;
  double* pl = reinterpret_cast<double*>(lds + kp * NN * LD);
  auto one = [&](double(&w)[NN]) {
    static_for<0, NN>([&](auto j) { pl[i * LD + j] = w[j]; });
    wave_lds_sync();
    static_for<0, NN>([&](auto j) { w[j] = pl[j * LD + i]; });
    wave_lds_sync();
  };
  one(vr);
  one(vi);
}

template <int NN>
__device__ __forceinline__ void x_to_z_d(double (&vr)[NN], double (&vi)[NN], float2* lds, int t) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  double* ld = reinterpret_cast<double*>(lds);
  auto one = [&](double(&w)[NN]) {
    static_for<0, NN>([&](auto xx) { ld[(kp * NN + xx) * LD + y] = w[xx]; });
    __syncthreads();
    static_for<0, KP>([&](auto k) {
      w[k] = ld[(k * NN + x) * LD + yp];
      w[N + k] = ld[(k * NN + x) * LD + yp + N];
    });
  };
  one(vr);
  __syncthreads();   // every wave has read the real parts
  one(vi);
}

template <int NN>
__device__ __forceinline__ void z_to_x_d(double (&vr)[NN], double (&vi)[NN], float2* lds, int t) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  double* ld = reinterpret_cast<double*>(lds);
  auto one = [&](double(&w)[NN]) {
    __syncthreads();
    static_for<0, KP>([&](auto k) {
      ld[(k * NN + x) * LD + yp] = w[k];
      ld[(k * NN + x) * LD + yp + N] = w[N + k];
    });
    __syncthreads();
    static_for<0, NN>([&](auto xx) { w[xx] = ld[(kp * NN + xx) * LD + y]; });
  };
  one(vr);
  one(vi);
}

// Y role, pencil along ky: multiply by a real spectral factor m(kx, ky, kz)
// that is even in every component.  getm(ky) returns (m at the pencil's own
// plane, m at kz = N).  Plane 0 carries kz = 0 (real part) and kz = N
// (imaginary part), each Hermitian in (kx, ky); multiplying the two by
// different factors m0, mN needs the value at (-kx, -ky), held by lane
// (NN - kx) % NN of wave 0:  v' = (m0 + mN)/2 v + (m0 - mN)/2 conj(v(-k)).
// Indices ky and -ky are handled together so that every lane reads its
// partner's values before either is overwritten.
template <int NN, typename T, typename G>
__device__ __forceinline__ void mode_multiply(T (&vr)[NN], T (&vi)[NN], int t, G&& getm) {
  if (t < 64) {
    const bool packed = t < NN;                 // plane 0
    const int partner = packed ? (NN - t) % NN : t;
    static_for<0, NN / 2 + 1>([&](auto j) {
      constexpr int jm = (NN - j) % NN;
      const T ar = __shfl(vr[jm], partner, 64), ai = __shfl(vi[jm], partner, 64);
      const T br = __shfl(vr[j], partner, 64), bi = __shfl(vi[j], partner, 64);
      {
        const auto m = getm(j);
        const T s = packed ? T(0.5) * (T(m.x) + T(m.y)) : T(m.x);
        const T d = packed ? T(0.5) * (T(m.x) - T(m.y)) : T(0);
        const T nr = s * vr[j] + d * ar, ni = s * vi[j] - d * ai;
        vr[j] = nr;
        vi[j] = ni;
      }
      if constexpr (jm != j) {
        const auto m = getm(std::integral_constant<int, jm>{});
        const T s = packed ? T(0.5) * (T(m.x) + T(m.y)) : T(m.x);
        const T d = packed ? T(0.5) * (T(m.x) - T(m.y)) : T(0);
        const T nr = s * vr[jm] + d * br, ni = s * vi[jm] - d * bi;
        vr[jm] = nr;
        vi[jm] = ni;
      }
    });
  } else {
    static_for<0, NN>([&](auto j) {
      const T m = T(getm(j).x);
      vr[j] *= m;
      vi[j] *= m;
    });
  }
}

// Doubles of wave 0's copy of K_j in its LDS region: its PW planes and the
// Nyquist plane kz = N.
template <int NN>
constexpr int kslice_doubles() { return (64 / NN + 1) * (NN / 2 + 1) * (NN / 2 + 1); }

// The same product for the FP64 pencils of the K_j step, written so that no
// branch produces a second copy of the pencil (a divergent or wave-level
// branch whose two sides both rewrite all 2 NN doubles made the compiler keep
// both, which spilled the whole gain loop).  Every lane multiplies by its own
// plane's factor; on the packed plane that factor is s = (m0 + mN)/2, which
// wave 0 writes over m0 in its LDS copy (and d = (m0 - mN)/2 over mN), and
// the packed lanes then add d conj(v(-k)) in place, one component at a time:
// the real part of v' = s v + d conj(v(-k)) needs only real parts, the
// imaginary part only imaginary parts.  The partner values come from a free
// part of wave 0's own region, after the K_j copy.
template <int NN, typename G>
__device__ __forceinline__ void mode_multiply_d(double (&vr)[NN], double (&vi)[NN], int t, double* region, G&& getm) {
  constexpr int P = NN / 2 + 1, PP = P * P, PW = 64 / NN;
  constexpr int OFF = (kslice_doubles<NN>() + 63) / 64 * 64;
  static_assert(OFF + NN * NN <= PW * NN * (NN + 1), "partner buffer exceeds the wave's LDS region");
  const bool packed = t < NN;                       // plane 0, wave 0
  const int lane = t % NN, partner = (NN - lane) % NN;
  double* buf = region + OFF;
  if (__builtin_amdgcn_readfirstlane(t) < 64)       // wave 0 (a wave-uniform branch)
    for (int q = t; q < PP; q += 64) {
      const double m0 = region[q], mN = region[PW * PP + q];
      region[q] = 0.5 * (m0 + mN);
      region[PW * PP + q] = 0.5 * (m0 - mN);
    }
  auto one = [&](double(&w)[NN], double sign) {
    if (packed) static_for<0, NN>([&](auto j) { buf[j * NN + lane] = w[j]; });
    wave_lds_sync();
    static_for<0, NN>([&](auto j) { w[j] *= getm(j).x; });
    if (packed)
      static_for<0, NN>([&](auto j) {
        constexpr int jm = (NN - j) % NN;
        w[j] = fma(sign * getm(j).y, buf[jm * NN + partner], w[j]);
      });
    wave_lds_sync();
  };
  one(vr, 1.0);
  one(vi, -1.0);
}

// The FP64 form of mode_multiply for a radial table (the loss's Omega and the
// gain's Phi_j in an FP64 apply), without a branch that copies the pencil:
// every lane multiplies by its own plane's factor m0, and wave 0's packed
// lanes then overwrite that product with s v + d conj(v(-k)), s and d as
// above, one component at a time, from the original values parked in the same
// free part of wave 0's LDS region that mode_multiply_d uses (so no
// difference of the two products is formed).
template <int NN, typename G>
__device__ __forceinline__ void mode_multiply_tab_d(double (&vr)[NN], double (&vi)[NN], int t, double* region,
                                                    G&& getm) {
  constexpr int PW = 64 / NN;
  constexpr int OFF = (kslice_doubles<NN>() + 63) / 64 * 64;
  static_assert(OFF + NN * NN <= PW * NN * (NN + 1), "partner buffer exceeds the wave's LDS region");
  const bool packed = t < NN;
  const int lane = t % NN, partner = (NN - lane) % NN;
  double* buf = region + OFF;
  auto one = [&](double(&w)[NN], double sign) {
    if (packed) static_for<0, NN>([&](auto j) { buf[j * NN + lane] = w[j]; });
    wave_lds_sync();
    static_for<0, NN>([&](auto j) { w[j] *= getm(j).x; });
    if (packed)
      static_for<0, NN>([&](auto j) {
        constexpr int jm = (NN - j) % NN;
        const auto m = getm(j);
        w[j] = fma(0.5 * (m.x - m.y), sign * buf[jm * NN + partner], 0.5 * (m.x + m.y) * buf[j * NN + lane]);
      });
    wave_lds_sync();
  };
  one(vr, 1.0);
  one(vi, -1.0);
}

// The pieces of the fused kernel that depend on the arithmetic type TL of
// everything after the product with M^h (float for F32 plans, double for F64):
// the exchanges through LDS, the radial-table product and the accumulator's
// chunks (two complex floats or one complex double).
template <int NN, typename TL>
__device__ __forceinline__ void exch_z_to_x(TL (&vr)[NN], TL (&vi)[NN], float2* lds, int t) {
  if constexpr (std::is_same<TL, float>::value) z_to_x<NN, float>(vr, vi, lds, t);
  else z_to_x_d<NN>(vr, vi, lds, t);
}
template <int NN, typename TL>
__device__ __forceinline__ void exch_x_to_z(TL (&vr)[NN], TL (&vi)[NN], float2* lds, int t) {
  if constexpr (std::is_same<TL, float>::value) x_to_z<NN, float>(vr, vi, lds, t);
  else x_to_z_d<NN>(vr, vi, lds, t);
}
template <int NN, typename TL>
__device__ __forceinline__ void exch_transpose(TL (&vr)[NN], TL (&vi)[NN], float2* lds, int t) {
  if constexpr (std::is_same<TL, float>::value) transpose_plane<NN, float>(vr, vi, lds, t);
  else transpose_plane_d<NN>(vr, vi, lds, t);
}
template <int NN, typename TL, typename G>
__device__ __forceinline__ void radial_multiply(TL (&vr)[NN], TL (&vi)[NN], int t, float2* lds, G&& getm) {
  if constexpr (std::is_same<TL, float>::value) {
    mode_multiply<NN, float>(vr, vi, t, getm);
  } else {
    constexpr int PW = 64 / NN, LD = NN + 1;
    mode_multiply_tab_d<NN>(vr, vi, t, reinterpret_cast<double*>(lds + (t / 64) * PW * NN * LD), getm);
  }
}

template <typename TL>
struct AccChunk;
template <>
struct AccChunk<float> {   // two complex values
  using V = float4;
  static constexpr int PER = 2;
  __device__ static float re(const V& a, int p) { return p ? a.z : a.x; }
  __device__ static float im(const V& a, int p) { return p ? a.w : a.y; }
  template <int NN>
  __device__ static V make(const float (&r)[NN], const float (&i)[NN], int c) {
    return V{r[2 * c], i[2 * c], r[2 * c + 1], i[2 * c + 1]};
  }
};
template <>
struct AccChunk<double> {   // one complex value
  using V = double2;
  static constexpr int PER = 1;
  __device__ static double re(const V& a, int) { return a.x; }
  __device__ static double im(const V& a, int) { return a.y; }
  template <int NN>
  __device__ static V make(const double (&r)[NN], const double (&i)[NN], int c) {
    return V{r[c], i[c]};
  }
};

template <typename TL>
using Cplx = typename std::conditional<std::is_same<TL, float>::value, float2, double2>::type;

// L+ = iDFT[L+^] from the Y-role pencils of one cell, added to out (Alg. 1,
// the inverse transform of the gain sum and the combination with the loss).
template <int NN, typename TL>
__device__ __forceinline__ void gain_inverse_add(TL (&Lr)[NN], TL (&Li)[NN], float2* lds, int t, TL* out, int cell,
                                                 int col1) {
  constexpr int N = NN / 2, NP = NN * NN;
  fft<NN, true>(Lr, Li);
  exch_transpose<NN, TL>(Lr, Li, lds, t);
  fft<NN, true>(Lr, Li);
  exch_x_to_z<NN, TL>(Lr, Li, lds, t);
  TL zr[NN], zi[NN];
  z_inverse<NN, TL>(Lr, Li, zr, zi);
  TL* o1 = out + ((size_t)cell * NP + col1) * NN;
  TL* o2 = o1 + (size_t)N * NN;
  static_for<0, NN>([&](auto z) {
    o1[z] = o1[z] + zr[z];
    o2[z] = o2[z] + zi[z];
  });
}

}  // namespace

// The whole apply (Algorithm 1) for each cell of the batch, one workgroup
// per cell at a time, persistent over cells (the body: fused_body.inc).
template <int NN, int KA, typename TL>
__global__ void __launch_bounds__(Cfg<NN>::T) k_fused(
    const TL* __restrict__ h, TL* __restrict__ out, int batch, int Bc, const double* __restrict__ fac64,
    const double* __restrict__ pref64, const uint32_t* __restrict__ mask, const double* __restrict__ Kh,
    const TL* __restrict__ nu, const TL* __restrict__ Phi, const TL* __restrict__ Om,
    double2* __restrict__ slots, int J, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a gated-off step of the device-resident GMRES
  constexpr bool SPLIT = false;
  constexpr int S = 1, LI = 0;
  Cplx<TL>* const partial = nullptr;
#include "fused_body.inc"
}

// The apply with each cell's J nodes split over S workgroups (for batches
// too small to fill the chip one cell per workgroup).  Work item w is part
// w % (S + LI) of cell w / (S + LI); part p < S writes its partial gain sum to
// partial[cell S + p]; with LI = 1, part S computes the loss term alone.
template <int NN, int KA, typename TL>
__global__ void __launch_bounds__(Cfg<NN>::T) k_fused_split(
    const TL* __restrict__ h, TL* __restrict__ out, int batch, int Bc, const double* __restrict__ fac64,
    const double* __restrict__ pref64, const uint32_t* __restrict__ mask, const double* __restrict__ Kh,
    const TL* __restrict__ nu, const TL* __restrict__ Phi, const TL* __restrict__ Om,
    double2* __restrict__ slots, int J, int S, int LI, Cplx<TL>* __restrict__ partial,
    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  constexpr bool SPLIT = true;
#include "fused_body.inc"
}

// Adds the S partial gain sums of each cell of a split apply, in part order,
// into its part 0 (in place: element e of a cell is read and written by one
// thread).  Spread over many workgroups, so that the sum reads the parts at
// the chip's bandwidth rather than one workgroup's.
template <typename T2>
__global__ void __launch_bounds__(256) k_fused_sum(T2* __restrict__ partial, long per_item, int batch, int S,
                                                   const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const long total = (long)batch * per_item;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long cell = i / per_item;
    T2* base = partial + cell * S * per_item + (i - cell * per_item);
    T2 acc = base[0];
    for (int p = 1; p < S; ++p) {
      const T2 v = base[p * per_item];
      acc.x += v.x;
      acc.y += v.y;
    }
    base[0] = acc;
  }
}

// Completes a split apply: from each cell's summed gain spectrum (its part 0
// after k_fused_sum), L+ = iDFT[L+^] and out += L+.
template <int NN, typename TL>
__global__ void __launch_bounds__(Cfg<NN>::T) k_fused_finish(TL* __restrict__ out, int batch,
                                                            const Cplx<TL>* __restrict__ partial, int S,
                                                            const int* __restrict__ gate) {
  using C = Cfg<NN>;
  if (gate && *gate == 0) return;
  __shared__ __align__(16) float2 lds[C::LDS_BYTES / 8];
  for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
    const int t = threadIdx.x;
    __syncthreads();   // the previous cell's exchange reads are done
    TL Lr[NN], Li[NN];
    const Cplx<TL>* pp = partial + (size_t)cell * S * NN * C::T;
    static_for<0, NN>([&](auto e) {
      const Cplx<TL> v = pp[e * C::T + t];
      Lr[e] = v.x;
      Li[e] = v.y;
    });
    gain_inverse_add<NN, TL>(Lr, Li, lds, t, out, cell, (t / (NN / 2)) * NN + t % (NN / 2));
  }
}

// ---- two pencils per thread ---------------------------------------------------
// The same computation with half the threads: thread t holds pencils
// p = t + s T2 (s = 0, 1; T2 = NN N / 2), so a workgroup is T2 / 64 waves,
// one per SIMD, and each lane may use the whole register file (VGPRs and
// AGPRs).  That leaves room to keep the L+ accumulator in registers across
// the nodes, so the only per-node traffic is the spectrum of r and K_j.
// Wave w owns the planes of its pencils in both slots; the exchanges below
// move both slots between one pair of barriers.

namespace {

template <int NN, typename T>
__device__ __forceinline__ void x_to_z_2(T (&vr)[2][NN], T (&vi)[2][NN], float2* lds, int t, int T2) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  static_for<0, 2>([&](auto s) {
    const int p = t + s * T2, kp = p / NN, y = p % NN;
    static_for<0, NN>([&](auto xx) {
      lds[(kp * NN + xx) * LD + y] = float2{float(vr[s][xx]), float(vi[s][xx])};
    });
  });
  __syncthreads();
  static_for<0, 2>([&](auto s) {
    const int p = t + s * T2, x = p / N, yp = p % N;
    static_for<0, KP>([&](auto k) {
      const float2 a = lds[(k * NN + x) * LD + yp];
      const float2 b = lds[(k * NN + x) * LD + yp + N];
      vr[s][k] = T(a.x); vi[s][k] = T(a.y);
      vr[s][N + k] = T(b.x); vi[s][N + k] = T(b.y);
    });
  });
}

template <int NN, typename T>
__device__ __forceinline__ void z_to_x_2(T (&vr)[2][NN], T (&vi)[2][NN], float2* lds, int t, int T2) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  __syncthreads();
  static_for<0, 2>([&](auto s) {
    const int p = t + s * T2, x = p / N, yp = p % N;
    static_for<0, KP>([&](auto k) {
      lds[(k * NN + x) * LD + yp] = float2{float(vr[s][k]), float(vi[s][k])};
      lds[(k * NN + x) * LD + yp + N] = float2{float(vr[s][N + k]), float(vi[s][N + k])};
    });
  });
  __syncthreads();
  static_for<0, 2>([&](auto s) {
    const int p = t + s * T2, kp = p / NN, y = p % NN;
    static_for<0, NN>([&](auto xx) {
      const float2 a = lds[(kp * NN + xx) * LD + y];
      vr[s][xx] = T(a.x);
      vi[s][xx] = T(a.y);
    });
  });
}

template <int NN>
__device__ __forceinline__ void x_to_z_2d(double (&vr)[2][NN], double (&vi)[2][NN], float2* lds, int t, int T2) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  double* ld = reinterpret_cast<double*>(lds);
  auto round = [&](double(&w)[2][NN]) {
    static_for<0, 2>([&](auto s) {
      const int p = t + s * T2, kp = p / NN, y = p % NN;
      static_for<0, NN>([&](auto xx) { ld[(kp * NN + xx) * LD + y] = w[s][xx]; });
    });
    __syncthreads();
    static_for<0, 2>([&](auto s) {
      const int p = t + s * T2, x = p / N, yp = p % N;
      static_for<0, KP>([&](auto k) {
        w[s][k] = ld[(k * NN + x) * LD + yp];
        w[s][N + k] = ld[(k * NN + x) * LD + yp + N];
      });
    });
  };
  round(vr);
  __syncthreads();   // every wave has read the real parts
  round(vi);
}

template <int NN>
__device__ __forceinline__ void z_to_x_2d(double (&vr)[2][NN], double (&vi)[2][NN], float2* lds, int t, int T2) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  double* ld = reinterpret_cast<double*>(lds);
  auto round = [&](double(&w)[2][NN]) {
    __syncthreads();
    static_for<0, 2>([&](auto s) {
      const int p = t + s * T2, x = p / N, yp = p % N;
      static_for<0, KP>([&](auto k) {
        ld[(k * NN + x) * LD + yp] = w[s][k];
        ld[(k * NN + x) * LD + yp + N] = w[s][N + k];
      });
    });
    __syncthreads();
    static_for<0, 2>([&](auto s) {
      const int p = t + s * T2, kp = p / NN, y = p % NN;
      static_for<0, NN>([&](auto xx) { w[s][xx] = ld[(kp * NN + xx) * LD + y]; });
    });
  };
  round(vr);
  round(vi);
}

// K_j rows of wave w's planes in both slots, and (wave 0) plane N, into the
// start of the wave's slot-0 plane region: [slot 0: PW planes][slot 1: PW
// planes][plane N], each plane P x P doubles.
template <int NN>
__device__ __forceinline__ void k_slice_dma_2(const double* Kj, float2* lds, int t, int T2) {
  constexpr int N = NN / 2, P = N + 1, PP = P * P, PW = 64 / NN, LD = NN + 1;
  const int wave = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64;
  float* dst = reinterpret_cast<float*>(lds + wave * PW * NN * LD);
  auto copy = [&](const float* src, float* d, int count) {
    for (int c = 0; c * 64 < count; ++c) {
      const int q = c * 64 + lane;
      if (q < count)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + q),
                                         (__attribute__((address_space(3))) void*)(d + c * 64), 4, 0, 0);
    }
  };
  copy(reinterpret_cast<const float*>(Kj + (size_t)wave * PW * PP), dst, PW * PP * 2);
  copy(reinterpret_cast<const float*>(Kj + (size_t)(wave * PW + T2 / NN) * PP), dst + PW * PP * 2, PW * PP * 2);
  if (wave == 0) copy(reinterpret_cast<const float*>(Kj + (size_t)N * PP), dst + 2 * PW * PP * 2, PP * 2);
}

}  // namespace

template <int NN>
__global__ void __launch_bounds__(Cfg<NN>::T / 2) k_fused2(
    const float* __restrict__ h, float* __restrict__ out, int batch, int Bc, const double* __restrict__ fac64,
    const double* __restrict__ pref64, const uint32_t* __restrict__ mask, const double* __restrict__ Kh,
    const float* __restrict__ nu, const float* __restrict__ Phi, const float* __restrict__ Om,
    double2* __restrict__ slots, int J, const int* __restrict__ gate) {
  using C = Cfg<NN>;
  if (gate && *gate == 0) return;   // a gated-off step of the device-resident GMRES
  constexpr int N = C::N, KP = C::KP, P = C::P, Q = C::Q, MW = C::MW, NP = NN * NN, PW = 64 / NN, LD = C::LD;
  constexpr int T2 = C::T / 2;
  __shared__ __align__(16) float2 lds[C::LDS_BYTES / 8];
  __shared__ double fs[9 * NN + 3];
  __shared__ float tab[Q];
  const int t0 = threadIdx.x;
  // Scratch slot of this workgroup: the spectrum of r (KP*NP complex double),
  // element i of pencil p at i*T + p.
  double2* Rs = slots + (size_t)blockIdx.x * (KP * NP);

  for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
    const int cc = Bc > 1 ? cell : 0;
    int t = t0;
    asm volatile("" : "+v"(t));
    const int ia = t % NN;                       // Y / X roles, both slots
    const int zyp = t % N;                       // Z role, both slots
    const int fx = ia <= N ? ia : NN - ia;
    __syncthreads();
    for (int i = t; i < 6 * NN; i += T2) fs[i] = fac64[(size_t)cc * 6 * NN + i];
    if (t < 2) fs[6 * NN + t] = pref64[2 * cc + t];
    for (int q = t; q < Q; q += T2) tab[q] = Om[q];
    __syncthreads();
    for (int i = t; i < 3 * NN; i += T2) fs[6 * NN + 2 + i] = 1.0 / fs[i];
    if (t == 0) fs[9 * NN + 2] = 1.0 / fs[6 * NN];
    __syncthreads();
    const double* ex = fs;
    const double* eh = fs + 3 * NN;
    const double prefM = fs[6 * NN], prefH = fs[6 * NN + 1];

    // ---------------- loss: U = iDFT[Omega DFT[h]] in float -------------------------
    {
      float fr[2][NN], fi[2][NN];
      static_for<0, 2>([&](auto s) {
        const int zx = (t + s * T2) / N;
        const float* h1 = h + ((size_t)cell * NP + zx * NN + zyp) * NN;
        const float* h2 = h1 + (size_t)N * NN;
        float zr[NN], zi[NN];
        static_for<0, NN>([&](auto z) { zr[z] = h1[z]; zi[z] = h2[z]; });
        z_forward<NN, float>(zr, zi, fr[s], fi[s]);
      });
      z_to_x_2<NN, float>(fr, fi, lds, t, T2);
      static_for<0, 2>([&](auto s) {
        const int p = t + s * T2, kp = p / NN;
        fft<NN, false>(fr[s], fi[s]);
        transpose_plane<NN, float>(fr[s], fi[s], lds, p);
        fft<NN, false>(fr[s], fi[s]);
        mode_multiply<NN, float>(fr[s], fi[s], p, [&](auto ky) {   // Omega(|k|^2) / n^3
          constexpr int fy = ky <= N ? ky : NN - ky;
          const int q = fx * fx + fy * fy;
          return float2{tab[q + kp * kp], tab[q + N * N]};
        });
        fft<NN, true>(fr[s], fi[s]);
        transpose_plane<NN, float>(fr[s], fi[s], lds, p);
        fft<NN, true>(fr[s], fi[s]);
      });
      x_to_z_2<NN, float>(fr, fi, lds, t, T2);
      static_for<0, 2>([&](auto s) {
        const int zx = (t + s * T2) / N, col1 = zx * NN + zyp;
        const float* h1 = h + ((size_t)cell * NP + col1) * NN;
        const float* h2 = h1 + (size_t)N * NN;
        float zr[NN], zi[NN];
        z_inverse<NN, float>(fr[s], fi[s], zr, zi);
        const float* n1 = nu + ((size_t)cc * NP + col1) * NN;
        const float* n2 = n1 + (size_t)N * NN;
        float* o1 = out + ((size_t)cell * NP + col1) * NN;
        float* o2 = o1 + (size_t)N * NN;
        const double mxy1 = prefM * ex[zx] * ex[NN + zyp], mxy2 = prefM * ex[zx] * ex[NN + zyp + N];
        static_for<0, NN>([&](auto z) {
          const double ez = ex[2 * NN + z];
          o1[z] = float(-(mxy1 * ez) * double(zr[z]) - double(n1[z]) * double(h1[z]));
          o2[z] = float(-(mxy2 * ez) * double(zi[z]) - double(n2[z]) * double(h2[z]));
        });
      });
    }
    // ---------------- R = DFT[chi h / M]: double arithmetic, double result --------
    {
      double vr[2][NN], vi[2][NN];
      static_for<0, 2>([&](auto s) {
        const int zx = (t + s * T2) / N, col1 = zx * NN + zyp;
        const float* h1 = h + ((size_t)cell * NP + col1) * NN;
        const float* h2 = h1 + (size_t)N * NN;
        const uint32_t* mk1 = mask + ((size_t)cc * NP + col1) * MW;
        const uint32_t* mk2 = mk1 + (size_t)N * MW;
        uint32_t b1[MW], b2[MW];
        static_for<0, MW>([&](auto w) { b1[w] = mk1[w]; b2[w] = mk2[w]; });
        const double* rx = fs + 6 * NN + 2;
        const double rxy = fs[9 * NN + 2] * rx[zx];
        const double r1 = rxy * rx[NN + zyp], r2 = rxy * rx[NN + zyp + N];
        double zr[NN], zi[NN];
        static_for<0, NN>([&](auto z) {
          const double rz = rx[2 * NN + z];
          const double q1 = double(h1[z]) * (r1 * rz), q2 = double(h2[z]) * (r2 * rz);
          zr[z] = ((b1[z / 32] >> (z % 32)) & 1u) ? q1 : 0.0;
          zi[z] = ((b2[z / 32] >> (z % 32)) & 1u) ? q2 : 0.0;
        });
        z_forward<NN, double>(zr, zi, vr[s], vi[s]);
      });
      z_to_x_2d<NN>(vr, vi, lds, t, T2);
      static_for<0, 2>([&](auto s) {
        const int p = t + s * T2;
        fft<NN, false>(vr[s], vi[s]);
        transpose_plane_d<NN>(vr[s], vi[s], lds, p);
        fft<NN, false>(vr[s], vi[s]);
        static_for<0, NN>([&](auto ky) { Rs[ky * C::T + p] = double2{vr[s][ky], vi[s][ky]}; });
      });
    }
    k_slice_dma_2<NN>(Kh + (size_t)cc * J * kh_stride(NN), lds, t, T2);   // K_0 into this wave's region

    // ---------------- gain loop: L+^ stays in registers -----------------------------
    float Lr[2][NN], Li[2][NN];
    static_for<0, 2>([&](auto s) {
      static_for<0, NN>([&](auto k) { Lr[s][k] = 0.f; Li[s][k] = 0.f; });
    });
    for (int j = 0; j < J; ++j) {
      asm volatile("" : "+v"(t));
      float fr[2][NN], fi[2][NN];
      {
        double vr[2][NN], vi[2][NN];
        static_for<0, 2>([&](auto s) {
          const int p = t + s * T2;
          static_for<0, NN>([&](auto ky) {
            const double2 v = Rs[ky * C::T + p];
            vr[s][ky] = v.x;
            vi[s][ky] = v.y;
          });
        });
        __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): this wave's copy of K_j has landed
        const double* Kw = reinterpret_cast<const double*>(lds + (t / 64) * PW * NN * LD);
        static_for<0, 2>([&](auto s) {
          const int p = t + s * T2, kw = (t % 64) / NN + s * PW;
          mode_multiply<NN, double>(vr[s], vi[s], p, [&](auto ky) {     // K_j / n^3
            constexpr int fy = ky <= N ? ky : NN - ky;
            return double2{Kw[(kw * P + fy) * P + fx], Kw[(2 * PW * P + fy) * P + fx]};
          });
        });
        static_for<0, 2>([&](auto s) {
          const int p = t + s * T2;
          fft<NN, true>(vr[s], vi[s]);
          transpose_plane_d<NN>(vr[s], vi[s], lds, p);
          fft<NN, true>(vr[s], vi[s]);
        });
        x_to_z_2d<NN>(vr, vi, lds, t, T2);
        // Every wave has used Phi_{j-1} by now: stream Phi_j into LDS while
        // the z stage runs.  It is complete and visible after the wait and
        // first barrier of the next X <- Z exchange.
        lds_dma(Phi + (size_t)j * phi_stride(NN), tab, Q, t, T2);
        static_for<0, 2>([&](auto s) {
          const int zx = (t + s * T2) / N;
          double zr[NN], zi[NN];
          z_inverse<NN, double>(vr[s], vi[s], zr, zi);
          const double hx = prefH * eh[zx];
          const double g1 = hx * eh[NN + zyp], g2 = hx * eh[NN + zyp + N];
          float qr[NN], qi[NN];
          static_for<0, NN>([&](auto z) {
            const double ez = eh[2 * NN + z];
            qr[z] = float(zr[z] * ez);
            qi[z] = float(zi[z] * ez);
          });
          z_forward<NN, float>(qr, qi, fr[s], fi[s], float(g1), float(g2));   // g1, g2 as in k_fused
        });
      }
      __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): this wave's table loads have landed
      z_to_x_2<NN, float>(fr, fi, lds, t, T2);
      static_for<0, 2>([&](auto s) {
        const int p = t + s * T2;
        fft<NN, false>(fr[s], fi[s]);
        transpose_plane<NN, float>(fr[s], fi[s], lds, p);
      });
      // This wave is done with its regions until the next node's K_j product;
      // its transpose reads complete (lgkmcnt(0)) before the copy may land.
      if (j + 1 < J) {
        __builtin_amdgcn_s_waitcnt(0xc07f);
        k_slice_dma_2<NN>(Kh + ((size_t)cc * J + j + 1) * kh_stride(NN), lds, t, T2);
      }
      static_for<0, 2>([&](auto s) {
        const int p = t + s * T2, kp = p / NN;
        fft<NN, false>(fr[s], fi[s]);
        mode_multiply<NN, float>(fr[s], fi[s], p, [&](auto ky) {       // Phi_j / n^3
          constexpr int fy = ky <= N ? ky : NN - ky;
          const int q = fx * fx + fy * fy;
          return float2{tab[q + kp * kp], tab[q + N * N]};
        });
        static_for<0, NN>([&](auto k) {
          Lr[s][k] += fr[s][k];
          Li[s][k] += fi[s][k];
        });
      });
    }
    // ---------------- L+ = iDFT[L+^], out += L+ -------------------------------------
    static_for<0, 2>([&](auto s) {
      const int p = t + s * T2;
      fft<NN, true>(Lr[s], Li[s]);
      transpose_plane<NN, float>(Lr[s], Li[s], lds, p);
      fft<NN, true>(Lr[s], Li[s]);
    });
    x_to_z_2<NN, float>(Lr, Li, lds, t, T2);
    static_for<0, 2>([&](auto s) {
      const int zx = (t + s * T2) / N, col1 = zx * NN + zyp;
      float zr[NN], zi[NN];
      z_inverse<NN, float>(Lr[s], Li[s], zr, zi);
      float* o1 = out + ((size_t)cell * NP + col1) * NN;
      float* o2 = o1 + (size_t)N * NN;
      static_for<0, NN>([&](auto z) {
        o1[z] = o1[z] + zr[z];
        o2[z] = o2[z] + zi[z];
      });
    });
  }
}

// F32 and F64 plans at n = 16 and 32 (dtype: 0 = F64, 1 = F32).
bool fused_supported(int n, int dtype) { return (dtype == 0 || dtype == 1) && (n == 16 || n == 32); }

size_t fused_scratch_bytes(int n, int nslots, int ppt, int dtype) {
  // per slot: R (complex double) and, with one pencil per thread, the L+
  // accumulator (complex float, or complex double for F64); with two pencils
  // (F32 only) it stays in registers
  const size_t acc = ppt == 2 ? 0 : dtype == 0 ? sizeof(double2) : sizeof(float2);
  return (size_t)nslots * (n / 2) * n * n * (sizeof(double2) + acc);
}

// Workgroups resident per compute unit: n = 32 needs all of a CU's LDS, the
// n = 16 workgroup (two waves, 22 KB of LDS, up to 256 registers) fits four
// times by registers.
int fused_max_per_cu(int n) { return n == 16 ? 4 : 1; }

int fused_slots(int n, int batch, int per_cu, int cus) {
  const int pc = per_cu > 0 && per_cu <= fused_max_per_cu(n) ? per_cu : fused_max_per_cu(n);
  const int slots = (cus > 0 ? cus : 256) * pc;
  return batch < slots ? batch : slots;
}

int fused_auto_split(int n, int J, int batch, int cus) {
  const int cu = cus > 0 ? cus : 256;
  const int c = cu * fused_max_per_cu(n);   // workgroups resident at once
  if (batch <= 0 || batch >= c) return 1;
  // At most one work item per resident workgroup: c / batch per cell, one of
  // them kept for the loss term where that leaves two parts or more (the
  // loss then runs beside the gain parts instead of before part 0's); two
  // parts without it only while that is still one item per compute unit.
  // The apply takes as long as its longest part, ceil(J / S) nodes: take the
  // fewest parts that reach the shortest longest part (measured on MI355X:
  // 16 cells at n = 32 run faster in 9 parts of at most 2 nodes than in 15;
  // 64 cells in 3 parts and the loss than in 4 parts without; 512 cells at
  // n = 16 unsplit).
  int smax = c / batch - 1;
  if (smax < 2) smax = 2 * batch <= cu ? 2 : 1;
  if (smax > J) smax = J;
  if (smax <= 1) return 1;
  const int per = (J + smax - 1) / smax;
  return (J + per - 1) / per;
}

int fused_loss_item(int n, int batch, int S, int cus) {
  return S > 1 && (long)batch * (S + 1) <= (long)(cus > 0 ? cus : 256) * fused_max_per_cu(n) ? 1 : 0;
}

size_t fused_partial_offset(int n, int nslots, int dtype) {
  return (fused_scratch_bytes(n, nslots, 1, dtype) + 255) / 256 * 256;
}

size_t fused_split_scratch_bytes(int n, int nslots, int batch, int S, int dtype) {
  const size_t cplx = dtype == 0 ? sizeof(double2) : sizeof(float2);
  return fused_partial_offset(n, nslots, dtype) + (size_t)batch * S * (n / 2) * n * n * cplx;
}

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the host-side name of a __device__ array is only a
// stand-in, never a device address).
namespace {
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64];
}  // namespace

hipError_t fused_noalloc_scratch(int device, void** ptr, size_t* bytes) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = p;
  }
  *ptr = g_noalloc_ptr[device];
  *bytes = NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

// Accumulator splits compiled for each plan type (chunks of two complex
// floats for F32, of one complex double for F64).
bool fused_keep_valid(int n, int dtype, int keep) {
  if (dtype == 1) return keep == 0 || keep == 4 || keep == 8 || (n == 32 && keep == 16);
  if (dtype == 0) return keep == 0 || (n == 32 && keep == 4) || keep == 8 || (n == 16 && keep == 16);
  return false;
}

int fused_default_keep(int n, int dtype) {
  if (dtype == 0) return n == 16 ? 16 : 0;
  return 8;
}

namespace {

template <int NN, int KA, typename TL>
void launch_fused(const ApplyCtx& c, int slots) {
  k_fused<NN, KA, TL><<<slots, Cfg<NN>::T, 0, c.stream>>>(
      static_cast<const TL*>(c.h), static_cast<TL*>(c.out), c.batch, c.Bc, c.fac64, c.pref64, c.mask,
      static_cast<const double*>(c.Kh), static_cast<const TL*>(c.nu), static_cast<const TL*>(c.Phi),
      static_cast<const TL*>(c.Om), static_cast<double2*>(c.R), c.J, c.gate);
}

template <int NN, int KA, typename TL>
void launch_fused_split(const ApplyCtx& c, int slots) {
  const int S = c.fused_split;
  Cplx<TL>* partial =
      reinterpret_cast<Cplx<TL>*>(static_cast<char*>(c.R) + fused_partial_offset(NN, slots, c.dtype));
  k_fused_split<NN, KA, TL><<<slots, Cfg<NN>::T, 0, c.stream>>>(
      static_cast<const TL*>(c.h), static_cast<TL*>(c.out), c.batch, c.Bc, c.fac64, c.pref64, c.mask,
      static_cast<const double*>(c.Kh), static_cast<const TL*>(c.nu), static_cast<const TL*>(c.Phi),
      static_cast<const TL*>(c.Om), static_cast<double2*>(c.R), c.J, S, fused_loss_item(NN, c.batch, S, c.cus),
      partial, c.gate);
  const long per_item = (long)NN * Cfg<NN>::T;
  const long blocks = ((long)c.batch * per_item + 255) / 256;
  const int sum_grid = (int)(blocks < 8L * c.cus ? blocks : 8L * c.cus);
  k_fused_sum<Cplx<TL>><<<sum_grid, 256, 0, c.stream>>>(partial, per_item, c.batch, S, c.gate);
  const int cells = c.batch < c.cus * fused_max_per_cu(NN) ? c.batch : c.cus * fused_max_per_cu(NN);
  k_fused_finish<NN, TL><<<cells, Cfg<NN>::T, 0, c.stream>>>(static_cast<TL*>(c.out), c.batch, partial, S, c.gate);
}

template <int NN, int KA, typename TL>
void launch_fused_any(const ApplyCtx& c, int slots) {
  if (c.fused_split > 1) launch_fused_split<NN, KA, TL>(c, slots);
  else launch_fused<NN, KA, TL>(c, slots);
}

template <int NN>
void launch_fused2(const ApplyCtx& c, int slots) {
  k_fused2<NN><<<slots, Cfg<NN>::T / 2, 0, c.stream>>>(
      static_cast<const float*>(c.h), static_cast<float*>(c.out), c.batch, c.Bc, c.fac64, c.pref64, c.mask,
      static_cast<const double*>(c.Kh), static_cast<const float*>(c.nu), static_cast<const float*>(c.Phi),
      static_cast<const float*>(c.Om), static_cast<double2*>(c.R), c.J, c.gate);
}

}  // namespace

hipError_t fused_apply(const ApplyCtx& c) {
  const int S = c.fused_split;
  if (!fused_supported(c.n, c.dtype) || !fused_keep_valid(c.n, c.dtype, c.fused_keep)) return hipErrorInvalidValue;
  if (c.fused_ppt == 2 && c.dtype != 1) return hipErrorInvalidValue;
  if (S < 1 || S > c.J || (S > 1 && c.fused_ppt != 1)) return hipErrorInvalidValue;
  // the kernels are persistent over their work items (cells, or cell parts)
  int slots = fused_slots(c.n, S > 1 ? c.batch * (S + fused_loss_item(c.n, c.batch, S, c.cus)) : c.batch, c.per_cu,
                          c.cus);
  if (c.max_slots > 0 && slots > c.max_slots) slots = c.max_slots;
  const int k = c.fused_keep;
  if (c.dtype == 1) {
    if (c.n == 16) {
      if (c.fused_ppt == 2) launch_fused2<16>(c, slots);
      else if (k == 0) launch_fused_any<16, 0, float>(c, slots);
      else if (k == 4) launch_fused_any<16, 4, float>(c, slots);
      else launch_fused_any<16, 8, float>(c, slots);
    } else {
      if (c.fused_ppt == 2) launch_fused2<32>(c, slots);
      else if (k == 0) launch_fused_any<32, 0, float>(c, slots);
      else if (k == 4) launch_fused_any<32, 4, float>(c, slots);
      else if (k == 8) launch_fused_any<32, 8, float>(c, slots);
      else launch_fused_any<32, 16, float>(c, slots);
    }
  } else {
    if (c.n == 16) {
      if (k == 0) launch_fused_any<16, 0, double>(c, slots);
      else if (k == 8) launch_fused_any<16, 8, double>(c, slots);
      else launch_fused_any<16, 16, double>(c, slots);
    } else {
      if (k == 0) launch_fused_any<32, 0, double>(c, slots);
      else if (k == 4) launch_fused_any<32, 4, double>(c, slots);
      else launch_fused_any<32, 8, double>(c, slots);
    }
  }
  return hipGetLastError();
}

}  // namespace lincoll
