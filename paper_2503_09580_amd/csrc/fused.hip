// Fused persistent kernel: one workgroup per cell (looping over cells), the
// whole of Algorithm 1 on chip except the FP64 spectrum of r, which streams
// from a per-workgroup scratch slot (L2 / Infinity-cache resident).
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
// Transposes between roles go through LDS.
//
// Precision (FP32 storage at the HBM boundary): every butterfly runs in
// double.  The spectrum of r = chi h / M and the inverse transforms that
// produce psi_j keep double storage as well: r is large where M is small and
// any rounding of its spectral or partially transformed values spreads that
// size over the whole box (Sec. 3.3).  After the product with M^h the data
// is concentrated where M is not small and float storage suffices.
#include "fft.h"
#include "internal.h"

namespace lincoll {

namespace {

template <typename S> struct V2f;
template <> struct V2f<float> { using t = float2; };
template <> struct V2f<double> { using t = double2; };

template <int NN>
struct Cfg {
  static constexpr int N = NN / 2;
  static constexpr int KP = N;                 // packed planes
  static constexpr int T = NN * N;             // threads
  static constexpr int P = N + 1;
  static constexpr int Q = 3 * N * N + 1;
  static constexpr int MW = (NN + 31) / 32;
  static constexpr int LD = NN + 1;            // padded LDS row
  // LDS transpose buffer: one full volume of float2 (KP * NN * LD * 8 B)
  static constexpr int LDS_BYTES = KP * NN * LD * 8;
  // rounds needed to move a double volume through it
  static constexpr int R64 = 2;
};

__device__ __forceinline__ int foldk(int K, int NN) { return K <= NN / 2 ? K : NN - K; }

// ---- z stage: two real columns <-> their packed half spectra ------------------
// forward: a, b real (as zr, zi) -> s1[k], s2[k], k < N, with bin 0 holding
// (A(0), A(N)) and bins 1..N-1 the complex A(k).
template <int NN, typename T>
__device__ __forceinline__ void z_forward(T (&zr)[NN], T (&zi)[NN], T (&s1r)[NN / 2], T (&s1i)[NN / 2],
                                          T (&s2r)[NN / 2], T (&s2i)[NN / 2]) {
  constexpr int N = NN / 2;
  fft<NN, false>(zr, zi);
  T Ar[N + 1], Ai[N + 1], Br[N + 1], Bi[N + 1];
  split_real_pair<NN>(zr, zi, Ar, Ai, Br, Bi);
  s1r[0] = Ar[0];
  s1i[0] = Ar[N];
  s2r[0] = Br[0];
  s2i[0] = Br[N];
  static_for<1, N>([&](auto k) {
    s1r[k] = Ar[k];
    s1i[k] = Ai[k];
    s2r[k] = Br[k];
    s2i[k] = Bi[k];
  });
}

template <int NN, typename T>
__device__ __forceinline__ void z_inverse(const T (&s1r)[NN / 2], const T (&s1i)[NN / 2], const T (&s2r)[NN / 2],
                                          const T (&s2i)[NN / 2], T (&zr)[NN], T (&zi)[NN]) {
  constexpr int N = NN / 2;
  T Ar[N + 1], Ai[N + 1], Br[N + 1], Bi[N + 1];
  Ar[0] = s1r[0]; Ai[0] = T(0); Ar[N] = s1i[0]; Ai[N] = T(0);
  Br[0] = s2r[0]; Bi[0] = T(0); Br[N] = s2i[0]; Bi[N] = T(0);
  static_for<1, N>([&](auto k) {
    Ar[k] = s1r[k]; Ai[k] = s1i[k];
    Br[k] = s2r[k]; Bi[k] = s2i[k];
  });
  join_real_pair<NN>(Ar, Ai, Br, Bi, zr, zi);
  fft<NN, true>(zr, zi);
}

// ---- transposes through LDS ---------------------------------------------------
// Within each plane kp: thread (kp, i) holds v[j] = element (i, j); afterwards
// it holds v[j] = element (j, i).  S is the LDS storage type; ROUNDS splits
// the planes into groups when a volume of S does not fit the buffer.
template <int NN, int ROUNDS, typename S, typename T>
__device__ __forceinline__ void transpose_plane(T (&vr)[NN], T (&vi)[NN], void* ldsv, int t) {
  using S2 = typename V2f<S>::t;
  constexpr int KP = NN / 2, LD = NN + 1, KPR = KP / ROUNDS;
  S2* lds = static_cast<S2*>(ldsv);
  const int kp = t / NN, i = t % NN;
  static_for<0, ROUNDS>([&](auto r) {
    const bool mine = (kp / KPR) == r;
    const int kl = kp % KPR;
    if (mine) static_for<0, NN>([&](auto j) { lds[(kl * NN + i) * LD + j] = S2{S(vr[j]), S(vi[j])}; });
    __syncthreads();
    if (mine)
      static_for<0, NN>([&](auto j) {
        const S2 v = lds[(kl * NN + j) * LD + i];
        vr[j] = T(v.x);
        vi[j] = T(v.y);
      });
    __syncthreads();
  });
}

// X role (kp, y) holding v[x]  ->  Z role (x, yp) holding s1[kp] = (kp, x, yp),
// s2[kp] = (kp, x, yp + N).  The same registers are reused: v and (s1, s2)
// are two views of NN complex values.
template <int NN, int ROUNDS, typename S, typename T>
__device__ __forceinline__ void x_to_z(T (&vr)[NN], T (&vi)[NN], void* ldsv, int t) {
  using S2 = typename V2f<S>::t;
  constexpr int N = NN / 2, KP = N, LD = NN + 1, XR = NN / ROUNDS;
  S2* lds = static_cast<S2*>(ldsv);
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  T o1r[N], o1i[N], o2r[N], o2i[N];
  static_for<0, ROUNDS>([&](auto r) {
    static_for<0, XR>([&](auto xl) {
      lds[(kp * XR + xl) * LD + y] = S2{S(vr[r * XR + xl]), S(vi[r * XR + xl])};
    });
    __syncthreads();
    if (x / XR == r) {
      const int xl = x % XR;
      static_for<0, KP>([&](auto k) {
        const S2 a = lds[(k * XR + xl) * LD + yp];
        const S2 b = lds[(k * XR + xl) * LD + yp + N];
        o1r[k] = T(a.x); o1i[k] = T(a.y);
        o2r[k] = T(b.x); o2i[k] = T(b.y);
      });
    }
    __syncthreads();
  });
  static_for<0, N>([&](auto k) {
    vr[k] = o1r[k]; vi[k] = o1i[k];
    vr[N + k] = o2r[k]; vi[N + k] = o2i[k];
  });
}

// Z role -> X role (inverse of x_to_z), one round of float storage.
template <int NN, typename S, typename T>
__device__ __forceinline__ void z_to_x(T (&vr)[NN], T (&vi)[NN], void* ldsv, int t) {
  using S2 = typename V2f<S>::t;
  constexpr int N = NN / 2, KP = N, LD = NN + 1;
  S2* lds = static_cast<S2*>(ldsv);
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  static_for<0, KP>([&](auto k) {
    lds[(k * NN + x) * LD + yp] = S2{S(vr[k]), S(vi[k])};
    lds[(k * NN + x) * LD + yp + N] = S2{S(vr[N + k]), S(vi[N + k])};
  });
  __syncthreads();
  static_for<0, NN>([&](auto xx) {
    const S2 a = lds[(kp * NN + xx) * LD + y];
    vr[xx] = T(a.x);
    vi[xx] = T(a.y);
  });
  __syncthreads();
}

// Z role -> X role for double storage, two rounds over the halves of x.
template <int NN>
__device__ __forceinline__ void z_to_x64(double (&vr)[NN], double (&vi)[NN], void* ldsv, int t) {
  constexpr int N = NN / 2, KP = N, LD = NN + 1, XR = NN / 2;
  double2* lds = static_cast<double2*>(ldsv);
  const int kp = t / NN, y = t % NN;
  const int x = t / N, yp = t % N;
  double orr[NN], oi[NN];
  static_for<0, 2>([&](auto r) {
    if (x / XR == r) {
      const int xl = x % XR;
      static_for<0, KP>([&](auto k) {
        lds[(k * XR + xl) * LD + yp] = double2{vr[k], vi[k]};
        lds[(k * XR + xl) * LD + yp + N] = double2{vr[N + k], vi[N + k]};
      });
    }
    __syncthreads();
    static_for<0, XR>([&](auto xl) {
      const double2 a = lds[(kp * XR + xl) * LD + y];
      orr[r * XR + xl] = a.x;
      oi[r * XR + xl] = a.y;
    });
    __syncthreads();
  });
  static_for<0, NN>([&](auto i) { vr[i] = orr[i]; vi[i] = oi[i]; });
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
        const T s = packed ? T(0.5) * (m.x + m.y) : m.x;
        const T d = packed ? T(0.5) * (m.x - m.y) : T(0);
        const T nr = s * vr[j] + d * ar, ni = s * vi[j] - d * ai;
        vr[j] = nr;
        vi[j] = ni;
      }
      if constexpr (jm != j) {
        const auto m = getm(std::integral_constant<int, jm>{});
        const T s = packed ? T(0.5) * (m.x + m.y) : m.x;
        const T d = packed ? T(0.5) * (m.x - m.y) : T(0);
        const T nr = s * vr[jm] + d * br, ni = s * vi[jm] - d * bi;
        vr[jm] = nr;
        vi[jm] = ni;
      }
    });
  } else {
    static_for<0, NN>([&](auto j) {
      const T m = getm(j).x;
      vr[j] *= m;
      vi[j] *= m;
    });
  }
}

}  // namespace

template <int NN>
__global__ void __launch_bounds__(Cfg<NN>::T) k_fused(
    const float* __restrict__ h, float* __restrict__ out, int batch, int Bc, const double* __restrict__ fac64,
    const double* __restrict__ pref64, const uint32_t* __restrict__ mask, const float* __restrict__ Kh,
    const float* __restrict__ nu, const float* __restrict__ Phi, const float* __restrict__ Om,
    double2* __restrict__ scratch, int J) {
  using C = Cfg<NN>;
  constexpr int N = C::N, KP = C::KP, P = C::P, Q = C::Q, MW = C::MW, NP = NN * NN, P3 = P * P * P;
  __shared__ __align__(16) unsigned char lds_raw[C::LDS_BYTES];
  __shared__ double fs[6 * NN + 2];
  __shared__ float tab[Q];
  __shared__ float Ks[P3];
  void* lds = lds_raw;
  const int t = threadIdx.x;
  const int kp = t / NN, ia = t % NN;          // Y / X roles
  const int zx = t / N, zyp = t % N;           // Z role
  const int fx = ia <= N ? ia : NN - ia;
  double2* Rs = scratch + (size_t)blockIdx.x * KP * NP;

  for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
    const int cc = Bc > 1 ? cell : 0;
    __syncthreads();
    for (int i = t; i < 6 * NN; i += C::T) fs[i] = fac64[(size_t)cc * 6 * NN + i];
    if (t < 2) fs[6 * NN + t] = pref64[2 * cc + t];
    for (int q = t; q < Q; q += C::T) tab[q] = Om[q];
    __syncthreads();
    const double* ex = fs;
    const double* eh = fs + 3 * NN;
    const double prefM = fs[6 * NN], prefH = fs[6 * NN + 1];
    const int col1 = zx * NN + zyp;
    const float* h1 = h + ((size_t)cell * NP + col1) * NN;
    const float* h2 = h1 + (size_t)N * NN;
    const double mxy1 = prefM * ex[zx] * ex[NN + zyp], mxy2 = prefM * ex[zx] * ex[NN + zyp + N];

    // ---------------- loss: U = iDFT[Omega DFT[h]] in float -------------------------
    {
      float fr[NN], fi[NN];
      {
        float zr[NN], zi[NN];
        static_for<0, NN>([&](auto z) { zr[z] = h1[z]; zi[z] = h2[z]; });
        float a1r[N], a1i[N], a2r[N], a2i[N];
        z_forward<NN, float>(zr, zi, a1r, a1i, a2r, a2i);
        static_for<0, N>([&](auto k) { fr[k] = a1r[k]; fi[k] = a1i[k]; fr[N + k] = a2r[k]; fi[N + k] = a2i[k]; });
      }
      z_to_x<NN, float, float>(fr, fi, lds, t);
      fft<NN, false>(fr, fi);
      transpose_plane<NN, 1, float, float>(fr, fi, lds, t);
      fft<NN, false>(fr, fi);
      mode_multiply<NN, float>(fr, fi, t, [&](auto ky) {   // Omega(|k|^2) / n^3
        constexpr int fy = ky <= N ? ky : NN - ky;
        const int q = fx * fx + fy * fy;
        return float2{tab[q + kp * kp], tab[q + N * N]};
      });
      fft<NN, true>(fr, fi);
      transpose_plane<NN, 1, float, float>(fr, fi, lds, t);
      fft<NN, true>(fr, fi);
      x_to_z<NN, 1, float, float>(fr, fi, lds, t);
      float s1r[N], s1i[N], s2r[N], s2i[N], zr[NN], zi[NN];
      static_for<0, N>([&](auto k) { s1r[k] = fr[k]; s1i[k] = fi[k]; s2r[k] = fr[N + k]; s2i[k] = fi[N + k]; });
      z_inverse<NN, float>(s1r, s1i, s2r, s2i, zr, zi);
      const float* n1 = nu + ((size_t)cc * NP + col1) * NN;
      const float* n2 = n1 + (size_t)N * NN;
      float* o1 = out + ((size_t)cell * NP + col1) * NN;
      float* o2 = o1 + (size_t)N * NN;
      static_for<0, NN>([&](auto z) {
        const double ez = ex[2 * NN + z];
        o1[z] = float(-(mxy1 * ez) * double(zr[z]) - double(n1[z]) * double(h1[z]));
        o2[z] = float(-(mxy2 * ez) * double(zi[z]) - double(n2[z]) * double(h2[z]));
      });
    }
    // ---------------- R = DFT[chi h / M] in double ------------------------------
    {
      double vr[NN], vi[NN];
      {
        const uint32_t* mk1 = mask + ((size_t)cc * NP + col1) * MW;
        const uint32_t* mk2 = mk1 + (size_t)N * MW;
        uint32_t b1[MW], b2[MW];
        static_for<0, MW>([&](auto w) { b1[w] = mk1[w]; b2[w] = mk2[w]; });
        double zr[NN], zi[NN];
        static_for<0, NN>([&](auto z) {
          const double ez = ex[2 * NN + z];
          zr[z] = ((b1[z / 32] >> (z % 32)) & 1u) ? double(h1[z]) / (mxy1 * ez) : 0.0;
          zi[z] = ((b2[z / 32] >> (z % 32)) & 1u) ? double(h2[z]) / (mxy2 * ez) : 0.0;
        });
        double a1r[N], a1i[N], a2r[N], a2i[N];
        z_forward<NN, double>(zr, zi, a1r, a1i, a2r, a2i);
        static_for<0, N>([&](auto k) { vr[k] = a1r[k]; vi[k] = a1i[k]; vr[N + k] = a2r[k]; vi[N + k] = a2i[k]; });
      }
      z_to_x64<NN>(vr, vi, lds, t);
      fft<NN, false>(vr, vi);
      transpose_plane<NN, C::R64, double, double>(vr, vi, lds, t);
      fft<NN, false>(vr, vi);
      // store R: [kp][ky][kx], lanes along kx
      static_for<0, NN>([&](auto ky) { Rs[((size_t)kp * NN + ky) * NN + ia] = double2{vr[ky], vi[ky]}; });
    }

    // ---------------- gain loop ---------------------------------------------------
    float Lr[NN], Li[NN];
    static_for<0, NN>([&](auto ky) { Lr[ky] = 0.f; Li[ky] = 0.f; });
    for (int j = 0; j < J; ++j) {
      __syncthreads();
      for (int q = t; q < Q; q += C::T) tab[q] = Phi[(size_t)j * Q + q];
      {
        const float* Kj = Kh + ((size_t)cc * J + j) * P3;
        for (int q = t; q < P3; q += C::T) Ks[q] = Kj[q];
      }
      __syncthreads();
      float fr[NN], fi[NN];
      {
        double vr[NN], vi[NN];
        static_for<0, NN>([&](auto ky) {
          const double2 v = Rs[((size_t)kp * NN + ky) * NN + ia];
          vr[ky] = v.x;
          vi[ky] = v.y;
        });
        mode_multiply<NN, double>(vr, vi, t, [&](auto ky) {     // K_j / n^3
          constexpr int fy = ky <= N ? ky : NN - ky;
          return double2{double(Ks[(kp * P + fy) * P + fx]), double(Ks[(N * P + fy) * P + fx])};
        });
        fft<NN, true>(vr, vi);
        transpose_plane<NN, C::R64, double, double>(vr, vi, lds, t);
        fft<NN, true>(vr, vi);
        x_to_z<NN, C::R64, double, double>(vr, vi, lds, t);
        // psi on the two columns, times M^h; float from here on
        double s1r[N], s1i[N], s2r[N], s2i[N], zr[NN], zi[NN];
        static_for<0, N>([&](auto k) { s1r[k] = vr[k]; s1i[k] = vi[k]; s2r[k] = vr[N + k]; s2i[k] = vi[N + k]; });
        z_inverse<NN, double>(s1r, s1i, s2r, s2i, zr, zi);
        const double hx = prefH * eh[zx];
        const double g1 = hx * eh[NN + zyp], g2 = hx * eh[NN + zyp + N];
        float qr[NN], qi[NN];
        static_for<0, NN>([&](auto z) {
          const double ez = eh[2 * NN + z];
          qr[z] = float(zr[z] * (g1 * ez));
          qi[z] = float(zi[z] * (g2 * ez));
        });
        float t1r[N], t1i[N], t2r[N], t2i[N];
        z_forward<NN, float>(qr, qi, t1r, t1i, t2r, t2i);
        static_for<0, N>([&](auto k) { fr[k] = t1r[k]; fi[k] = t1i[k]; fr[N + k] = t2r[k]; fi[N + k] = t2i[k]; });
      }
      z_to_x<NN, float, float>(fr, fi, lds, t);
      fft<NN, false>(fr, fi);
      transpose_plane<NN, 1, float, float>(fr, fi, lds, t);
      fft<NN, false>(fr, fi);
      mode_multiply<NN, float>(fr, fi, t, [&](auto ky) {       // Phi_j / n^3
        constexpr int fy = ky <= N ? ky : NN - ky;
        const int q = fx * fx + fy * fy;
        return float2{tab[q + kp * kp], tab[q + N * N]};
      });
      static_for<0, NN>([&](auto ky) {
        Lr[ky] += fr[ky];
        Li[ky] += fi[ky];
      });
    }
    // ---------------- L+ = iDFT[L+^], out += L+ -------------------------------------
    fft<NN, true>(Lr, Li);
    transpose_plane<NN, 1, float, float>(Lr, Li, lds, t);
    fft<NN, true>(Lr, Li);
    x_to_z<NN, 1, float, float>(Lr, Li, lds, t);
    {
      float s1r[N], s1i[N], s2r[N], s2i[N], zr[NN], zi[NN];
      static_for<0, N>([&](auto k) { s1r[k] = Lr[k]; s1i[k] = Li[k]; s2r[k] = Lr[N + k]; s2i[k] = Li[N + k]; });
      z_inverse<NN, float>(s1r, s1i, s2r, s2i, zr, zi);
      float* o1 = out + ((size_t)cell * NP + col1) * NN;
      float* o2 = o1 + (size_t)N * NN;
      static_for<0, NN>([&](auto z) {
        o1[z] = o1[z] + zr[z];
        o2[z] = o2[z] + zi[z];
      });
    }
  }
}

bool fused_supported(int n, int dtype) { return dtype == 1 && (n == 16 || n == 32); }


size_t fused_scratch_bytes(int n, int nslots) {
  return (size_t)nslots * (n / 2) * n * n * sizeof(double2);
}

int fused_slots(int n, int batch) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int per_cu = n == 16 ? 4 : 1;
  const int slots = cus * per_cu;
  return batch < slots ? batch : slots;
}

hipError_t fused_apply(const ApplyCtx& c) {
  const int slots = fused_slots(c.n, c.batch);
  const float* h = static_cast<const float*>(c.h);
  float* out = static_cast<float*>(c.out);
  const double* fac64 = c.fac64;
  const double* pref64 = c.pref64;
  const float* Kh = static_cast<const float*>(c.Kh);
  const float* nu = static_cast<const float*>(c.nu);
  const float* Phi = static_cast<const float*>(c.Phi);
  const float* Om = static_cast<const float*>(c.Om);
  double2* scr = static_cast<double2*>(c.R);
  switch (c.n) {
    case 16:
      k_fused<16><<<slots, Cfg<16>::T, 0, c.stream>>>(h, out, c.batch, c.Bc, fac64, pref64, c.mask, Kh, nu, Phi, Om,
                                                       scr, c.J);
      break;
    case 32:
      k_fused<32><<<slots, Cfg<32>::T, 0, c.stream>>>(h, out, c.batch, c.Bc, fac64, pref64, c.mask, Kh, nu, Phi, Om,
                                                       scr, c.J);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lincoll
