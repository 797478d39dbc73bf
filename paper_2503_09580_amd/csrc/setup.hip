// Per-cell FP64 setup (Algorithm 1, the per-Maxwellian quantities) and the
// invariant projection.
#include <cmath>

#include "internal.h"

namespace lincoll {

hipError_t nu_chunk_dispatch(int n, const double* fac64, const double* pref64, const double* Om64, double2* planes,
                             double* nu64, int ncell, hipStream_t s);

// One block per cell.  Writes
//   fac64[c][0..2][i] = exp(-(v_i - u_d)^2 / (2 theta))   (M = pref[0] * product)
//   fac64[c][3..5][i] = exp(-(v_i - u_d)^2 / theta)       (M^h = pref[1] * product)
//   pref64[c] = {rho (2 pi theta)^-3/2, rho (pi theta)^-3/2}
//   gfac64[c][d] = exp(-(d h_v)^2 / theta), d = 0..n/2   (G = pref[1] * product, eq. (24))
//   mask bits: M/rho >= eps (eq. (25)), decided in FP64
//   Ainv: inverse Gram matrix of {1, v1, v2, v3, |v|^2} under M (projection)
__global__ void __launch_bounds__(256) k_cell_setup(const double* __restrict__ params, int n, double L, double eps,
                                                     double* __restrict__ fac64, double* __restrict__ pref64,
                                                     double* __restrict__ gfac64, uint32_t* __restrict__ mask,
                                                     double* __restrict__ Ainv) {
  const int c = blockIdx.x;
  const double rho = params[5 * c], th = params[5 * c + 4];
  const double u[3] = {params[5 * c + 1], params[5 * c + 2], params[5 * c + 3]};
  const double hv = 2.0 * L / n;
  const int N = n / 2, MW = (n + 31) / 32;
  double* f = fac64 + (size_t)c * 6 * n;
  for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) {
    const int d = t / n, i = t % n;
    const double dv = -L + i * hv - u[d];
    f[d * n + i] = exp(-dv * dv / (2.0 * th));
    f[(3 + d) * n + i] = exp(-dv * dv / th);
  }
  const double pm = pow(2.0 * M_PI * th, -1.5);
  if (threadIdx.x == 0) {
    pref64[2 * c] = rho * pm;
    pref64[2 * c + 1] = rho * pow(M_PI * th, -1.5);
  }
  for (int d = threadIdx.x; d <= N; d += blockDim.x) gfac64[(size_t)c * (N + 1) + d] = exp(-(d * hv) * (d * hv) / th);
  for (int col = threadIdx.x; col < n * n; col += blockDim.x) {
    const int x = col / n, y = col % n;
    const double dx = -L + x * hv - u[0], dy = -L + y * hv - u[1];
    for (int w = 0; w < MW; ++w) {
      uint32_t bits = 0;
      for (int b = 0; b < 32 && 32 * w + b < n; ++b) {
        const int z = 32 * w + b;
        const double dz = -L + z * hv - u[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        const bool keep = eps <= 0.0 || pm * exp(-d2 / (2.0 * th)) >= eps;
        bits |= (keep ? 1u : 0u) << b;
      }
      mask[((size_t)c * n * n + col) * MW + w] = bits;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // 1-D moments mk[d][p] = sum_i ex_d[i] v_i^p, p = 0..4
    double mk[3][5];
    for (int d = 0; d < 3; ++d)
      for (int p = 0; p < 5; ++p) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
          const double v = -L + i * hv;
          double vp = 1.0;
          for (int q = 0; q < p; ++q) vp *= v;
          s += f[d * n + i] * vp;
        }
        mk[d][p] = s;
      }
    // sum over the grid of M * monomial(a, b, c) = pref * mk0[a] mk1[b] mk2[c]
    auto mom = [&](int a, int b, int e) { return rho * pm * mk[0][a] * mk[1][b] * mk[2][e]; };
    // basis phi: 1, v1, v2, v3, |v|^2 written as sums of monomials (a,b,c)
    double A[5][10];
    const int ex[5][3][3] = {{{0, 0, 0}, {-1, 0, 0}, {-1, 0, 0}},
                             {{1, 0, 0}, {-1, 0, 0}, {-1, 0, 0}},
                             {{0, 1, 0}, {-1, 0, 0}, {-1, 0, 0}},
                             {{0, 0, 1}, {-1, 0, 0}, {-1, 0, 0}},
                             {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}}};
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b) {
        double s = 0.0;
        for (int ta = 0; ta < 3; ++ta) {
          if (ex[a][ta][0] < 0) continue;
          for (int tb = 0; tb < 3; ++tb) {
            if (ex[b][tb][0] < 0) continue;
            s += mom(ex[a][ta][0] + ex[b][tb][0], ex[a][ta][1] + ex[b][tb][1], ex[a][ta][2] + ex[b][tb][2]);
          }
        }
        A[a][b] = s;
        A[a][5 + b] = (a == b) ? 1.0 : 0.0;
      }
    // Gauss-Jordan with partial pivoting
    for (int col = 0; col < 5; ++col) {
      int piv = col;
      for (int r = col + 1; r < 5; ++r)
        if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
      if (piv != col)
        for (int k = 0; k < 10; ++k) {
          const double t = A[col][k];
          A[col][k] = A[piv][k];
          A[piv][k] = t;
        }
      const double inv = 1.0 / A[col][col];
      for (int k = 0; k < 10; ++k) A[col][k] *= inv;
      for (int r = 0; r < 5; ++r) {
        if (r == col) continue;
        const double fct = A[r][col];
        for (int k = 0; k < 10; ++k) A[r][k] -= fct * A[col][k];
      }
    }
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b) Ainv[(size_t)c * 25 + 5 * a + b] = A[a][5 + b];
  }
}

// One pass of the folded DFT of the even kernel G phi_j over the octant:
// in [cell][j][a][b][c] -> out [cell][j][b][c][ka], transform along a.
// FIRST: input is G(a,b,c) phi_j(a,b,c) built on the fly.
// LAST: output scaled by 1/n^3 and stored in the apply dtype T.
template <int P, bool FIRST, bool LAST, typename T>
__global__ void __launch_bounds__(256) k_kh_pass(const double* __restrict__ in, void* __restrict__ outv,
                                                  const double* __restrict__ phi, const double* __restrict__ gfac,
                                                  const double* __restrict__ pref64, const double* __restrict__ Cm,
                                                  int J, int ncell, double scale) {
  constexpr int P2 = P * P, P3 = P * P * P;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)ncell * J * P2) return;
  const int cj = (int)(gid / P2), bc = (int)(gid % P2);
  const int cell = cj / J, j = cj % J;
  const int b = bc / P, c = bc % P;
  double acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = 0.0;
  const double* g = gfac + (size_t)cell * P;
  const double gbc = FIRST ? pref64[2 * cell + 1] * g[b] * g[c] : 0.0;
  for (int a = 0; a < P; ++a) {
    double x;
    if (FIRST) {
      x = gbc * g[a] * phi[(size_t)j * P3 + (size_t)a * P2 + bc];
    } else {
      x = in[(size_t)cj * P3 + (size_t)a * P2 + bc];
    }
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] += Cm[k * P + a] * x;
  }
  if (LAST) {
    T* out = static_cast<T*>(outv) + (size_t)cj * kh_stride(2 * (P - 1)) + (size_t)bc * P;
#pragma unroll
    for (int k = 0; k < P; ++k) out[k] = static_cast<T>(acc[k] * scale);
  } else {
    double* out = static_cast<double*>(outv) + (size_t)cj * P3 + (size_t)bc * P;
#pragma unroll
    for (int k = 0; k < P; ++k) out[k] = acc[k];
  }
}

template <typename T>
__global__ void k_convert(const double* __restrict__ in, T* __restrict__ out, long count) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = static_cast<T>(in[i]);
}

template <int P, typename T>
static hipError_t kh_chunk(const SetupCtx& c, int c0, int nc) {
  const long threads = (long)nc * c.J * P * P;
  const dim3 grid((unsigned)((threads + 255) / 256));
  const double scale = 1.0 / ((double)c.n * c.n * c.n);
  const double* gf = c.gfac64 + (size_t)c0 * P;
  const double* pr = c.pref64 + (size_t)c0 * 2;
  T* Kh = static_cast<T*>(c.Kh) + (size_t)c0 * c.J * kh_stride(c.n);
  k_kh_pass<P, true, false, T><<<grid, 256, 0, c.stream>>>(nullptr, c.tmpA, c.phi, gf, pr, c.Cdct, c.J, nc, 1.0);
  k_kh_pass<P, false, false, T><<<grid, 256, 0, c.stream>>>(c.tmpA, c.tmpB, c.phi, gf, pr, c.Cdct, c.J, nc, 1.0);
  k_kh_pass<P, false, true, T><<<grid, 256, 0, c.stream>>>(c.tmpB, Kh, c.phi, gf, pr, c.Cdct, c.J, nc, scale);
  return hipGetLastError();
}

template <typename T>
static hipError_t kh_dispatch(const SetupCtx& c, int c0, int nc) {
  switch (c.n / 2 + 1) {
    case 5: return kh_chunk<5, T>(c, c0, nc);
    case 9: return kh_chunk<9, T>(c, c0, nc);
    case 17: return kh_chunk<17, T>(c, c0, nc);
    case 33: return kh_chunk<33, T>(c, c0, nc);
  }
  return hipErrorInvalidValue;
}

hipError_t setup_cells(const SetupCtx& c) {
  const int n = c.n, P = n / 2 + 1;
  k_cell_setup<<<c.Bc, 256, 0, c.stream>>>(c.params, n, c.L, c.eps, c.fac64, c.pref64, c.gfac64, c.mask, c.Ainv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long nf = (long)c.Bc * 6 * n, np = (long)c.Bc * 2;
  if (c.dtype != 0) {
    k_convert<float><<<(unsigned)((nf + 255) / 256), 256, 0, c.stream>>>(c.fac64, static_cast<float*>(c.facT), nf);
    k_convert<float><<<(unsigned)((np + 255) / 256), 256, 0, c.stream>>>(c.pref64, static_cast<float*>(c.prefT), np);
  }
  for (int c0 = 0; c0 < c.Bc; c0 += c.chunk) {
    const int nc = c.Bc - c0 < c.chunk ? c.Bc - c0 : c.chunk;
    // K_j is kept in double for every dtype: its product with the spectrum of
    // r (large where M is small, Sec. 3.3) turns a float rounding of K_j into
    // an error of about 1e-5 of the result.
    e = kh_dispatch<double>(c, c0, nc);
    if (e != hipSuccess) return e;
    // nu in FP64 for this chunk, written to tmpA (n^3 doubles per cell fit:
    // J P^3 >= n^3 for every supported n), then stored in the apply dtype
    double* nu64 = c.dtype == 0 ? static_cast<double*>(c.nu) + (size_t)c0 * n * n * n : c.tmpA;
    e = nu_chunk_dispatch(n, c.fac64 + (size_t)c0 * 6 * n, c.pref64 + (size_t)c0 * 2, c.Om64,
                          reinterpret_cast<double2*>(c.planes64), nu64, nc, c.stream);
    if (e != hipSuccess) return e;
    if (c.dtype != 0) {
      const long cnt = (long)nc * n * n * n;
      k_convert<float><<<(unsigned)((cnt + 255) / 256), 256, 0, c.stream>>>(
          nu64, static_cast<float*>(c.nu) + (size_t)c0 * n * n * n, cnt);
    }
  }
  (void)P;
  return hipGetLastError();
}

// ------------------------------------------------------------ projection
// y = x - M sum_a phi_a (A^-1 m[x])_a per cell; moments reduced in FP64.
constexpr int PROJ_TB = 1024;

// One block per cell: the five moments of x (FP64 sums in a fixed tree), the
// coefficients A^-1 m, then y = x - M sum_a coef_a phi_a.  n is a power of
// two, so velocity indices come from shifts of the flat index.  x and y may
// be the same array (the in-place projection of an apply's output), so
// neither is declared __restrict__.
template <typename T>
__global__ void __launch_bounds__(PROJ_TB) k_project(const T* x, T* y, int n, int lgn,
                                                     double L, const double* __restrict__ fac64,
                                                     const double* __restrict__ pref64,
                                                     const double* __restrict__ Ainv, int Bc,
                                                     const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double red[5][PROJ_TB];
  __shared__ double coef[5];
  const int cell = blockIdx.x, cc = Bc > 1 ? cell : 0;
  const int n3 = n << (2 * lgn), msk = n - 1;
  const T* xc = x + (size_t)cell * n3;
  T* yc = y + (size_t)cell * n3;
  const double hv = 2.0 * L / n;
  double m[5] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < n3; i += PROJ_TB) {
    const int ix = i >> (2 * lgn), iy = (i >> lgn) & msk, iz = i & msk;
    const double v1 = -L + ix * hv, v2 = -L + iy * hv, v3 = -L + iz * hv;
    const double xv = (double)xc[i];
    m[0] += xv;
    m[1] += xv * v1;
    m[2] += xv * v2;
    m[3] += xv * v3;
    m[4] += xv * (v1 * v1 + v2 * v2 + v3 * v3);
  }
  for (int a = 0; a < 5; ++a) red[a][threadIdx.x] = m[a];
  __syncthreads();
  for (int s = PROJ_TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int a = 0; a < 5; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int b = 0; b < 5; ++b) s += Ainv[(size_t)cc * 25 + 5 * threadIdx.x + b] * red[b][0];
    coef[threadIdx.x] = s;
  }
  __syncthreads();
  const double* f = fac64 + (size_t)cc * 6 * n;
  const double pm = pref64[2 * cc];
  for (int i = threadIdx.x; i < n3; i += PROJ_TB) {
    const int ix = i >> (2 * lgn), iy = (i >> lgn) & msk, iz = i & msk;
    const double v1 = -L + ix * hv, v2 = -L + iy * hv, v3 = -L + iz * hv;
    const double M = pm * f[ix] * f[n + iy] * f[2 * n + iz];
    const double corr = coef[0] + coef[1] * v1 + coef[2] * v2 + coef[3] * v3 + coef[4] * (v1 * v1 + v2 * v2 + v3 * v3);
    yc[i] = static_cast<T>((double)xc[i] - M * corr);
  }
}

hipError_t project_cells(const ProjectCtx& c) {
  int lgn = 0;
  while ((1 << lgn) < c.n) ++lgn;
  if ((1 << lgn) != c.n) return hipErrorInvalidValue;
  if (c.dtype == 0)
    k_project<double><<<c.batch, PROJ_TB, 0, c.stream>>>(static_cast<const double*>(c.x), static_cast<double*>(c.y),
                                                          c.n, lgn, c.L, c.fac64, c.pref64, c.Ainv, c.Bc, c.gate);
  else
    k_project<float><<<c.batch, PROJ_TB, 0, c.stream>>>(static_cast<const float*>(c.x), static_cast<float*>(c.y), c.n,
                                                         lgn, c.L, c.fac64, c.pref64, c.Ainv, c.Bc, c.gate);
  return hipGetLastError();
}

// ---- non-finite check (LINCOLL_OPT_CHECK_FINITE) -----------------------------
namespace {

__global__ void k_flag_clear(int* flag) { *flag = 0; }

template <typename T>
__global__ void __launch_bounds__(256) k_nonfinite(const T* __restrict__ x, long count, int* __restrict__ flag) {
  bool bad = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) *flag = 1;   // a plain vector store; any writer leaves 1
}

}  // namespace

hipError_t nonfinite_check(const void* x, long count, int dtype_f64, int* flag, hipStream_t s) {
  k_flag_clear<<<1, 1, 0, s>>>(flag);
  const long blocks = count / 256 + 1 < 4096 ? count / 256 + 1 : 4096;
  if (dtype_f64) k_nonfinite<double><<<(unsigned)blocks, 256, 0, s>>>(static_cast<const double*>(x), count, flag);
  else k_nonfinite<float><<<(unsigned)blocks, 256, 0, s>>>(static_cast<const float*>(x), count, flag);
  return hipGetLastError();
}

}  // namespace lincoll
