// Device side of the steady 1-D solver (Sec. 5, Appendix B): per-cell velocity
// moments, the upwind transport term of eq. (discrete_eq) with ghost cells of
// the fully accommodating walls (eq. (maxwell_bc)), the initial guess of
// eq. (initial), and the vector operations of restarted GMRES.  All FP64.
//
// Layout: a field is [nx][n][n][n] (cell-major, last velocity index fastest),
// velocity of index i along an axis -L + i h_v.  Reductions use a fixed tree,
// so every result is bitwise reproducible for a given launch shape.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "steady.h"

namespace lincoll {

namespace {

constexpr int TB = 256;          // threads per block
constexpr int EPT = 8;           // elements per thread in the vector kernels
constexpr int WAVES = TB / 64;
constexpr int SWEEP_VEL = 32;      // velocities per sweep block
constexpr int SWEEP_CHUNKS = 8;    // cell chunks per velocity (one thread each)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums NV per-thread values over the block; every thread gets the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sm[NV][WAVES];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    const double s = wave_sum(v[a]);
    if (l == 0) sm[a][w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double s = sm[a][0];
#pragma unroll
    for (int k = 1; k < WAVES; ++k) s += sm[a][k];
    v[a] = s;
  }
  __syncthreads();
}

// sums[c][0..6] = sum f, sum v1 f, sum v2 f, sum v3 f, sum |v|^2 f, sum v1+ f, sum v1- f
__global__ void __launch_bounds__(TB) k_cell_sums(const double* __restrict__ f, int n, double L, double hv,
                                                  double* __restrict__ sums) {
  const long n3 = (long)n * n * n;
  const int lgn = 31 - __builtin_clz(n), msk = n - 1;   // n is a power of two
  const double* x = f + (long)blockIdx.x * n3;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long e = threadIdx.x; e < n3; e += TB) {
    const int i1 = (int)(e >> (2 * lgn)), i2 = (int)(e >> lgn) & msk, i3 = (int)e & msk;
    const double v1 = -L + i1 * hv, v2 = -L + i2 * hv, v3 = -L + i3 * hv, y = x[e];
    v[0] += y;
    v[1] += v1 * y;
    v[2] += v2 * y;
    v[3] += v3 * y;
    v[4] += (v1 * v1 + v2 * v2 + v3 * v3) * y;
    v[5] += (v1 > 0.0 ? v1 : 0.0) * y;
    v[6] += (v1 < 0.0 ? v1 : 0.0) * y;
  }
  block_sum<7>(v);
  if (threadIdx.x < 7) sums[(long)blockIdx.x * SUMS_STRIDE + threadIdx.x] = v[threadIdx.x];
}

// (rho, u, theta) of each cell from its sums: rho = h^3 sum f, u = sum v f / sum f,
// theta = (sum |v|^2 f / sum f - |u|^2) / 3.
__global__ void k_params(const double* __restrict__ sums, int nx, double h3, double* __restrict__ params) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx) return;
  const double* s = sums + (long)c * SUMS_STRIDE;
  const double m = s[0], u1 = s[1] / m, u2 = s[2] / m, u3 = s[3] / m;
  params[5 * c + 0] = h3 * m;
  params[5 * c + 1] = u1;
  params[5 * c + 2] = u2;
  params[5 * c + 3] = u3;
  params[5 * c + 4] = (s[4] / m - (u1 * u1 + u2 * u2 + u3 * u3)) / 3.0;
}

// wall[0] = sum v1- x over the first cell, wall[1] = sum v1+ x over the last
// (a launch of one block computes wall[0] only).
// Only the velocities towards the wall contribute: the planes v1 < 0
// (i1 < n/2) at the left wall and v1 > 0 (i1 > n/2) at the right.  A single
// wide block per wall (the sum sits between the two sweeps, on the critical
// path) reads them plane by plane.
constexpr int TBW = 1024;
__global__ void __launch_bounds__(TBW) k_wall_sums(const double* __restrict__ x, int n, int nx, double L, double hv,
                                                   double* __restrict__ wall, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int n2 = n * n;
  const long n3 = (long)n2 * n;
  const bool left = blockIdx.x == 0;
  const double* c = x + (left ? 0 : (long)(nx - 1) * n3);
  const int i1a = left ? 0 : n / 2 + 1, i1b = left ? n / 2 : n;
  double v = 0.0;
  for (int i1 = i1a; i1 < i1b; ++i1) {
    const double v1 = -L + i1 * hv;
    const double* p = c + (long)i1 * n2;
    for (int r = threadIdx.x; r < n2; r += TBW) v += v1 * p[r];
  }
  __shared__ double sm[TBW / 64];
  v = wave_sum(v);
  if (threadIdx.x % 64 == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < TBW / 64; ++w) t += sm[w];
    wall[blockIdx.x] = t;
  }
}

__device__ __forceinline__ double wall_shape(double v1, double v2, double v3, const WallGeom& w, int side) {
  const double a = v1 - w.u[side][0], b = v2 - w.u[side][1], c = v3 - w.u[side][2];
  const double d2 = a * a + b * b + c * c;
  return exp(-d2 / (2.0 * w.theta[side]));
}

// out = T[x] + alpha (y - ymean_c), T[x]_c = (v1+ (x_c - x_{c-1}) + v1- (x_{c+1} - x_c)) / dx
// with the wall ghosts x_{-1} = rho_L E_L, x_{nx} = rho_R E_R,
// rho_L = -wall[0] / sum v1+ E_L, rho_R = -wall[1] / sum v1- E_R.
// y may be null (no collision term); ysums may be null (no mean removal).
template <typename T>
__global__ void __launch_bounds__(TB) k_transport(const double* __restrict__ x, const double* __restrict__ wall,
                                                  WallGeom wg, const T* __restrict__ y, double alpha,
                                                  const double* __restrict__ ysums, double* __restrict__ out, int n,
                                                  int nx, double L, double hv, double dx,
                                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const long n3 = (long)n * n * n, total = (long)nx * n3;
  const int lgn = 31 - __builtin_clz(n), msk = n - 1;   // n is a power of two
  const double rdx = 1.0 / dx;
  for (long idx = (long)blockIdx.x * TB + threadIdx.x; idx < total; idx += (long)gridDim.x * TB) {
    const long c = idx >> (3 * lgn), e = idx & (n3 - 1);
    const int i1 = (int)(e >> (2 * lgn)), i2 = (int)(e >> lgn) & msk, i3 = (int)e & msk;
    const double v1 = -L + i1 * hv;
    const double xc = x[idx];
    double t = 0.0;
    if (v1 > 0.0) {
      double nb;
      if (c > 0) {
        nb = x[idx - n3];
      } else {
        const double rho = -wall[0] / wg.flux_in[0];
        nb = rho * wall_shape(v1, -L + i2 * hv, -L + i3 * hv, wg, 0);
      }
      t = v1 * (xc - nb) * rdx;
    } else if (v1 < 0.0) {
      double nb;
      if (c < nx - 1) {
        nb = x[idx + n3];
      } else {
        const double rho = -wall[1] / wg.flux_in[1];
        nb = rho * wall_shape(v1, -L + i2 * hv, -L + i3 * hv, wg, 1);
      }
      t = v1 * (nb - xc) * rdx;
    }
    if (y) {
      const double m = ysums ? ysums[c * SUMS_STRIDE] / (double)n3 : 0.0;
      t += alpha * ((double)y[idx] - m);
    }
    out[idx] = t;
  }
}

// Transport sweep z = (T + D/Kn)^-1 y, D = diag(nu_c(v)) the loss collision
// frequency of each cell's linearized operator: per velocity a first-order
// recurrence along x in the upwind direction (the fast sweeping of the source
// iteration, Sec. 5.2):
//   z_c = (y_c + |v1|/dx z_prev) / (|v1|/dx + nu_c/Kn) = alpha_c z_prev + beta_c.
// NEG (v1 <= 0) runs from the right wall leftwards with an empty (zero) ghost;
// the POS pass (v1 > 0) runs rightwards from the left ghost rho_L E_L with
// rho_L = -wall[0] / sum v1+ E_L, wall[0] = sum v1- z over the first cell as
// left by the NEG pass.  A fixed linear map, used as a preconditioner.
//
// The recurrence is linear, so each velocity's cells are cut into
// SWEEP_CHUNKS chunks run by different threads: each chunk first composes its
// map z_out = A z_in + B from a zero start, one thread per velocity chains the
// chunk maps from the ghost, and each chunk then reruns its cells from its
// exact carry-in.  A block holds SWEEP_VEL velocities x SWEEP_CHUNKS chunks.
template <typename TN, bool NEG>
__global__ void __launch_bounds__(SWEEP_VEL * SWEEP_CHUNKS) k_sweep(const double* __restrict__ y,
                                                                    double* __restrict__ z,
                                                                    const TN* __restrict__ nu,
                                                                    const double* __restrict__ wall, WallGeom wg,
                                                                    int n, int nx, double L, double hv, double dx,
                                                                    double kn, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double cA[SWEEP_CHUNKS][SWEEP_VEL], cB[SWEEP_CHUNKS][SWEEP_VEL];
  const long n2 = (long)n * n, n3 = n2 * n;
  const long count = NEG ? (long)(n / 2 + 1) * n2 : (long)(n / 2 - 1) * n2;
  const int lv = threadIdx.x % SWEEP_VEL, ch = threadIdx.x / SWEEP_VEL;
  const long t = (long)blockIdx.x * SWEEP_VEL + lv;
  const bool live = t < count;
  const long e = (NEG ? 0 : (long)(n / 2 + 1) * n2) + (live ? t : 0);
  const int i1 = (int)(e / n2), i2 = (int)((e / n) % n), i3 = (int)(e % n);
  const double v1 = -L + i1 * hv, a = fabs(v1) / dx, ikn = 1.0 / kn;
  const int per = (nx + SWEEP_CHUNKS - 1) / SWEEP_CHUNKS;
  const int k0 = ch * per, k1 = min(nx, k0 + per);   // steps k of this chunk (k = 0 at the inflow wall)
  auto cell = [&](int k) { return (long)(NEG ? nx - 1 - k : k) * n3 + e; };
  // 1. the chunk's map from a zero carry-in
  double A = 1.0, B = 0.0;
  if (live)
    for (int k = k0; k < k1; ++k) {
      const long i = cell(k);
      const double d = a + fmax((double)nu[i], 0.0) * ikn;
      const double al = d > 0.0 ? a / d : 0.0, be = d > 0.0 ? y[i] / d : 0.0;
      A *= al;
      B = al * B + be;
    }
  cA[ch][lv] = A;
  cB[ch][lv] = B;
  __syncthreads();
  // 2. chain the chunks from the ghost
  if (ch == 0) {
    double carry = 0.0;
    if (!NEG && live) carry = -wall[0] / wg.flux_in[0] * wall_shape(v1, -L + i2 * hv, -L + i3 * hv, wg, 0);
    for (int c = 0; c < SWEEP_CHUNKS; ++c) {
      const double in = carry;
      carry = cA[c][lv] * in + cB[c][lv];
      cA[c][lv] = in;   // becomes chunk c's carry-in
    }
  }
  __syncthreads();
  // 3. rerun the chunk from its carry-in
  if (!live) return;
  double prev = cA[ch][lv];
  for (int k = k0; k < k1; ++k) {
    const long i = cell(k);
    const double d = a + fmax((double)nu[i], 0.0) * ikn;
    const double v = d > 0.0 ? (y[i] + a * prev) / d : 0.0;
    z[i] = v;
    prev = v;
  }
}

// eq. (initial): f_c(v) = C/(x_R - x_L) (2 pi theta_c)^(-3/2) exp(-|v|^2/(2 theta_c)),
// theta_c linear between the wall temperatures at the cell centre x_c.
__global__ void __launch_bounds__(TB) k_initial(double* __restrict__ f, int n, int nx, double L, double hv,
                                                double x_l, double x_r, double theta_l, double theta_r, double C) {
  const long n3 = (long)n * n * n, total = (long)nx * n3;
  const double dx = (x_r - x_l) / nx;
  for (long idx = (long)blockIdx.x * TB + threadIdx.x; idx < total; idx += (long)gridDim.x * TB) {
    const long c = idx / n3, e = idx - c * n3;
    const double xc = x_l + ((double)c + 0.5) * dx;
    const double th = ((x_r - xc) * theta_l + (xc - x_l) * theta_r) / (x_r - x_l);
    const double v1 = -L + (int)(e / ((long)n * n)) * hv, v2 = -L + (int)((e / n) % n) * hv,
                 v3 = -L + (int)(e % n) * hv;
    const double d2 = v1 * v1 + v2 * v2 + v3 * v3;
    f[idx] = C / (x_r - x_l) * pow(2.0 * M_PI * th, -1.5) * exp(-d2 / (2.0 * th));
  }
}

// ---- vector operations (N elements, EPT per thread, coalesced) ------------

__device__ __forceinline__ long vec_index(int r) { return ((long)blockIdx.x * EPT + r) * TB + threadIdx.x; }

// partial[b][i] = block b's part of <V_i, w>, i < k
__global__ void __launch_bounds__(TB) k_mdot(const double* __restrict__ V, long N, int k, const double* __restrict__ w,
                                             double* __restrict__ partial, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double sm[GMRES_MAXK][WAVES];
  double wr[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    wr[r] = i < N ? w[i] : 0.0;
  }
  const int wv = threadIdx.x / 64, l = threadIdx.x % 64;
  for (int a = 0; a < k; ++a) {
    const double* Va = V + (long)a * N;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
      const long i = vec_index(r);
      if (i < N) s += Va[i] * wr[r];
    }
    s = wave_sum(s);
    if (l == 0) sm[a][wv] = s;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < k; a += TB) {
    double s = sm[a][0];
    for (int q = 1; q < WAVES; ++q) s += sm[a][q];
    partial[(long)blockIdx.x * GMRES_MAXK + a] = s;
  }
}

// out[a] = sum over blocks of partial[b][a], a < k (one block per a)
__global__ void __launch_bounds__(TB) k_reduce_cols(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int a = blockIdx.x;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nblk; b += TB) v[0] += partial[(long)b * GMRES_MAXK + a];
  block_sum<1>(v);
  if (threadIdx.x == 0) out[a] = v[0];
}

// w -= sum_{a<k} h[a] V_a; partial[b][0] = block b's part of |w|^2
__global__ void __launch_bounds__(TB) k_update(double* __restrict__ w, const double* __restrict__ V, long N, int k,
                                               const double* __restrict__ h, double* __restrict__ partial,
                                               const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  double v[1] = {0.0};
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) {
      double acc = w[i];
      for (int a = 0; a < k; ++a) acc -= h[a] * V[(long)a * N + i];
      w[i] = acc;
      v[0] += acc * acc;
    }
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) partial[(long)blockIdx.x * GMRES_MAXK] = v[0];
}

// x += sum_{a<k} y[a] V_a, with k = *kdev when kdev is set
__global__ void __launch_bounds__(TB) k_combine(double* __restrict__ x, const double* __restrict__ V, long N, int k,
                                                const double* __restrict__ y, const int* __restrict__ kdev,
                                                const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  if (kdev) k = *kdev;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) {
      double acc = x[i];
      for (int a = 0; a < k; ++a) acc += y[a] * V[(long)a * N + i];
      x[i] = acc;
    }
  }
}

// partial[b][0] = block b's part of sum x
__global__ void __launch_bounds__(TB) k_sum(const double* __restrict__ x, long N, double* __restrict__ partial,
                                            const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  double v[1] = {0.0};
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) v[0] += x[i];
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) partial[(long)blockIdx.x * GMRES_MAXK] = v[0];
}

// z -= (*sz * *ifmass) f
__global__ void __launch_bounds__(TB) k_remove_mass(double* __restrict__ z, const double* __restrict__ f,
                                                    const double* __restrict__ sz, const double* __restrict__ ifmass,
                                                    long N, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const double c = *sz * *ifmass;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) z[i] -= c * f[i];
  }
}

// out = a x + b y (y may be null: out = a x); out may alias x or y
__global__ void __launch_bounds__(TB) k_axpby(double* out, double a, const double* x, double b, const double* y,
                                              long N, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) out[i] = y ? a * x[i] + b * y[i] : a * x[i];
  }
}

__global__ void __launch_bounds__(TB) k_to_f32(const double* __restrict__ x, float* __restrict__ y, long N,
                                               const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) y[i] = (float)x[i];
  }
}

unsigned grid_stride_blocks(long total) {
  const long b = (total + TB - 1) / TB;
  return (unsigned)(b < 8192 ? b : 8192);
}

}  // namespace

unsigned vec_blocks(long N) { return (unsigned)((N + (long)TB * EPT - 1) / ((long)TB * EPT)); }

hipError_t st_cell_sums(const double* f, int nx, int n, double L, double* sums, hipStream_t s) {
  k_cell_sums<<<nx, TB, 0, s>>>(f, n, L, 2.0 * L / n, sums);
  return hipGetLastError();
}

hipError_t st_params(const double* sums, int nx, int n, double L, double* params, hipStream_t s) {
  const double hv = 2.0 * L / n;
  k_params<<<(nx + 63) / 64, 64, 0, s>>>(sums, nx, hv * hv * hv, params);
  return hipGetLastError();
}

hipError_t st_wall_sums(const double* x, int nx, int n, double L, double* wall, hipStream_t s, const int* gate) {
  k_wall_sums<<<2, TBW, 0, s>>>(x, n, nx, L, 2.0 * L / n, wall, gate);
  return hipGetLastError();
}

hipError_t st_sweep(const double* y, double* z, const void* nu, int nu_f32, double* wall, const WallGeom& wg, int nx,
                    int n, double L, double dx, double kn, hipStream_t s, const int* gate) {
  const double hv = 2.0 * L / n;
  const long n2 = (long)n * n;
  const unsigned bneg = (unsigned)(((n / 2 + 1) * n2 + SWEEP_VEL - 1) / SWEEP_VEL),
                 bpos = (unsigned)(((n / 2 - 1) * n2 + SWEEP_VEL - 1) / SWEEP_VEL);
  constexpr int TBS = SWEEP_VEL * SWEEP_CHUNKS;
  if (nu_f32) {
    const float* q = static_cast<const float*>(nu);
    k_sweep<float, true><<<bneg, TBS, 0, s>>>(y, z, q, wall, wg, n, nx, L, hv, dx, kn, gate);
    k_wall_sums<<<1, TBW, 0, s>>>(z, n, nx, L, hv, wall, gate);
    k_sweep<float, false><<<bpos, TBS, 0, s>>>(y, z, q, wall, wg, n, nx, L, hv, dx, kn, gate);
  } else {
    const double* q = static_cast<const double*>(nu);
    k_sweep<double, true><<<bneg, TBS, 0, s>>>(y, z, q, wall, wg, n, nx, L, hv, dx, kn, gate);
    k_wall_sums<<<1, TBW, 0, s>>>(z, n, nx, L, hv, wall, gate);
    k_sweep<double, false><<<bpos, TBS, 0, s>>>(y, z, q, wall, wg, n, nx, L, hv, dx, kn, gate);
  }
  return hipGetLastError();
}

hipError_t st_transport(const double* x, const double* wall, const WallGeom& wg, const void* y, int y_f32,
                        double alpha, const double* ysums, double* out, int nx, int n, double L, double dx,
                        hipStream_t s, const int* gate) {
  const long total = (long)nx * n * n * n;
  const double hv = 2.0 * L / n;
  if (y_f32)
    k_transport<float><<<grid_stride_blocks(total), TB, 0, s>>>(x, wall, wg, static_cast<const float*>(y), alpha,
                                                                ysums, out, n, nx, L, hv, dx, gate);
  else
    k_transport<double><<<grid_stride_blocks(total), TB, 0, s>>>(x, wall, wg, static_cast<const double*>(y), alpha,
                                                                 ysums, out, n, nx, L, hv, dx, gate);
  return hipGetLastError();
}

hipError_t st_initial(double* f, int nx, int n, double L, double x_l, double x_r, double theta_l, double theta_r,
                      double C, hipStream_t s) {
  const long total = (long)nx * n * n * n;
  k_initial<<<grid_stride_blocks(total), TB, 0, s>>>(f, n, nx, L, 2.0 * L / n, x_l, x_r, theta_l, theta_r, C);
  return hipGetLastError();
}

hipError_t st_mdot(const double* V, long N, int k, const double* w, double* partial, double* out, hipStream_t s,
                   const int* gate) {
  const unsigned nb = vec_blocks(N);
  k_mdot<<<nb, TB, 0, s>>>(V, N, k, w, partial, gate);
  k_reduce_cols<<<k, TB, 0, s>>>(partial, (int)nb, out, gate);
  return hipGetLastError();
}

hipError_t st_update(double* w, const double* V, long N, int k, const double* h, double* partial, double* norm2,
                     hipStream_t s, const int* gate) {
  const unsigned nb = vec_blocks(N);
  k_update<<<nb, TB, 0, s>>>(w, V, N, k, h, partial, gate);
  k_reduce_cols<<<1, TB, 0, s>>>(partial, (int)nb, norm2, gate);
  return hipGetLastError();
}

hipError_t st_combine(double* x, const double* V, long N, int k, const double* y, hipStream_t s) {
  k_combine<<<vec_blocks(N), TB, 0, s>>>(x, V, N, k, y, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t st_axpby(double* out, double a, const double* x, double b, const double* y, long N, hipStream_t s,
                    const int* gate) {
  k_axpby<<<vec_blocks(N), TB, 0, s>>>(out, a, x, b, y, N, gate);
  return hipGetLastError();
}

hipError_t st_remove_mass(double* z, const double* f, const double* ifsum, long N, double* partial, double* red,
                          hipStream_t s, const int* gate) {
  const unsigned nb = vec_blocks(N);
  k_sum<<<nb, TB, 0, s>>>(z, N, partial, gate);
  k_reduce_cols<<<1, TB, 0, s>>>(partial, (int)nb, red, gate);
  k_remove_mass<<<nb, TB, 0, s>>>(z, f, red, ifsum, N, gate);
  return hipGetLastError();
}

hipError_t st_to_f32(const double* x, float* y, long N, hipStream_t s, const int* gate) {
  k_to_f32<<<vec_blocks(N), TB, 0, s>>>(x, y, N, gate);
  return hipGetLastError();
}

// ---- restarted flexible GMRES with its bookkeeping on the device -----------
// One thread does the O(m) Givens work of an Arnoldi step and the O(m^2)
// back substitution of a cycle; the vector kernels of a step are gated by
// st->active, those of a cycle by st->go, and the restart product by st->pro,
// so a whole cycle can be replayed as one recorded graph and the host reads
// the state once per cycle.

namespace {

__global__ void k_gm_init(GmresState* st, int m, double target, int budget, int mode, int iters0) {
  st->m = m;
  st->j = 0;
  st->iters = iters0;
  st->budget = budget;
  st->mode = mode;
  st->go = 1;
  st->active = 0;
  st->pro = 0;
  st->done = 0;
  st->target = target;
  st->beta = 0.0;
  st->resid = 0.0;
  st->inv = 1.0;
}

// V0 = b (mode 0, start x = 0), kept (mode 1: it holds the residual of the
// given start) or b - A x (mode 2, restarts; tmp = A x)
__global__ void __launch_bounds__(TB) k_gm_v0(double* __restrict__ V0, const double* __restrict__ b,
                                              const double* __restrict__ tmp, const GmresState* __restrict__ st,
                                              long N) {
  if (!st->go || st->mode == 1) return;
  const bool rs = st->mode == 2;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) V0[i] = rs ? b[i] - tmp[i] : b[i];
  }
}

// red[0] = |V0|^2: start of a cycle
__global__ void k_gm_begin(GmresState* st, const double* red) {
  if (!st->go) return;
  if (st->pro) ++st->iters;   // the restart product A x
  const double beta = sqrt(red[0]);
  st->beta = beta;
  st->resid = beta;
  if (!(beta > st->target) || (st->pro && st->iters >= st->budget)) {
    st->go = 0;
    st->done = 1;
    st->active = 0;
    st->j = 0;
    st->pro = 0;
    return;
  }
  st->pro = 0;
  for (int i = 0; i <= st->m; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->inv = 1.0 / beta;
  st->j = 0;
  st->active = 1;
}

// Step j: red[0..j] = <V_i, w>, red[j + 1] = |w|^2 after the Gram-Schmidt
// update.  Applies the previous rotations to the new column, forms the next
// one, updates g and the residual estimate |g[j+1]|.
__global__ void k_gm_step(GmresState* st, const double* red, int j) {
  if (!st->active) return;
  const int m = st->m;
  ++st->iters;
  double col[GMRES_MAXK + 1];
  for (int i = 0; i <= j + 1; ++i) col[i] = red[i];
  const double hn = sqrt(fmax(col[j + 1], 0.0));
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = st->cs[i] * col[i] + st->sn[i] * col[i + 1];
    col[i + 1] = -st->sn[i] * col[i] + st->cs[i] * col[i + 1];
    col[i] = t;
  }
  const double rr = hypot(col[j], col[j + 1]);
  st->cs[j] = rr > 0.0 ? col[j] / rr : 1.0;
  st->sn[j] = rr > 0.0 ? col[j + 1] / rr : 0.0;
  col[j] = rr;
  for (int i = 0; i <= j; ++i) st->R[i * m + j] = col[i];
  st->g[j + 1] = -st->sn[j] * st->g[j];
  st->g[j] = st->cs[j] * st->g[j];
  const double resid = fabs(st->g[j + 1]);
  st->resid = resid;
  st->j = j + 1;
  if (!(hn > 0.0) || !isfinite(resid)) {   // breakdown (exact) or non-finite values
    st->active = 0;
    st->done = 1;
    st->inv = 1.0;
    return;
  }
  st->inv = 1.0 / hn;
  if (resid <= st->target || st->iters >= st->budget) {
    st->active = 0;
    st->done = 1;
  }
}

// back substitution R y = g over the st->j columns of this cycle
__global__ void k_gm_end(GmresState* st) {
  if (!st->go) return;
  const int m = st->m, j = st->j;
  for (int i = j - 1; i >= 0; --i) {
    double t = st->g[i];
    for (int k = i + 1; k < j; ++k) t -= st->R[i * m + k] * st->y[k];
    st->y[i] = t / st->R[i * m + i];
  }
}

// after the cycle's combine: restart (mode 2) unless done or out of budget
__global__ void k_gm_finish(GmresState* st) {
  if (!st->go) return;
  st->active = 0;
  if (st->done || st->iters >= st->budget) {
    st->done = 1;
    st->go = 0;
    st->pro = 0;
  } else {
    st->mode = 2;
    st->pro = 1;
  }
}

// x *= *a
__global__ void __launch_bounds__(TB) k_scale_dev(double* __restrict__ x, const double* __restrict__ a, long N,
                                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const double c = *a;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const long i = vec_index(r);
    if (i < N) x[i] *= c;
  }
}

__global__ void k_set(double* dst, double v) { *dst = v; }

}  // namespace

hipError_t gm_init(GmresState* st, int m, double target, int budget, int mode, int iters0, hipStream_t s) {
  k_gm_init<<<1, 1, 0, s>>>(st, m, target, budget, mode, iters0);
  return hipGetLastError();
}

hipError_t gm_v0(double* V0, const double* b, const double* tmp, const GmresState* st, long N, hipStream_t s) {
  k_gm_v0<<<vec_blocks(N), TB, 0, s>>>(V0, b, tmp, st, N);
  return hipGetLastError();
}

hipError_t gm_begin(GmresState* st, const double* red, hipStream_t s) {
  k_gm_begin<<<1, 1, 0, s>>>(st, red);
  return hipGetLastError();
}

hipError_t gm_step(GmresState* st, const double* red, int j, hipStream_t s) {
  k_gm_step<<<1, 1, 0, s>>>(st, red, j);
  return hipGetLastError();
}

hipError_t gm_end(GmresState* st, hipStream_t s) {
  k_gm_end<<<1, 1, 0, s>>>(st);
  return hipGetLastError();
}

hipError_t gm_finish(GmresState* st, hipStream_t s) {
  k_gm_finish<<<1, 1, 0, s>>>(st);
  return hipGetLastError();
}

hipError_t st_scale_dev(double* x, const double* a, long N, const int* gate, hipStream_t s) {
  k_scale_dev<<<vec_blocks(N), TB, 0, s>>>(x, a, N, gate);
  return hipGetLastError();
}

hipError_t st_combine_dev(double* x, const double* V, long N, const int* k, const double* y, const int* gate,
                          hipStream_t s) {
  k_combine<<<vec_blocks(N), TB, 0, s>>>(x, V, N, 0, y, k, gate);
  return hipGetLastError();
}

hipError_t st_set(double* dst, double v, hipStream_t s) {
  k_set<<<1, 1, 0, s>>>(dst, v);
  return hipGetLastError();
}

}  // namespace lincoll
