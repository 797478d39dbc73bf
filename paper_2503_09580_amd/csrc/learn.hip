// Learned correction of the steady solver's inner solves: per-cell Hermite
// moments, the cell features, the macroscopic correction field, and the
// small FP32 network (26 -> 128 tanh -> 5) with its forward pass, MSE
// backward pass and Adam update.
//
// Per cell c with local Maxwellian (rho, u, theta):
//   psi_0 = 1, psi_d = (v_d - u_d)/sqrt(theta), psi_4 = (|v-u|^2/theta - 3)/sqrt 6,
//   m_a(c) = h^3 sum_v z_c(v) psi_a(v) / rho_c,
// features (26): with s = sqrt(mean m^2) (1 if zero), ms = m/s, x_c = (c+1/2)/nx:
//   ms | (sum_{c'<=c} ms - ms/2)/nx | (sum_{c'>=c} ms - ms/2)/nx
//      | sum_{c'<=c} ms x_c'/nx | sum_{c'>=c} ms x_c'/nx | x_c,
// correction: Delta_c(v) = sum_a s y_a(c) M_c(v) psi_a(v).
// Weights are one packed float array: W1 [26][128], b1 [128], W2 [128][5], b2 [5].
#include <hip/hip_runtime.h>

#include "learn.h"

namespace lincoll {

namespace {

constexpr int TB = 256;
constexpr int WAVES = TB / 64;
constexpr int OFF_B1 = MLP_IN * MLP_HID, OFF_W2 = OFF_B1 + MLP_HID, OFF_B2 = OFF_W2 + MLP_HID * MLP_OUT;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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

struct Cell {
  double rho, u1, u2, u3, rt, norm;   // rt = 1/sqrt(theta), norm = rho (2 pi theta)^-3/2
  double itheta;
};

__device__ __forceinline__ Cell cell_of(const double* p) {
  Cell c;
  c.rho = p[0];
  c.u1 = p[1];
  c.u2 = p[2];
  c.u3 = p[3];
  c.itheta = 1.0 / p[4];
  c.rt = sqrt(c.itheta);
  c.norm = p[0] * pow(2.0 * M_PI * p[4], -1.5);
  return c;
}

__device__ __forceinline__ void psi5(const Cell& c, double v1, double v2, double v3, double (&ps)[5]) {
  const double w1 = (v1 - c.u1) * c.rt, w2 = (v2 - c.u2) * c.rt, w3 = (v3 - c.u3) * c.rt;
  ps[0] = 1.0;
  ps[1] = w1;
  ps[2] = w2;
  ps[3] = w3;
  ps[4] = (w1 * w1 + w2 * w2 + w3 * w3 - 3.0) / sqrt(6.0);
}

// m[c][a] = h^3 sum z psi_a / rho; b (optional): z - b
__global__ void __launch_bounds__(TB) k_hermite(const double* __restrict__ z, const double* __restrict__ b,
                                                const double* __restrict__ params, int n, double L, double hv,
                                                double* __restrict__ m) {
  const long n3 = (long)n * n * n;
  const long base = (long)blockIdx.x * n3;
  const Cell c = cell_of(params + 5 * blockIdx.x);
  double acc[5] = {0, 0, 0, 0, 0};
  for (long e = threadIdx.x; e < n3; e += TB) {
    const double v1 = -L + (int)(e / ((long)n * n)) * hv, v2 = -L + (int)((e / n) % n) * hv,
                 v3 = -L + (int)(e % n) * hv;
    double ps[5];
    psi5(c, v1, v2, v3, ps);
    const double y = b ? z[base + e] - b[base + e] : z[base + e];
#pragma unroll
    for (int a = 0; a < 5; ++a) acc[a] += y * ps[a];
  }
  block_sum<5>(acc);
  if (threadIdx.x < 5) m[5 * (long)blockIdx.x + threadIdx.x] = hv * hv * hv * acc[threadIdx.x] / c.rho;
}

// One block: s = sqrt(mean m^2) (1 if zero) into *s, the features into X.
__global__ void __launch_bounds__(TB) k_features(const double* __restrict__ m, int nx, float* __restrict__ X,
                                                 double* __restrict__ s_out) {
  __shared__ double s_sh;
  double q[1] = {0.0};
  for (int i = threadIdx.x; i < 5 * nx; i += TB) q[0] += m[i] * m[i];
  block_sum<1>(q);
  if (threadIdx.x == 0) {
    double s = sqrt(q[0] / (5.0 * nx));
    if (s == 0.0) s = 1.0;
    s_sh = s;
    *s_out = s;
  }
  __syncthreads();
  const double is = 1.0 / s_sh, inx = 1.0 / nx;
  for (int c = threadIdx.x; c < nx; c += TB) {
    float* x = X + (long)c * MLP_IN;
    for (int a = 0; a < 5; ++a) x[a] = (float)(m[5 * c + a] * is);
    x[25] = (float)((c + 0.5) * inx);
  }
  // prefix (threads 0..4) and suffix (threads 5..9) scans, one moment each
  if (threadIdx.x < 10) {
    const int a = threadIdx.x % 5;
    const bool left = threadIdx.x < 5;
    double run = 0.0, runx = 0.0;
    for (int k = 0; k < nx; ++k) {
      const int c = left ? k : nx - 1 - k;
      const double ms = m[5 * c + a] * is, xc = (c + 0.5) * inx;
      run += ms;
      runx += ms * xc;
      float* x = X + (long)c * MLP_IN;
      x[(left ? 5 : 10) + a] = (float)((run - 0.5 * ms) * inx);
      x[(left ? 15 : 20) + a] = (float)(runx * inx);
    }
  }
}

// out (=|+=) sum_a s y_a(c) M_c psi_a, grid-stride over all cells
__global__ void __launch_bounds__(TB) k_correction(const float* __restrict__ Y, const double* __restrict__ s,
                                                   const double* __restrict__ params, int n, int nx, double L,
                                                   double hv, int accumulate, double* __restrict__ out) {
  const long n3 = (long)n * n * n, total = (long)nx * n3;
  const double sc = *s;
  for (long idx = (long)blockIdx.x * TB + threadIdx.x; idx < total; idx += (long)gridDim.x * TB) {
    const long cc = idx / n3, e = idx - cc * n3;
    const Cell c = cell_of(params + 5 * cc);
    const double v1 = -L + (int)(e / ((long)n * n)) * hv, v2 = -L + (int)((e / n) % n) * hv,
                 v3 = -L + (int)(e % n) * hv;
    double ps[5];
    psi5(c, v1, v2, v3, ps);
    const double d1 = v1 - c.u1, d2 = v2 - c.u2, d3 = v3 - c.u3;
    const double M = c.norm * exp(-0.5 * (d1 * d1 + d2 * d2 + d3 * d3) * c.itheta);
    double t = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) t += (double)Y[5 * cc + a] * ps[a];
    const double d = sc * M * t;
    out[idx] = accumulate ? out[idx] + d : d;
  }
}

// T[c][a] = m[c][a] / s (float)
__global__ void k_scale_targets(const double* __restrict__ m, const double* __restrict__ s, int count,
                                float* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) T[i] = (float)(m[i] / *s);
}

// ---- network ----------------------------------------------------------------

// one block of MLP_HID threads per row
__global__ void __launch_bounds__(MLP_HID) k_mlp_fwd(const float* __restrict__ X, const float* __restrict__ W,
                                                     int rows, float* __restrict__ H, float* __restrict__ Y) {
  __shared__ float x[MLP_IN];
  __shared__ float part[MLP_OUT][MLP_HID];
  const int row = blockIdx.x, k = threadIdx.x;
  if (k < MLP_IN) x[k] = X[(long)row * MLP_IN + k];
  __syncthreads();
  float a = W[OFF_B1 + k];
  for (int i = 0; i < MLP_IN; ++i) a += x[i] * W[i * MLP_HID + k];
  const float h = tanhf(a);
  if (H) H[(long)row * MLP_HID + k] = h;
  for (int o = 0; o < MLP_OUT; ++o) part[o][k] = h * W[OFF_W2 + k * MLP_OUT + o];
  __syncthreads();
  for (int w = MLP_HID / 2; w > 0; w >>= 1) {
    if (k < w)
      for (int o = 0; o < MLP_OUT; ++o) part[o][k] += part[o][k + w];
    __syncthreads();
  }
  if (k < MLP_OUT) Y[(long)row * MLP_OUT + k] = part[k][0] + W[OFF_B2 + k];
}

// dY = 2 (Y - T) / (rows MLP_OUT); lossp[block] = block's sum of (Y - T)^2
__global__ void __launch_bounds__(TB) k_mlp_dy(const float* __restrict__ Y, const float* __restrict__ T, int count,
                                               float* __restrict__ dY, double* __restrict__ lossp) {
  const int i = blockIdx.x * TB + threadIdx.x;
  double q[1] = {0.0};
  if (i < count) {
    const float e = Y[i] - T[i];
    dY[i] = 2.0f * e / (float)count;
    q[0] = (double)e * (double)e;
  }
  block_sum<1>(q);
  if (threadIdx.x == 0) lossp[blockIdx.x] = q[0];
}

// dH = (dY W2^T) (1 - H^2), one block of MLP_HID threads per row
__global__ void __launch_bounds__(MLP_HID) k_mlp_dh(const float* __restrict__ dY, const float* __restrict__ W,
                                                    const float* __restrict__ H, int rows, float* __restrict__ dH) {
  const int row = blockIdx.x, k = threadIdx.x;
  float s = 0.0f;
  for (int o = 0; o < MLP_OUT; ++o) s += dY[(long)row * MLP_OUT + o] * W[OFF_W2 + k * MLP_OUT + o];
  const float h = H[(long)row * MLP_HID + k];
  dH[(long)row * MLP_HID + k] = s * (1.0f - h * h);
}

// one thread per weight: sum over rows (double accumulation)
__global__ void __launch_bounds__(TB) k_mlp_wgrad(const float* __restrict__ X, const float* __restrict__ H,
                                                  const float* __restrict__ dY, const float* __restrict__ dH,
                                                  int rows, float* __restrict__ G) {
  const int w = blockIdx.x * TB + threadIdx.x;
  if (w >= MLP_WEIGHTS) return;
  double acc = 0.0;
  if (w < OFF_B1) {
    const int i = w / MLP_HID, k = w % MLP_HID;
    for (int b = 0; b < rows; ++b) acc += (double)X[(long)b * MLP_IN + i] * dH[(long)b * MLP_HID + k];
  } else if (w < OFF_W2) {
    const int k = w - OFF_B1;
    for (int b = 0; b < rows; ++b) acc += dH[(long)b * MLP_HID + k];
  } else if (w < OFF_B2) {
    const int k = (w - OFF_W2) / MLP_OUT, o = (w - OFF_W2) % MLP_OUT;
    for (int b = 0; b < rows; ++b) acc += (double)H[(long)b * MLP_HID + k] * dY[(long)b * MLP_OUT + o];
  } else {
    const int o = w - OFF_B2;
    for (int b = 0; b < rows; ++b) acc += dY[(long)b * MLP_OUT + o];
  }
  G[w] = (float)acc;
}

// Adam with bias correction: c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
__global__ void __launch_bounds__(TB) k_adam(float* __restrict__ W, const float* __restrict__ G,
                                             float* __restrict__ Mo, float* __restrict__ Vo, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
  const int w = blockIdx.x * TB + threadIdx.x;
  if (w >= MLP_WEIGHTS) return;
  const float g = G[w];
  const float m = b1 * Mo[w] + (1.0f - b1) * g;
  const float v = b2 * Vo[w] + (1.0f - b2) * g * g;
  Mo[w] = m;
  Vo[w] = v;
  W[w] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

unsigned gs_blocks(long total) {
  const long b = (total + TB - 1) / TB;
  return (unsigned)(b < 8192 ? b : 8192);
}

}  // namespace

hipError_t ln_hermite(const double* z, const double* b, const double* params, int nx, int n, double L, double* m,
                      hipStream_t s) {
  k_hermite<<<nx, TB, 0, s>>>(z, b, params, n, L, 2.0 * L / n, m);
  return hipGetLastError();
}

hipError_t ln_features(const double* m, int nx, float* X, double* s_dev, hipStream_t s) {
  k_features<<<1, TB, 0, s>>>(m, nx, X, s_dev);
  return hipGetLastError();
}

hipError_t ln_correction(const float* Y, const double* s_dev, const double* params, int nx, int n, double L,
                         int accumulate, double* out, hipStream_t s) {
  k_correction<<<gs_blocks((long)nx * n * n * n), TB, 0, s>>>(Y, s_dev, params, n, nx, L, 2.0 * L / n, accumulate,
                                                              out);
  return hipGetLastError();
}

hipError_t ln_targets(const double* m, const double* s_dev, int nx, float* T, hipStream_t s) {
  k_scale_targets<<<(5 * nx + 255) / 256, 256, 0, s>>>(m, s_dev, 5 * nx, T);
  return hipGetLastError();
}

hipError_t mlp_forward(const float* X, const float* W, int rows, float* H, float* Y, hipStream_t s) {
  k_mlp_fwd<<<rows, MLP_HID, 0, s>>>(X, W, rows, H, Y);
  return hipGetLastError();
}

unsigned mlp_loss_blocks(int rows) { return (unsigned)((rows * MLP_OUT + TB - 1) / TB); }

hipError_t mlp_backward(const float* X, const float* T, const float* W, int rows, const float* H, const float* Y,
                        float* dY, float* dH, float* G, double* lossp, hipStream_t s) {
  k_mlp_dy<<<mlp_loss_blocks(rows), TB, 0, s>>>(Y, T, rows * MLP_OUT, dY, lossp);
  k_mlp_dh<<<rows, MLP_HID, 0, s>>>(dY, W, H, rows, dH);
  k_mlp_wgrad<<<(MLP_WEIGHTS + TB - 1) / TB, TB, 0, s>>>(X, H, dY, dH, rows, G);
  return hipGetLastError();
}

hipError_t mlp_adam(float* W, const float* G, float* Mo, float* Vo, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s) {
  k_adam<<<(MLP_WEIGHTS + TB - 1) / TB, TB, 0, s>>>(W, G, Mo, Vo, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lincoll
