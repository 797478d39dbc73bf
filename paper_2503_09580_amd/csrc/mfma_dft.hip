// Split-precision BF16 variant of the gain loop's forward plane transform
// (dtype LINCOLL_BF16X3, staged path, n = 32 and 64): the two in-plane DFT stages of
// DFT[M^h psi_j] (Sec. 3.2, eq. (23); Algorithm 1 loop) run as dense GEMMs on
// the matrix cores, followed by the product with Phi_j and the accumulation of
// L+^.  Everything else of the apply is the FP32 staged path.
//
// n = 32: a complex 32 x 32 plane X is transformed as Y = F X F (F = F^T is the
// forward DFT matrix).  In real form F acts as the 64 x 64 matrix
//   A = [[Fr, -Fi], [Fi, Fr]]  on  [Re; Im]  (64 x 32),
// so each stage is one 64 x 64 x 32 real GEMM: stage 1 multiplies A by
// [Re X; Im X], stage 2 multiplies A by [Re Y1^T; Im Y1^T] (the transpose goes
// through LDS), which yields Y^T.  Operands are split as x = x_hi + x_lo in
// bfloat16, and each product is taken as a_hi b_hi + a_hi b_lo + a_lo b_hi with
// FP32 accumulation (the a_lo b_lo term, of relative size 2^-16, is dropped):
// about 16 significant bits per operand instead of FP32's 24.
//
// Matrix-core shape: v_mfma_f32_32x32x16_bf16, wave64.  Lane l holds
// A[l%32][8(l/32)+v] and B[8(l/32)+v][l%32], v = 0..7, and receives
// D[8(v/4)+4(l/32)+v%4][l%32], v = 0..15.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "twiddles.h"

namespace lincoll {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NN = 32, P = NN / 2 + 1, NP = NN * NN, LD = NN + 1, WAVES = 4;

__device__ __forceinline__ void split(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;                 // round to nearest even
  lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ int fold32(int k) { return k <= NN / 2 ? k : NN - k; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry (m, kk) of the real form of the forward DFT matrix, m, kk < 64.
__device__ __forceinline__ float dft_real_form(int m, int kk) {
  const int e = (2 * (m % NN) * (kk % NN)) & 63;   // exp(-2 pi i mk/32) = TWC[e] - i TWS[e]
  const bool im_row = m >= NN, im_col = kk >= NN;
  if (im_row == im_col) return (float)TWC[e];       // Fr blocks
  return im_col ? (float)TWS[e] : -(float)TWS[e];   // -Fi (upper right), Fi (lower left)
}

// D(64 x 32) = A (64 x 64) B (64 x 32) in split precision; b_hi/b_lo hold this
// lane's B operand for the four k-steps.
__device__ __forceinline__ void gemm64(const bf16x8 (&ah)[2][4], const bf16x8 (&al)[2][4], const bf16x8 (&bh)[4],
                                       const bf16x8 (&bl)[4], f32x16 (&d)[2]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 c = {};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[mt][ks], bh[ks], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mt][ks], bl[ks], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mt][ks], bh[ks], c, 0, 0, 0);
    }
    d[mt] = c;
  }
}

// One wave per plane (cell, kz) of Wq: Lp = (first ? 0 : Lp) + Phi_j * (F Wq F).
__global__ void __launch_bounds__(64 * WAVES) k_plane_fwd_bf16x3(const float2* __restrict__ in,
                                                                 float2* __restrict__ out,
                                                                 const float* __restrict__ table, int j,
                                                                 int nplanes, int first) {
  __shared__ float2 lds[WAVES][NN * LD];
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int col = l % 32, half = l / 32;
  float2* sm = lds[wave];
  // A operand (the DFT matrix in real form), split once per wave
  bf16x8 ah[2][4], al[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        __bf16 h, lo;
        split(dft_real_form(32 * mt + col, 16 * ks + 8 * half + v), h, lo);
        ah[mt][ks][v] = h;
        al[mt][ks][v] = lo;
      }
  const float* tj = table + (size_t)j * phi_stride(NN);
  for (int pid = blockIdx.x * WAVES + wave; pid < nplanes; pid += gridDim.x * WAVES) {
    const int kz = pid % P;
    const float2* X = in + (size_t)pid * NP;
    // stage 1: B = [Re X; Im X], rows kk = 16 ks + 8 half + v
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const float2 x = X[(16 * r + 8 * half + v) * NN + col];
        __bf16 h, lo;
        split(x.x, h, lo);
        bh[r][v] = h;
        bl[r][v] = lo;
        split(x.y, h, lo);
        bh[r + 2][v] = h;
        bl[r + 2][v] = lo;
      }
    f32x16 d[2];
    gemm64(ah, al, bh, bl, d);
    // Y1[i][col], i = 8(v/4) + 4 half + v%4: real part from tile 0, imaginary from tile 1
#pragma unroll
    for (int v = 0; v < 16; ++v) sm[(8 * (v / 4) + 4 * half + v % 4) * LD + col] = float2{d[0][v], d[1][v]};
    wave_sync();
    // stage 2: B = [Re Y1^T; Im Y1^T]: B[kk][n] = Y1[n][kk]
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const float2 y = sm[col * LD + 16 * r + 8 * half + v];
        __bf16 h, lo;
        split(y.x, h, lo);
        bh[r][v] = h;
        bl[r][v] = lo;
        split(y.y, h, lo);
        bh[r + 2][v] = h;
        bl[r + 2][v] = lo;
      }
    wave_sync();
    gemm64(ah, al, bh, bl, d);
    // d holds Y^T: Y[col][i] (first-axis frequency col, second-axis frequency i)
#pragma unroll
    for (int v = 0; v < 16; ++v) sm[col * LD + 8 * (v / 4) + 4 * half + v % 4] = float2{d[0][v], d[1][v]};
    wave_sync();
    // times Phi_j(|k|^2), accumulate; coalesced over the plane
    float2* dst = out + (size_t)pid * NP;
#pragma unroll
    for (int t = 0; t < NP / 64; ++t) {
      const int e = l + 64 * t, k1 = e / NN, k2 = e % NN;
      const int f1 = fold32(k1), f2 = fold32(k2);
      const float m = tj[f1 * f1 + f2 * f2 + kz * kz];
      float2 y = sm[k1 * LD + k2];
      y.x *= m;
      y.y *= m;
      if (!first) {
        const float2 o = dst[e];
        y.x += o.x;
        y.y += o.y;
      }
      dst[e] = y;
    }
    wave_sync();
  }
}

// ----------------------------------------------------------------- n = 64
// The real form of F is 128 x 128 and a plane gives B = [Re X; Im X]
// (128 x 64), too large for one wave's registers.  One four-wave workgroup
// takes a plane: wave w computes rows 32 w .. 32 w + 31 of both stage
// products (M-tile w), with its slice of the split A operand held in
// registers for all planes.  The plane, the stage-1 product and the stage-2
// product pass through LDS as separate real and imaginary 64 x 65 arrays;
// waves 0, 1 write the real rows, waves 2, 3 the imaginary ones.
constexpr int N64 = 64, P64 = N64 / 2 + 1, NP64 = N64 * N64, LD64 = N64 + 1, TB64 = 256;

__device__ __forceinline__ int fold64(int k) { return k <= N64 / 2 ? k : N64 - k; }

// Entry (m, kk) of the real form of the 64-point forward DFT matrix, m, kk < 128.
__device__ __forceinline__ float dft_real_form64(int m, int kk) {
  const int e = ((m % N64) * (kk % N64)) & 63;   // exp(-2 pi i mk/64) = TWC[e] - i TWS[e]
  const bool im_row = m >= N64, im_col = kk >= N64;
  if (im_row == im_col) return (float)TWC[e];
  return im_col ? (float)TWS[e] : -(float)TWS[e];
}

// One 32 x 32 tile of D = A B over K = 128 in split precision.
__device__ __forceinline__ f32x16 gemm_tile128(const bf16x8 (&ah)[8], const bf16x8 (&al)[8], const bf16x8 (&bh)[8],
                                               const bf16x8 (&bl)[8]) {
  f32x16 c = {};
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ks], bh[ks], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ks], bl[ks], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ks], bh[ks], c, 0, 0, 0);
  }
  return c;
}

// B operand of N-tile nt: B[kk][n] = re/im of S[kk % 64][n] (TRANS false) or
// of S[n][kk % 64] (TRANS true), kk = 16 ks + 8 half + v, n = 32 nt + col;
// the real part for kk < 64.
template <bool TRANS>
__device__ __forceinline__ void load_b64(const float* sre, const float* sim, int nt, int col, int half,
                                         bf16x8 (&bh)[8], bf16x8 (&bl)[8]) {
  const int n = 32 * nt + col;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int k = 16 * r + 8 * half + v;
      const int at = TRANS ? n * LD64 + k : k * LD64 + n;
      __bf16 h, lo;
      split(sre[at], h, lo);
      bh[r][v] = h;
      bl[r][v] = lo;
      split(sim[at], h, lo);
      bh[r + 4][v] = h;
      bl[r + 4][v] = lo;
    }
}

// One workgroup per plane (cell, kz) of Wq: Lp = (first ? 0 : Lp) + Phi_j * (F Wq F).
__global__ void __launch_bounds__(TB64) __attribute__((amdgpu_waves_per_eu(2, 2))) k_plane_fwd_bf16x3_64(const float2* __restrict__ in,
                                                              float2* __restrict__ out,
                                                              const float* __restrict__ table, int j, int nplanes,
                                                              int first) {
  __shared__ float sre[N64 * LD64], sim[N64 * LD64];
  const int tid = threadIdx.x, w = tid / 64, l = tid % 64;
  const int col = l % 32, half = l / 32;
  // this wave's rows of A: A[32 w + col][16 ks + 8 half + v]
  bf16x8 ah[8], al[8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      __bf16 h, lo;
      split(dft_real_form64(32 * w + col, 16 * ks + 8 * half + v), h, lo);
      ah[ks][v] = h;
      al[ks][v] = lo;
    }
  float* dst_part = w < 2 ? sre : sim;   // rows 0..63 of a product are real, 64..127 imaginary
  const int row0 = 32 * (w % 2);
  const float* tj = table + (size_t)j * phi_stride(N64);
  for (int pid = blockIdx.x; pid < nplanes; pid += gridDim.x) {
    const int kz = pid % P64;
    const float2* X = in + (size_t)pid * NP64;
#pragma unroll
    for (int t = 0; t < NP64 / TB64; ++t) {
      const int e = tid + TB64 * t;
      const float2 x = X[e];
      sre[(e / N64) * LD64 + e % N64] = x.x;
      sim[(e / N64) * LD64 + e % N64] = x.y;
    }
    __syncthreads();
    // stage 1: [Re Y1; Im Y1] = A [Re X; Im X]
    f32x16 d[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      bf16x8 bh[8], bl[8];
      load_b64<false>(sre, sim, nt, col, half, bh, bl);
      d[nt] = gemm_tile128(ah, al, bh, bl);
    }
    __syncthreads();
    // Y1[k1][c], k1 = row0 + 8(v/4) + 4 half + v%4, c = 32 nt + col
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) dst_part[(row0 + 8 * (v / 4) + 4 * half + v % 4) * LD64 + 32 * nt + col] = d[nt][v];
    __syncthreads();
    // stage 2: [Re Y^T; Im Y^T] = A [Re Y1^T; Im Y1^T]
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      bf16x8 bh[8], bl[8];
      load_b64<true>(sre, sim, nt, col, half, bh, bl);
      d[nt] = gemm_tile128(ah, al, bh, bl);
    }
    __syncthreads();
    // Y[k1][k2] with k1 = 32 nt + col, k2 = row0 + 8(v/4) + 4 half + v%4
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) dst_part[(32 * nt + col) * LD64 + row0 + 8 * (v / 4) + 4 * half + v % 4] = d[nt][v];
    __syncthreads();
    // times Phi_j(|k|^2), accumulate; coalesced over the plane
    float2* dst = out + (size_t)pid * NP64;
#pragma unroll
    for (int t = 0; t < NP64 / TB64; ++t) {
      const int e = tid + TB64 * t, k1 = e / N64, k2 = e % N64;
      const int f1 = fold64(k1), f2 = fold64(k2);
      const float m = tj[f1 * f1 + f2 * f2 + kz * kz];
      float2 y{sre[k1 * LD64 + k2] * m, sim[k1 * LD64 + k2] * m};
      if (!first) {
        const float2 o = dst[e];
        y.x += o.x;
        y.y += o.y;
      }
      dst[e] = y;
    }
    __syncthreads();   // the next plane overwrites the arrays
  }
}

}  // namespace

hipError_t plane_fwd_bf16x3(int n, const float2* in, float2* out, const float* table, int j, int nplanes, int first,
                            int cus, hipStream_t s) {
  if (nplanes < 1) return hipSuccess;
  const int cu = cus > 0 ? cus : 256;
  if (n == 32) {
    const int need = (nplanes + WAVES - 1) / WAVES, cap = cu * 8;
    k_plane_fwd_bf16x3<<<need < cap ? need : cap, 64 * WAVES, 0, s>>>(in, out, table, j, nplanes, first);
  } else if (n == 64) {
    const int cap = cu * 4;
    k_plane_fwd_bf16x3_64<<<nplanes < cap ? nplanes : cap, TB64, 0, s>>>(in, out, table, j, nplanes, first);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lincoll
