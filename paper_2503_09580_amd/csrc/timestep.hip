// Stage combinations of the classical fourth-order Runge-Kutta scheme used for
// the spatially homogeneous linearized equation df/dt = L[f] (Sec. 4.2, first
// equation pair of that section, RK4 with a fixed step).  The operator
// applications themselves are the library's applies; these kernels only form
//   acc = f + a k (first stage) or acc += a k,   tmp = f + b k,
// and the final f = acc + a k, in double arithmetic on the apply dtype.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace lincoll {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_rk_stage(const T* __restrict__ f, const T* __restrict__ k,
                                                  T* __restrict__ acc, T* __restrict__ tmp, long count, double a,
                                                  double b, int first) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const double kv = (double)k[i], fv = (double)f[i];
    acc[i] = (T)((first ? fv : (double)acc[i]) + a * kv);
    tmp[i] = (T)(fv + b * kv);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_rk_final(T* __restrict__ f, const T* __restrict__ acc,
                                                  const T* __restrict__ k, long count, double a) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
    f[i] = (T)((double)acc[i] + a * (double)k[i]);
}

unsigned blocks_for(long count) {
  const long b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? b : 4096);
}

}  // namespace

hipError_t rk_stage(int dtype, const void* f, const void* k, void* acc, void* tmp, long count, double a, double b,
                    int first, hipStream_t s) {
  if (dtype == 0)
    k_rk_stage<double><<<blocks_for(count), 256, 0, s>>>(static_cast<const double*>(f), static_cast<const double*>(k),
                                                        static_cast<double*>(acc), static_cast<double*>(tmp), count,
                                                        a, b, first);
  else
    k_rk_stage<float><<<blocks_for(count), 256, 0, s>>>(static_cast<const float*>(f), static_cast<const float*>(k),
                                                       static_cast<float*>(acc), static_cast<float*>(tmp), count, a,
                                                       b, first);
  return hipGetLastError();
}

hipError_t rk_final(int dtype, void* f, const void* acc, const void* k, long count, double a, hipStream_t s) {
  if (dtype == 0)
    k_rk_final<double><<<blocks_for(count), 256, 0, s>>>(static_cast<double*>(f), static_cast<const double*>(acc),
                                                        static_cast<const double*>(k), count, a);
  else
    k_rk_final<float><<<blocks_for(count), 256, 0, s>>>(static_cast<float*>(f), static_cast<const float*>(acc),
                                                       static_cast<const float*>(k), count, a);
  return hipGetLastError();
}

}  // namespace lincoll
