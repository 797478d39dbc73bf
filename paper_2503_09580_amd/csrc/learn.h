// Interfaces of the learned-correction kernels (learn.hip).  Every function
// enqueues on stream s; arrays are device memory.
#pragma once
#include <hip/hip_runtime.h>

struct lincoll_mlp_s;

namespace lincoll {

const float* mlp_device_weights(const lincoll_mlp_s* m);   // packed weights on the device

constexpr int MLP_IN = 26, MLP_HID = 128, MLP_OUT = 5;
constexpr int MLP_WEIGHTS = MLP_IN * MLP_HID + MLP_HID + MLP_HID * MLP_OUT + MLP_OUT;

// m[c][a] = h^3 sum (z - b) psi_a / rho_c (b may be null), params [nx][5]
hipError_t ln_hermite(const double* z, const double* b, const double* params, int nx, int n, double L, double* m,
                      hipStream_t s);
// features X [nx][MLP_IN] (float) and the scale *s_dev from m [nx][5]
hipError_t ln_features(const double* m, int nx, float* X, double* s_dev, hipStream_t s);
// out (accumulate: out +=) sum_a s Y[c][a] M_c psi_a
hipError_t ln_correction(const float* Y, const double* s_dev, const double* params, int nx, int n, double L,
                         int accumulate, double* out, hipStream_t s);
// T = m / s (float), 5 nx values
hipError_t ln_targets(const double* m, const double* s_dev, int nx, float* T, hipStream_t s);

// Y = tanh(X W1 + b1) W2 + b2; H (optional) keeps the hidden activations
hipError_t mlp_forward(const float* X, const float* W, int rows, float* H, float* Y, hipStream_t s);
unsigned mlp_loss_blocks(int rows);
// gradient G of mean((Y - T)^2) (Y, H from mlp_forward); lossp: per-block partial sums of (Y - T)^2
hipError_t mlp_backward(const float* X, const float* T, const float* W, int rows, const float* H, const float* Y,
                        float* dY, float* dH, float* G, double* lossp, hipStream_t s);
hipError_t mlp_adam(float* W, const float* G, float* Mo, float* Vo, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s);

}  // namespace lincoll
