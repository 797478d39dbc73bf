// Host side of the learned correction's network (lincoll_mlp_*): weights,
// optimiser state and training buffers on the device, launch orchestration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lincoll.h"
#include "learn.h"

using namespace lincoll;

static_assert(LINCOLL_MLP_WEIGHTS == MLP_WEIGHTS, "packed weight count");

struct lincoll_mlp_s {
  int device = 0;
  hipStream_t stream = nullptr;
  float *d_w = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
  long t = 0;   // Adam steps taken
  int cap = 0;  // rows of the training buffers
  float *d_H = nullptr, *d_Y = nullptr, *d_dY = nullptr, *d_dH = nullptr;
  double* d_loss = nullptr;
};

namespace {

int fail(hipError_t e) { return e == hipErrorOutOfMemory ? LINCOLL_ENOMEM : LINCOLL_EHIP; }

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void free_buffers(lincoll_mlp_s* m) {
  void* ps[] = {m->d_H, m->d_Y, m->d_dY, m->d_dH, m->d_loss};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  m->d_H = m->d_Y = m->d_dY = m->d_dH = nullptr;
  m->d_loss = nullptr;
  m->cap = 0;
}

int ensure(lincoll_mlp_s* m, int rows) {
  if (rows <= m->cap) return LINCOLL_OK;
  free_buffers(m);
  hipError_t e;
  if ((e = hipMalloc(&m->d_H, (size_t)rows * MLP_HID * sizeof(float))) ||
      (e = hipMalloc(&m->d_Y, (size_t)rows * MLP_OUT * sizeof(float))) ||
      (e = hipMalloc(&m->d_dY, (size_t)rows * MLP_OUT * sizeof(float))) ||
      (e = hipMalloc(&m->d_dH, (size_t)rows * MLP_HID * sizeof(float))) ||
      (e = hipMalloc(&m->d_loss, (size_t)mlp_loss_blocks(rows) * sizeof(double))))
    return fail(e);
  m->cap = rows;
  return LINCOLL_OK;
}

// loss of the last backward pass from its per-block partial sums
int read_loss(lincoll_mlp_s* m, int rows, double* loss) {
  std::vector<double> p(mlp_loss_blocks(rows));
  hipError_t e;
  if ((e = hipMemcpyAsync(p.data(), m->d_loss, p.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream)) ||
      (e = hipStreamSynchronize(m->stream)))
    return fail(e);
  double s = 0.0;
  for (double v : p) s += v;
  *loss = s / ((double)rows * MLP_OUT);
  return LINCOLL_OK;
}

}  // namespace

namespace lincoll {
const float* mlp_device_weights(const lincoll_mlp_s* m) { return m->d_w; }
}  // namespace lincoll

extern "C" {

int lincoll_mlp_create(unsigned long long seed, lincoll_mlp_t* out) {
  if (!out) return LINCOLL_EINVAL;
  *out = nullptr;
  lincoll_mlp_s* m = new (std::nothrow) lincoll_mlp_s();
  if (!m) return LINCOLL_ENOMEM;
  std::vector<float> w(MLP_WEIGHTS, 0.0f);
  uint64_t st = seed;
  const double a1 = std::sqrt(6.0 / (MLP_IN + MLP_HID)), a2 = std::sqrt(6.0 / (MLP_HID + MLP_OUT));
  auto uni = [&](double a) { return (float)(a * (2.0 * ((splitmix64(st) >> 11) * 0x1.0p-53) - 1.0)); };
  for (int i = 0; i < MLP_IN * MLP_HID; ++i) w[i] = uni(a1);
  for (int i = 0; i < MLP_HID * MLP_OUT; ++i) w[MLP_IN * MLP_HID + MLP_HID + i] = uni(a2);
  hipError_t e;
  const size_t b = MLP_WEIGHTS * sizeof(float);
  if ((e = hipGetDevice(&m->device)) || (e = hipMalloc(&m->d_w, b)) || (e = hipMalloc(&m->d_m, b)) ||
      (e = hipMalloc(&m->d_v, b)) || (e = hipMalloc(&m->d_g, b)) ||
      (e = hipMemcpy(m->d_w, w.data(), b, hipMemcpyHostToDevice)) || (e = hipMemset(m->d_m, 0, b)) ||
      (e = hipMemset(m->d_v, 0, b))) {
    lincoll_mlp_destroy(m);
    return fail(e);
  }
  *out = m;
  return LINCOLL_OK;
}

void lincoll_mlp_destroy(lincoll_mlp_t m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  free_buffers(m);
  void* ps[] = {m->d_w, m->d_m, m->d_v, m->d_g};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  delete m;
}

int lincoll_mlp_set_stream(lincoll_mlp_t m, void* s) {
  if (!m) return LINCOLL_EINVAL;
  m->stream = static_cast<hipStream_t>(s);
  return LINCOLL_OK;
}

int lincoll_mlp_weights(lincoll_mlp_t m, float* w, long long count, int write) {
  if (!m || !w || count != MLP_WEIGHTS || (write != 0 && write != 1)) return LINCOLL_EINVAL;
  const size_t b = MLP_WEIGHTS * sizeof(float);
  hipError_t e;
  if (write) {
    if ((e = hipMemcpyAsync(m->d_w, w, b, hipMemcpyHostToDevice, m->stream)) ||
        (e = hipMemsetAsync(m->d_m, 0, b, m->stream)) || (e = hipMemsetAsync(m->d_v, 0, b, m->stream)))
      return fail(e);
    m->t = 0;
  } else if ((e = hipMemcpyAsync(w, m->d_w, b, hipMemcpyDeviceToHost, m->stream))) {
    return fail(e);
  }
  if ((e = hipStreamSynchronize(m->stream))) return fail(e);
  return LINCOLL_OK;
}

int lincoll_mlp_forward(lincoll_mlp_t m, const float* X, float* Y, int rows) {
  if (!m || !X || !Y || rows < 1) return LINCOLL_EINVAL;
  hipError_t e = mlp_forward(X, m->d_w, rows, nullptr, Y, m->stream);
  return e ? fail(e) : LINCOLL_OK;
}

int lincoll_mlp_loss_grad(lincoll_mlp_t m, const float* X, const float* T, int rows, float* grad, double* loss) {
  if (!m || !X || !T || rows < 1) return LINCOLL_EINVAL;
  int st = ensure(m, rows);
  if (st) return st;
  hipError_t e;
  if ((e = mlp_forward(X, m->d_w, rows, m->d_H, m->d_Y, m->stream)) ||
      (e = mlp_backward(X, T, m->d_w, rows, m->d_H, m->d_Y, m->d_dY, m->d_dH, grad ? grad : m->d_g, m->d_loss,
                        m->stream)))
    return fail(e);
  if (loss) return read_loss(m, rows, loss);
  if ((e = hipStreamSynchronize(m->stream))) return fail(e);
  return LINCOLL_OK;
}

int lincoll_mlp_train(lincoll_mlp_t m, const float* X, const float* T, int rows, int steps, double lr, double* loss) {
  if (!m || !X || !T || rows < 1 || steps < 0 || !(lr > 0.0)) return LINCOLL_EINVAL;
  int st = ensure(m, rows);
  if (st) return st;
  const double b1 = 0.9, b2 = 0.999;
  hipError_t e;
  for (int i = 0; i < steps; ++i) {
    ++m->t;
    const double c1 = 1.0 / (1.0 - std::pow(b1, (double)m->t)), c2 = 1.0 / (1.0 - std::pow(b2, (double)m->t));
    if ((e = mlp_forward(X, m->d_w, rows, m->d_H, m->d_Y, m->stream)) ||
        (e = mlp_backward(X, T, m->d_w, rows, m->d_H, m->d_Y, m->d_dY, m->d_dH, m->d_g, m->d_loss, m->stream)) ||
        (e = mlp_adam(m->d_w, m->d_g, m->d_m, m->d_v, (float)lr, (float)b1, (float)b2, 1e-8f, (float)c1, (float)c2,
                      m->stream)))
      return fail(e);
  }
  if (loss && steps > 0) return read_loss(m, rows, loss);
  if ((e = hipStreamSynchronize(m->stream))) return fail(e);
  return LINCOLL_OK;
}

}  // extern "C"
