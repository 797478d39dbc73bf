// Interfaces between the steady-solver driver (solver.cpp) and its kernels
// (steady.hip).  Every function enqueues on stream s and returns the launch
// status; arrays are device memory.
#pragma once
#include <hip/hip_runtime.h>

namespace lincoll {

constexpr int SUMS_STRIDE = 8;   // doubles per cell in the moment sums
constexpr int GMRES_MAXK = 65;   // largest Krylov basis (restart length 64, plus one)

// Diffuse walls: index 0 = left (x_l), 1 = right (x_r).
struct WallGeom {
  double u[2][3];
  double theta[2];
  double flux_in[2];   // sum v1+ E_L (left) and sum v1- E_R (right), E_W = exp(-|v-u_W|^2/(2 theta_W))
};

unsigned vec_blocks(long N);   // blocks of the vector kernels (rows of their partial-sum buffers)

// Optional gate: when set, a kernel does nothing unless *gate != 0 (device
// flags of the device-resident GMRES below).
hipError_t st_cell_sums(const double* f, int nx, int n, double L, double* sums, hipStream_t s);
hipError_t st_params(const double* sums, int nx, int n, double L, double* params, hipStream_t s);
hipError_t st_wall_sums(const double* x, int nx, int n, double L, double* wall, hipStream_t s,
                        const int* gate = nullptr);
hipError_t st_transport(const double* x, const double* wall, const WallGeom& wg, const void* y, int y_f32,
                        double alpha, const double* ysums, double* out, int nx, int n, double L, double dx,
                        hipStream_t s, const int* gate = nullptr);
// z = (T + diag(nu)/Kn)^-1 y by upwind sweeps (left wall ghost from z, right
// ghost empty); nu: [nx][n^3] in float (nu_f32) or double; wall: scratch.
hipError_t st_sweep(const double* y, double* z, const void* nu, int nu_f32, double* wall, const WallGeom& wg, int nx,
                    int n, double L, double dx, double kn, hipStream_t s, const int* gate = nullptr);
hipError_t st_initial(double* f, int nx, int n, double L, double x_l, double x_r, double theta_l, double theta_r,
                      double C, hipStream_t s);
// out[a] = <V_a, w>, a < k (V: k vectors of N, contiguous); partial: [vec_blocks(N)][GMRES_MAXK]
hipError_t st_mdot(const double* V, long N, int k, const double* w, double* partial, double* out, hipStream_t s,
                   const int* gate = nullptr);
// w -= sum_{a<k} h[a] V_a; *norm2 = |w|^2
hipError_t st_update(double* w, const double* V, long N, int k, const double* h, double* partial, double* norm2,
                     hipStream_t s, const int* gate = nullptr);
// x += sum_{a<k} y[a] V_a
hipError_t st_combine(double* x, const double* V, long N, int k, const double* y, hipStream_t s);
// the same with k and the gate read from device memory
hipError_t st_combine_dev(double* x, const double* V, long N, const int* k, const double* y, const int* gate,
                          hipStream_t s);
// out = a x + b y (y null: out = a x)
hipError_t st_axpby(double* out, double a, const double* x, double b, const double* y, long N, hipStream_t s,
                    const int* gate = nullptr);
// x *= *a (a device scalar)
hipError_t st_scale_dev(double* x, const double* a, long N, const int* gate, hipStream_t s);
// z -= (sum z) * (*ifsum) f, *ifsum = 1 / sum f (sets the total of z to zero
// along f); partial, red: scratch as for st_mdot
hipError_t st_remove_mass(double* z, const double* f, const double* ifsum, long N, double* partial, double* red,
                          hipStream_t s, const int* gate = nullptr);
hipError_t st_to_f32(const double* x, float* y, long N, hipStream_t s, const int* gate = nullptr);
hipError_t st_set(double* dst, double v, hipStream_t s);   // *dst = v on the device

// Device state of restarted flexible GMRES (Givens QR of the Hessenberg
// matrix, residual estimate, flags).  go: the inner solve is still running;
// active: the current cycle's Arnoldi steps still run; pro: the next cycle
// starts with the restart product A x; done: converged, broken down or out of
// its operator budget.
struct GmresState {
  int m, j, iters, budget, mode, go, active, pro, done, pad_;
  double target, beta, resid, inv;
  double cs[GMRES_MAXK], sn[GMRES_MAXK], g[GMRES_MAXK + 1], y[GMRES_MAXK];
  double R[GMRES_MAXK * GMRES_MAXK];
};
// mode 0: start from x = 0 (V0 = b); 1: V0 holds the residual of a given
// start; 2: restart.  iters0 operator applications already spent.
hipError_t gm_init(GmresState* st, int m, double target, int budget, int mode, int iters0, hipStream_t s);
hipError_t gm_v0(double* V0, const double* b, const double* tmp, const GmresState* st, long N, hipStream_t s);
hipError_t gm_begin(GmresState* st, const double* red, hipStream_t s);
hipError_t gm_step(GmresState* st, const double* red, int j, hipStream_t s);
hipError_t gm_end(GmresState* st, hipStream_t s);
hipError_t gm_finish(GmresState* st, hipStream_t s);

}  // namespace lincoll
