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

hipError_t st_cell_sums(const double* f, int nx, int n, double L, double* sums, hipStream_t s);
hipError_t st_params(const double* sums, int nx, int n, double L, double* params, hipStream_t s);
hipError_t st_wall_sums(const double* x, int nx, int n, double L, double* wall, hipStream_t s);
hipError_t st_transport(const double* x, const double* wall, const WallGeom& wg, const void* y, int y_f32,
                        double alpha, const double* ysums, double* out, int nx, int n, double L, double dx,
                        hipStream_t s);
// z = (T + diag(nu)/Kn)^-1 y by upwind sweeps (left wall ghost from z, right
// ghost empty); nu: [nx][n^3] in float (nu_f32) or double; wall: scratch.
hipError_t st_sweep(const double* y, double* z, const void* nu, int nu_f32, double* wall, const WallGeom& wg, int nx,
                    int n, double L, double dx, double kn, hipStream_t s);
hipError_t st_initial(double* f, int nx, int n, double L, double x_l, double x_r, double theta_l, double theta_r,
                      double C, hipStream_t s);
// out[a] = <V_a, w>, a < k (V: k vectors of N, contiguous); partial: [vec_blocks(N)][GMRES_MAXK]
hipError_t st_mdot(const double* V, long N, int k, const double* w, double* partial, double* out, hipStream_t s);
// w -= sum_{a<k} h[a] V_a; *norm2 = |w|^2
hipError_t st_update(double* w, const double* V, long N, int k, const double* h, double* partial, double* norm2,
                     hipStream_t s);
// x += sum_{a<k} y[a] V_a
hipError_t st_combine(double* x, const double* V, long N, int k, const double* y, hipStream_t s);
// out = a x + b y (y null: out = a x)
hipError_t st_axpby(double* out, double a, const double* x, double b, const double* y, long N, hipStream_t s);
// z -= (sum z / fsum) f, fsum = sum f (sets the total of z to zero along f);
// partial, red: scratch as for st_mdot
hipError_t st_remove_mass(double* z, const double* f, double fsum, long N, double* partial, double* red,
                          hipStream_t s);
hipError_t st_to_f32(const double* x, float* y, long N, hipStream_t s);

}  // namespace lincoll
