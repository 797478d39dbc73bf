// Steady 1-D problem with diffuse walls (Sec. 5, Appendix B): residual,
// modified Newton operator and the modified Newton iteration with restarted
// flexible GMRES as the inner solver.  Host orchestration of device work: the
// operator applications are the library's own (quadcoll_apply for the
// residual, the linearized apply with the invariant projection inside the
// Newton operator) and the remaining steps are the kernels of steady.hip.
// GMRES keeps its bookkeeping on the device (steady.h, GmresState): a whole
// restart cycle is one fixed sequence of launches, gated by device flags once
// the cycle has converged, recorded into a hipGraph once per solve and
// replayed (LINCOLL_OPT_GRAPH), with one host read of the state per cycle.
// Work memory belongs to the plan and is kept between calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "../../include/lincoll.h"
#include "internal.h"
#include "learn.h"
#include "steady.h"

using namespace lincoll;

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

#define HIPCK(x)                                                             \
  do {                                                                       \
    const hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                                  \
      plan_note_hip(pl, e_);                                                 \
      return e_ == hipErrorOutOfMemory ? LINCOLL_ENOMEM : LINCOLL_EHIP;      \
    }                                                                        \
  } while (0)
#define STCK(x)                 \
  do {                          \
    const int s_ = (x);         \
    if (s_ != LINCOLL_OK) return s_; \
  } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_params(const lincoll_steady_params_t* sp) {
  if (!sp || sp->nx < 1) return LINCOLL_EINVAL;
  if (!std::isfinite(sp->x_l) || !std::isfinite(sp->x_r) || !(sp->x_l < sp->x_r)) return LINCOLL_EINVAL;
  if (!finite_pos(sp->kn) || !finite_pos(sp->mass) || !finite_pos(sp->theta_l) || !finite_pos(sp->theta_r))
    return LINCOLL_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(sp->u_l[d]) || !std::isfinite(sp->u_r[d])) return LINCOLL_EINVAL;
  if (!(sp->tol >= 0.0) || !(sp->inner_rtol >= 0.0) || !(sp->inner_atol >= 0.0)) return LINCOLL_EINVAL;
  if (sp->max_newton < 0 || sp->max_inner < 1 || sp->restart < 1 || sp->restart > GMRES_MAXK - 1)
    return LINCOLL_EINVAL;
  if (sp->init != 0 && sp->init != 1) return LINCOLL_EINVAL;
  if (sp->precond != LINCOLL_PRECOND_NONE && sp->precond != LINCOLL_PRECOND_SWEEP &&
      sp->precond != LINCOLL_PRECOND_LEARNED)
    return LINCOLL_EINVAL;
  if (sp->precond == LINCOLL_PRECOND_LEARNED && !sp->mlp) return LINCOLL_EINVAL;
  if ((sp->rec_X == nullptr) != (sp->rec_T == nullptr) || sp->rec_cap < 0) return LINCOLL_EINVAL;
  if (sp->inner != LINCOLL_INNER_GMRES && sp->inner != LINCOLL_INNER_SOURCE) return LINCOLL_EINVAL;
  if (sp->backtrack != 0 && sp->backtrack != 1) return LINCOLL_EINVAL;
  return LINCOLL_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

struct Solver {
  lincoll_plan_t pl = nullptr;
  hipStream_t s = nullptr;
  lincoll_steady_params_t sp{};
  int n = 0, nx = 0, dtype = 0;
  long n3 = 0, N = 0;
  double L = 0.0, hv = 0.0, h3 = 0.0, dx = 0.0, wnorm = 0.0;   // wnorm = sqrt(dx h_v^3)
  WallGeom wg{};
  int project_before = 0;
  const double* f_cur = nullptr;   // iterate whose local Maxwellians are set
  double f_sum = 0.0;              // its plain sum (mass / (dx h^3))
  bool project_set = false;
  long matvecs = 0;
  // Work memory carved from the plan's steady-solver buffer.
  char* carve_at = nullptr;
  size_t carve_left = 0;
  // small buffers
  double *d_sums = nullptr, *d_ysums = nullptr, *d_params = nullptr, *d_wall = nullptr;
  double *d_partial = nullptr, *d_red = nullptr, *d_y = nullptr, *d_ifsum = nullptr;
  GmresState* d_gm = nullptr;
  // learned correction: moments, scale, features, network output
  double *d_m5 = nullptr, *d_scale = nullptr;
  float *d_X = nullptr, *d_Y = nullptr;
  int rec_rows = 0;
  // fields of N values
  double* d_q = nullptr;     // Q(f, f)
  double* d_aux = nullptr;   // a spare field (lincoll_steady_residual without an output)
  void* d_in = nullptr;      // apply input (plan dtype)
  void* d_o = nullptr;       // apply output (plan dtype)
  // solve only: residual, correction, restart scratch, Krylov bases
  double *d_r = nullptr, *d_g = nullptr, *d_tmp = nullptr, *d_V = nullptr, *d_Z = nullptr;
  // the recorded GMRES cycle of this solve (LINCOLL_OPT_GRAPH)
  hipGraphExec_t cycle = nullptr;

  ~Solver() {
    if (pl) (void)hipStreamSynchronize(s);   // work may still read the plan's buffers
    if (cycle) (void)hipGraphExecDestroy(cycle);
    if (project_set) (void)lincoll_set_option(pl, LINCOLL_OPT_PROJECT, project_before);
  }

  static size_t rnd(size_t b) { return (b + 255) / 256 * 256; }

  template <typename P>
  void carve(P** p, size_t bytes) {
    *p = reinterpret_cast<P*>(carve_at);
    carve_at += rnd(bytes);
    carve_left -= rnd(bytes);
  }

  int init(lincoll_plan_t plan, const lincoll_steady_params_t* params, bool full = false) {
    pl = plan;
    if (!pl) return LINCOLL_EINVAL;
    STCK(check_params(params));
    sp = *params;
    double v;
    STCK(lincoll_get_info(pl, LINCOLL_INFO_N, &v));
    n = (int)v;
    if (n != 8 && n != 16 && n != 32) return LINCOLL_ENOTIMPL;   // the residual's binary operator
    STCK(lincoll_get_info(pl, LINCOLL_INFO_DTYPE, &v));
    dtype = (int)v;
    STCK(lincoll_get_info(pl, LINCOLL_INFO_L, &v));
    L = v;
    STCK(lincoll_get_info(pl, LINCOLL_INFO_PROJECT, &v));
    project_before = (int)v;
    s = plan_stream(pl);
    nx = sp.nx;
    n3 = (long)n * n * n;
    N = (long)nx * n3;
    hv = 2.0 * L / n;
    h3 = hv * hv * hv;
    dx = (sp.x_r - sp.x_l) / nx;
    wnorm = std::sqrt(dx * h3);
    // walls: shapes E_W and the incoming-flux normalisations sum v1+ E_L, sum v1- E_R
    const double* us[2] = {sp.u_l, sp.u_r};
    const double th[2] = {sp.theta_l, sp.theta_r};
    for (int w = 0; w < 2; ++w) {
      for (int d = 0; d < 3; ++d) wg.u[w][d] = us[w][d];
      wg.theta[w] = th[w];
      double acc = 0.0;
      for (int i1 = 0; i1 < n; ++i1) {
        const double v1 = -L + i1 * hv;
        if (w == 0 ? !(v1 > 0.0) : !(v1 < 0.0)) continue;
        for (int i2 = 0; i2 < n; ++i2)
          for (int i3 = 0; i3 < n; ++i3) {
            const double a = v1 - us[w][0], b = -L + i2 * hv - us[w][1], c = -L + i3 * hv - us[w][2];
            acc += v1 * std::exp(-(a * a + b * b + c * c) / (2.0 * th[w]));
          }
      }
      if (acc == 0.0) return LINCOLL_EINVAL;
      wg.flux_in[w] = acc;
    }
    // one block of plan memory for everything this call needs
    const size_t nb = vec_blocks(N), es = dtype == LINCOLL_F64 ? sizeof(double) : sizeof(float);
    const size_t vec = (size_t)N * sizeof(double);
    const size_t sizes[] = {(size_t)nx * SUMS_STRIDE * 8, (size_t)nx * SUMS_STRIDE * 8, (size_t)nx * 5 * 8, 8 * 8,
                            nb * GMRES_MAXK * 8, (GMRES_MAXK + 1) * 8, GMRES_MAXK * 8, 8, sizeof(GmresState),
                            (size_t)nx * 5 * 8, 8, (size_t)nx * MLP_IN * 4, (size_t)nx * MLP_OUT * 4,
                            vec, vec, (size_t)N * es, (size_t)N * es};
    size_t total = 0;
    for (size_t b : sizes) total += rnd(b);
    if (full) total += rnd(vec) * (3 + 2 * (size_t)sp.restart + 1);
    int st = LINCOLL_OK;
    carve_at = static_cast<char*>(plan_steady_work(pl, total, &st));
    if (!carve_at) return st;
    carve_left = total;
    carve(&d_sums, sizes[0]);
    carve(&d_ysums, sizes[1]);
    carve(&d_params, sizes[2]);
    carve(&d_wall, sizes[3]);
    carve(&d_partial, sizes[4]);
    carve(&d_red, sizes[5]);
    carve(&d_y, sizes[6]);
    carve(&d_ifsum, sizes[7]);
    carve(&d_gm, sizes[8]);
    carve(&d_m5, sizes[9]);
    carve(&d_scale, sizes[10]);
    carve(&d_X, sizes[11]);
    carve(&d_Y, sizes[12]);
    carve(&d_q, sizes[13]);
    carve(&d_aux, sizes[14]);
    carve(&d_in, sizes[15]);
    carve(&d_o, sizes[16]);
    if (full) {
      carve(&d_r, vec);
      carve(&d_g, vec);
      carve(&d_tmp, vec);
      carve(&d_V, vec * (sp.restart + 1));
      carve(&d_Z, vec * sp.restart);
    }
    return LINCOLL_OK;
  }

  int host_copy(void* dst, const void* src, size_t bytes) {
    HIPCK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    return LINCOLL_OK;
  }

  // plain dot product <a, b> on the host
  int dot(const double* a, const double* b, double* out) {
    HIPCK(st_mdot(a, N, 1, b, d_partial, d_red, s));
    return host_copy(out, d_red, sizeof(double));
  }

  // r = T[f] - (Q(f,f) - mean Q)/Kn; *norm = sqrt(dx h^3 |r|^2)
  int residual(const double* f, double* r, double* norm) {
    STCK(quadcoll_apply(pl, f, d_q, nx));
    HIPCK(st_cell_sums(d_q, nx, n, L, d_ysums, s));
    HIPCK(st_wall_sums(f, nx, n, L, d_wall, s));
    HIPCK(st_transport(f, d_wall, wg, d_q, 0, -1.0 / sp.kn, d_ysums, r, nx, n, L, dx, s));
    if (norm) {
      double v = 0.0;
      STCK(dot(r, r, &v));
      *norm = std::sqrt(v) * wnorm;
    }
    return LINCOLL_OK;
  }

  // d_params <- local Maxwellian parameters of f
  int local_params(const double* f) {
    HIPCK(st_cell_sums(f, nx, n, L, d_sums, s));
    HIPCK(st_params(d_sums, nx, n, L, d_params, s));
    return LINCOLL_OK;
  }

  // Maxwellians of the plan <- local Maxwellians of f (checked on the host)
  int set_local(const double* f) {
    STCK(local_params(f));
    std::vector<double> hp((size_t)nx * 5);
    STCK(host_copy(hp.data(), d_params, hp.size() * sizeof(double)));
    f_cur = f;
    f_sum = 0.0;
    for (int c = 0; c < nx; ++c) f_sum += hp[(size_t)c * 5] / h3;
    HIPCK(st_set(d_ifsum, 1.0 / f_sum, s));
    for (int c = 0; c < nx; ++c) {
      const double* q = &hp[(size_t)c * 5];
      if (!finite_pos(q[0]) || !finite_pos(q[4]) || !std::isfinite(q[1]) || !std::isfinite(q[2]) ||
          !std::isfinite(q[3]))
        return LINCOLL_EDIVERGED;
    }
    STCK(lincoll_set_maxwellians(pl, d_params, nx));
    if (!project_set) {
      STCK(lincoll_set_option(pl, LINCOLL_OPT_PROJECT, 1));
      project_set = true;
    }
    return LINCOLL_OK;
  }

  // out = T[x] - P L P x / Kn about the Maxwellians set by set_local; with a
  // gate, nothing is written unless *gate != 0 (on the staged path the
  // linearized apply itself still runs)
  int matvec(const double* x, double* out, const int* gate = nullptr) {
    if (dtype == LINCOLL_F64)
      HIPCK(st_axpby(static_cast<double*>(d_in), 1.0, x, 0.0, nullptr, N, s, gate));
    else
      HIPCK(st_to_f32(x, static_cast<float*>(d_in), N, s, gate));
    STCK(plan_apply_on(pl, d_in, d_o, nx, s, gate));
    HIPCK(st_wall_sums(x, nx, n, L, d_wall, s, gate));
    HIPCK(st_transport(x, d_wall, wg, d_o, dtype != LINCOLL_F64, -1.0 / sp.kn, nullptr, out, nx, n, L, dx, s, gate));
    if (!gate) ++matvecs;
    return LINCOLL_OK;
  }

  // rescales f to the discrete mass C; *mass_before receives its mass before
  int constrain(double* f, double* mass_before) {
    HIPCK(st_cell_sums(f, nx, n, L, d_sums, s));
    std::vector<double> hs((size_t)nx * SUMS_STRIDE);
    STCK(host_copy(hs.data(), d_sums, hs.size() * sizeof(double)));
    double m = 0.0;
    for (int c = 0; c < nx; ++c) m += hs[(size_t)c * SUMS_STRIDE];
    m *= dx * h3;
    if (mass_before) *mass_before = m;
    if (!finite_pos(m)) return LINCOLL_EDIVERGED;
    HIPCK(st_axpby(f, sp.mass / m, f, 0.0, nullptr, N, s));
    return LINCOLL_OK;
  }

  // The Newton operator maps onto zero-mass fields and is singular along one
  // direction of non-zero mass (the steady state's mass mode), so a
  // zero-mass right-hand side has a unique zero-mass solution.  Keeping every
  // preconditioned vector at zero mass (removing its total along the current
  // iterate f) keeps the inner solution on it: the correction is then well
  // defined (and learnable) and the Newton update preserves the mass.
  int zero_mass(double* z, const int* gate = nullptr) {
    HIPCK(st_remove_mass(z, f_cur, d_ifsum, N, d_partial, d_red, s, gate));
    return LINCOLL_OK;
  }

  // Absolute inner stop, never above 1 % of the Newton tolerance (an inner
  // solve stopped above the outer tolerance would stall the iteration there).
  double inner_atol() const { return std::min(sp.inner_atol, 0.01 * sp.tol); }

  // z = M^-1 v, the right preconditioner (z = v without one)
  int precondition(const double* v, double* z, const int* gate = nullptr) {
    if (sp.precond == LINCOLL_PRECOND_NONE) {
      HIPCK(st_axpby(z, 1.0, v, 0.0, nullptr, N, s, gate));
      return LINCOLL_OK;
    }
    HIPCK(st_sweep(v, z, plan_nu(pl), dtype != LINCOLL_F64, d_wall, wg, nx, n, L, dx, sp.kn, s, gate));
    return zero_mass(z, gate);
  }

  // features of z (about d_params) into X, scale into d_scale
  int features(const double* z, float* X) {
    HIPCK(ln_hermite(z, nullptr, d_params, nx, n, L, d_m5, s));
    HIPCK(ln_features(d_m5, nx, X, d_scale, s));
    return LINCOLL_OK;
  }

  // Learned start of an inner solve: z = sweep(b), Delta = correction of
  // mlp(features(z)); x0 = a z + alpha Delta with (a, alpha) minimising
  // |b - A x0| (two operator applications), so the start is never worse in
  // residual than zero or the sweep alone.  On return x0 holds the start and
  // V[0] its residual b - A x0; Z[0] and V[1] are used as scratch.
  int learned_start(const double* b, double* x0, double* V, double* Z) {
    double *D = Z, *Az = V, *AD = V + N;
    STCK(precondition(b, x0));
    STCK(features(x0, d_X));
    HIPCK(mlp_forward(d_X, mlp_device_weights(sp.mlp), nx, nullptr, d_Y, s));
    HIPCK(ln_correction(d_Y, d_scale, d_params, nx, n, L, 0, D, s));
    STCK(zero_mass(D));
    STCK(matvec(x0, Az));
    STCK(matvec(D, AD));
    double g[4];
    HIPCK(st_mdot(V, N, 2, AD, d_partial, d_red, s));       // <Az,AD>, <AD,AD>
    STCK(host_copy(g, d_red, 2 * sizeof(double)));
    HIPCK(st_mdot(V, N, 1, Az, d_partial, d_red, s));       // <Az,Az>
    STCK(host_copy(g + 2, d_red, sizeof(double)));
    double rb[2];
    HIPCK(st_mdot(V, N, 2, b, d_partial, d_red, s));        // <Az,b>, <AD,b>
    STCK(host_copy(rb, d_red, 2 * sizeof(double)));
    const double a11 = g[2], a12 = g[0], a22 = g[1], det = a11 * a22 - a12 * a12;
    double a = 0.0, al = 0.0;
    if (det > 1e-14 * a11 * a22) {
      a = (rb[0] * a22 - rb[1] * a12) / det;
      al = (a11 * rb[1] - a12 * rb[0]) / det;
    } else if (a11 > 0.0) {
      a = rb[0] / a11;
    }
    if (!std::isfinite(a) || !std::isfinite(al)) a = al = 0.0;
    if (al == 0.0) {
      // the network's term is dropped (also when its output is not finite:
      // 0 * NaN would still poison the start), leaving the scaled sweep
      HIPCK(st_axpby(x0, a, x0, 0.0, nullptr, N, s));
      HIPCK(st_axpby(V, -a, V, 1.0, b, N, s));              // V0 = b - a Az
      return LINCOLL_OK;
    }
    HIPCK(st_axpby(x0, a, x0, al, D, N, s));
    HIPCK(st_axpby(V, -a, V, 1.0, b, N, s));                // V0 = b - a Az
    HIPCK(st_axpby(V, 1.0, V, -al, AD, N, s));              //      - alpha A Delta
    return LINCOLL_OK;
  }

  // appends nx training rows: features of z = sweep(b), targets m(g - z)/s
  int record(const double* b, const double* g, double* z) {
    if (!sp.rec_X || rec_rows + nx > sp.rec_cap) return LINCOLL_OK;
    STCK(precondition(b, z));
    STCK(features(z, sp.rec_X + (size_t)rec_rows * MLP_IN));
    HIPCK(ln_hermite(g, z, d_params, nx, n, L, d_m5, s));
    HIPCK(ln_targets(d_m5, d_scale, nx, sp.rec_T + (size_t)rec_rows * MLP_OUT, s));
    rec_rows += nx;
    return LINCOLL_OK;
  }

  // Restarted flexible GMRES for A x = b from x = 0 with right
  // preconditioning (A M^-1 u = b, x = M^-1 u; the preconditioned vectors Z
  // are kept, so M may change between iterations) and classical Gram-Schmidt.
  // Stops when the weighted residual <= max(inner_rtol |b|, inner_atol) or
  // after max_inner operator evaluations.  V: (restart + 1) vectors, Z:
  // restart vectors, tmp: one.
  // Source iteration (Sec. 5.2, eq. (source_iteration)): x <- x + M^-1 (b - A x) from x = 0, M^-1 the
  // zero-mass sweep; stops like gmres.  w, z: scratch vectors.
  int source_iteration(const double* b, double bnorm, double* x, double* w, double* z, int* iters) {
    const double target = std::max(sp.inner_rtol * bnorm * wnorm, inner_atol()) / wnorm;   // plain norm
    const long start = matvecs;
    *iters = 0;
    HIPCK(hipMemsetAsync(x, 0, (size_t)N * sizeof(double), s));
    if (!(bnorm > target)) return LINCOLL_OK;
    HIPCK(st_axpby(w, 1.0, b, 0.0, nullptr, N, s));            // w = b - A x with x = 0
    for (;;) {
      HIPCK(st_sweep(w, z, plan_nu(pl), dtype != LINCOLL_F64, d_wall, wg, nx, n, L, dx, sp.kn, s));
      STCK(zero_mass(z));
      HIPCK(st_axpby(x, 1.0, x, 1.0, z, N, s));
      STCK(matvec(x, w));
      HIPCK(st_axpby(w, 1.0, b, -1.0, w, N, s));
      double rr = 0.0;
      STCK(dot(w, w, &rr));
      const double res = std::sqrt(rr);
      if (!std::isfinite(res)) break;
      if (res <= target || matvecs - start >= sp.max_inner) break;
    }
    *iters = (int)(matvecs - start);
    return LINCOLL_OK;
  }

  // One restart cycle of flexible GMRES, as a fixed sequence of launches on s:
  // the restart product and V0, then `restart` Arnoldi steps (preconditioner,
  // operator, classical Gram-Schmidt, Givens update on the device), the back
  // substitution and x += Z y.  Device flags make the launches after
  // convergence (or of a finished solve) return at once.
  int cycle_launches(const double* b, double* x, double* V, double* Z, double* tmp) {
    const int m = sp.restart;
    const int* go = &d_gm->go;
    const int* act = &d_gm->active;
    STCK(matvec(x, tmp, &d_gm->pro));
    HIPCK(gm_v0(V, b, tmp, d_gm, N, s));
    HIPCK(st_mdot(V, N, 1, V, d_partial, d_red, s, go));
    HIPCK(gm_begin(d_gm, d_red, s));
    HIPCK(st_scale_dev(V, &d_gm->inv, N, act, s));
    for (int j = 0; j < m; ++j) {
      double* w = V + (long)(j + 1) * N;
      double* zj = Z + (long)j * N;
      STCK(precondition(V + (long)j * N, zj, act));
      STCK(matvec(zj, w, act));
      HIPCK(st_mdot(V, N, j + 1, w, d_partial, d_red, s, act));
      HIPCK(st_update(w, V, N, j + 1, d_red, d_partial, d_red + (j + 1), s, act));
      HIPCK(gm_step(d_gm, d_red, j, s));
      HIPCK(st_scale_dev(w, &d_gm->inv, N, act, s));
    }
    HIPCK(gm_end(d_gm, s));
    HIPCK(st_combine_dev(x, Z, N, &d_gm->j, d_gm->y, go, s));
    HIPCK(gm_finish(d_gm, s));
    return LINCOLL_OK;
  }

  // Runs one cycle: replays the recorded graph (recording it on first use,
  // on a stream the plan owns) or launches the same sequence directly.
  int run_cycle(const double* b, double* x, double* V, double* Z, double* tmp) {
    if (!plan_graph_option(pl)) return cycle_launches(b, x, V, Z, tmp);
    if (!cycle) {
      hipStream_t cap = nullptr, s0 = s;
      HIPCK(plan_capture_stream(pl, &cap));
      HIPCK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      s = cap;
      const int st = cycle_launches(b, x, V, Z, tmp);
      s = s0;
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(cap, &g);
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (!e) e = hipGraphInstantiate(&cycle, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e) cycle = nullptr;
      HIPCK(e);
    }
    HIPCK(hipGraphLaunch(cycle, s));
    return LINCOLL_OK;
  }

  // Restarted flexible GMRES for A x = b with right preconditioning
  // (A M^-1 u = b, x = M^-1 u; the preconditioned vectors Z are kept, so M
  // may change between iterations) and classical Gram-Schmidt.  Stops when
  // the weighted residual <= max(inner_rtol |b|, inner_atol) or after
  // max_inner operator evaluations.  Without x0, x starts at 0; with x0, x
  // holds the start and V[0] its residual b - A x (the tolerance stays
  // relative to |b|), and `spent` operator evaluations count against the
  // budget.  V: restart + 1 vectors, Z: restart vectors, tmp: one.
  int gmres(const double* b, double bnorm, double* x, double* V, double* Z, double* tmp, int* iters, bool x0 = false,
            int spent = 0) {
    const double target = std::max(sp.inner_rtol * bnorm * wnorm, inner_atol()) / wnorm;   // plain norm
    STCK(plan_ensure_work(pl, nx));   // no allocation may happen while a cycle is recorded
    if (!x0) HIPCK(hipMemsetAsync(x, 0, (size_t)N * sizeof(double), s));
    HIPCK(gm_init(d_gm, sp.restart, target, sp.max_inner, x0 ? 1 : 0, spent, s));
    GmresState h;
    for (;;) {
      STCK(run_cycle(b, x, V, Z, tmp));
      HIPCK(hipMemcpyAsync(&h, d_gm, offsetof(GmresState, cs), hipMemcpyDeviceToHost, s));
      HIPCK(hipStreamSynchronize(s));
      if (!h.go) break;
    }
    *iters = h.iters;
    matvecs += h.iters - spent;
    return LINCOLL_OK;
  }

  int solve(double* f, lincoll_steady_report_t* rep) {
    const clk::time_point t0 = clk::now();
    lincoll_steady_report_t rp;
    std::memset(&rp, 0, sizeof(rp));
    double *r = d_r, *gcor = d_g, *V = d_V, *Z = d_Z, *tmp = d_tmp;
    if (sp.init) HIPCK(st_initial(f, nx, n, L, sp.x_l, sp.x_r, sp.theta_l, sp.theta_r, sp.mass, s));
    int status = constrain(f, nullptr);
    double res_prev = 0.0, lambda = 1.0;
    for (int k = 0; status == LINCOLL_OK;) {
      clk::time_point t = clk::now();
      double res = 0.0;
      if ((status = residual(f, r, &res))) break;
      rp.ms_residual += ms_since(t);
      if (!std::isfinite(res)) {
        status = LINCOLL_EDIVERGED;
        break;
      }
      // backtracking: a step that did not lower the residual is halved
      // (f = f_prev - lambda g), at most three times
      if (sp.backtrack && k > 0 && !(res < res_prev) && !(res < sp.tol) && lambda > 0.125) {
        lambda *= 0.5;
        if (hipError_t e = st_axpby(f, 1.0, f, lambda, gcor, N, s)) {
          plan_note_hip(pl, e);
          status = LINCOLL_EHIP;
          break;
        }
        ++rp.backtracks;
        status = constrain(f, nullptr);
        continue;
      }
      if (k <= 64) rp.res_history[k] = res;
      rp.residual = res;
      if (res < sp.tol) {
        rp.converged = 1;
        break;
      }
      if (k == sp.max_newton) break;
      res_prev = res;
      lambda = 1.0;
      t = clk::now();
      int its = 0;
      const bool learned = sp.inner == LINCOLL_INNER_GMRES && sp.precond == LINCOLL_PRECOND_LEARNED;
      const long mv0 = matvecs;
      if ((status = set_local(f))) break;
      if (sp.inner == LINCOLL_INNER_SOURCE) {
        if ((status = source_iteration(r, res / wnorm, gcor, V, V + N, &its))) break;
      } else if ((learned && (status = learned_start(r, gcor, V, Z))) ||
                 (status = gmres(r, res / wnorm, gcor, V, Z, tmp, &its, learned, (int)(matvecs - mv0)))) {
        break;
      }
      if ((status = record(r, gcor, tmp))) break;
      rp.ms_inner += ms_since(t);
      if (k < 64) rp.inner_history[k] = its;
      rp.inner_iters += its;
      rp.newton_iters = ++k;
      if (hipError_t e = st_axpby(f, 1.0, f, -1.0, gcor, N, s)) {
        plan_note_hip(pl, e);
        status = LINCOLL_EHIP;
        break;
      }
      status = constrain(f, nullptr);
    }
    if (status == LINCOLL_OK || status == LINCOLL_EDIVERGED) {
      double m = 0.0;
      if (constrain_mass(f, &m) == LINCOLL_OK) rp.mass = m;
    }
    rp.ms_total = ms_since(t0);
    rp.rec_rows = rec_rows;
    if (rep) *rep = rp;
    return status;
  }

  // discrete mass of f (no rescaling)
  int constrain_mass(const double* f, double* m) {
    HIPCK(st_cell_sums(f, nx, n, L, d_sums, s));
    std::vector<double> hs((size_t)nx * SUMS_STRIDE);
    STCK(host_copy(hs.data(), d_sums, hs.size() * sizeof(double)));
    double t = 0.0;
    for (int c = 0; c < nx; ++c) t += hs[(size_t)c * SUMS_STRIDE];
    *m = t * dx * h3;
    return LINCOLL_OK;
  }
};

}  // namespace

extern "C" {

void lincoll_steady_default(lincoll_steady_params_t* sp, int nx) {
  if (!sp) return;
  std::memset(sp, 0, sizeof(*sp));
  sp->nx = nx;
  sp->x_l = -0.5;
  sp->x_r = 0.5;
  sp->kn = 0.1;
  sp->mass = 1.0;
  sp->theta_l = 1.0;
  sp->theta_r = 1.5;
  sp->tol = 1e-5;
  sp->inner_rtol = 1e-3;
  sp->inner_atol = 1e-7;
  sp->max_newton = 30;
  sp->max_inner = 2000;
  sp->restart = 30;
  sp->init = 1;
  sp->precond = LINCOLL_PRECOND_SWEEP;
  sp->inner = LINCOLL_INNER_GMRES;
  sp->backtrack = 1;
}

int lincoll_steady_residual(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f, double* r,
                            double* norm) {
  if (!plan || !f) return LINCOLL_EINVAL;
  Solver S;
  STCK(S.init(plan, sp));
  if (r && overlap(f, r, (size_t)S.N * sizeof(double))) return LINCOLL_EINVAL;
  double* out = r ? r : S.d_aux;
  double v = 0.0;
  STCK(S.residual(f, out, &v));
  lincoll_plan_t pl = plan;
  HIPCK(hipStreamSynchronize(S.s));
  if (norm) *norm = v;
  return LINCOLL_OK;
}

int lincoll_steady_newton_apply(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                                const double* g, double* out) {
  if (!plan || !f || !g || !out) return LINCOLL_EINVAL;
  Solver S;
  STCK(S.init(plan, sp));
  if (overlap(g, out, (size_t)S.N * sizeof(double))) return LINCOLL_EINVAL;
  STCK(S.set_local(f));
  STCK(S.matvec(g, out));
  lincoll_plan_t pl = plan;
  HIPCK(hipStreamSynchronize(S.s));
  return LINCOLL_OK;
}

int lincoll_steady_precondition(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                                const double* y, double* z) {
  if (!plan || !f || !y || !z) return LINCOLL_EINVAL;
  Solver S;
  STCK(S.init(plan, sp));
  if (overlap(y, z, (size_t)S.N * sizeof(double))) return LINCOLL_EINVAL;
  STCK(S.set_local(f));
  STCK(S.precondition(y, z));
  lincoll_plan_t pl = plan;
  HIPCK(hipStreamSynchronize(S.s));
  return LINCOLL_OK;
}

int lincoll_learned_features(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                             const double* z, float* X, double* sc) {
  if (!plan || !f || !z || !X) return LINCOLL_EINVAL;
  Solver S;
  STCK(S.init(plan, sp));
  STCK(S.local_params(f));
  STCK(S.features(z, X));
  double v = 0.0;
  STCK(S.host_copy(&v, S.d_scale, sizeof(double)));
  if (sc) *sc = v;
  return LINCOLL_OK;
}

int lincoll_learned_correction(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                               const float* Y, double sc, double* out) {
  if (!plan || !f || !Y || !out || !std::isfinite(sc)) return LINCOLL_EINVAL;
  Solver S;
  STCK(S.init(plan, sp));
  lincoll_plan_t pl = plan;
  STCK(S.local_params(f));
  HIPCK(hipMemcpyAsync(S.d_scale, &sc, sizeof(double), hipMemcpyHostToDevice, S.s));
  HIPCK(ln_correction(Y, S.d_scale, S.d_params, S.nx, S.n, S.L, 0, out, S.s));
  HIPCK(hipStreamSynchronize(S.s));
  return LINCOLL_OK;
}

int lincoll_steady_solve(lincoll_plan_t plan, const lincoll_steady_params_t* sp, double* f,
                         lincoll_steady_report_t* rep) {
  if (!plan || !f) return LINCOLL_EINVAL;
  Solver S;
  STCK(S.init(plan, sp, true));
  return S.solve(f, rep);
}

}  // extern "C"
