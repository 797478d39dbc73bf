// C ABI of liblincoll (declared in include/lincoll.h): argument checks,
// plan ownership, table upload and launch orchestration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lincoll.h"
#include "host_tables.h"
#include "internal.h"

using namespace lincoll;

struct lincoll_plan_s {
  lincoll_params_t p{};
  HostTables t;
  int device = 0;
  hipStream_t stream = nullptr;
  int last_hip = 0;
  size_t bytes = 0;
  // plan tables
  void* d_Phi = nullptr;      // [J][phi_stride(n)] apply dtype, / n^3
  void* d_Om = nullptr;       // [Q]    apply dtype, / n^3
  double* d_Om64 = nullptr;   // [Q]    FP64, / n^3
  double* d_phi = nullptr;    // [J][P^3]
  double* d_Cdct = nullptr;   // [P][P]
  // per-cell cache
  int Bc = 0, cap_cells = 0;
  double* d_params = nullptr;
  double* d_fac64 = nullptr;
  double* d_pref64 = nullptr;
  double* d_gfac64 = nullptr;
  double* d_Ainv = nullptr;
  void* d_facT = nullptr;
  void* d_prefT = nullptr;
  uint32_t* d_mask = nullptr;
  void* d_Kh = nullptr;
  void* d_nu = nullptr;
  // setup scratch
  int setup_chunk = 0;
  double* d_tmpA = nullptr;
  double* d_tmpB = nullptr;
  double* d_planes64 = nullptr;
  // apply work
  int cap_work = 0, cap_pin = 0;
  void* d_R = nullptr;
  void* d_H = nullptr;
  void* d_W = nullptr;
  void* d_Wq = nullptr;
  void* d_Lp = nullptr;
  void* d_pin = nullptr;      // projected input when p.project
  size_t R_bytes = 0;         // size of d_R (shared by the staged and fused paths)
  int cus = 256;              // compute units of the plan's device
  // options (lincoll_set_option)
  int opt_graph = 0, opt_per_cu = 0;
  int opt_zblk = 128, opt_tile = 0, opt_tune_cache = 1, opt_ppt = 1;
  int opt_keep = -1;   // fused accumulator chunks kept in registers (-1: the default for n)
  int opt_split = 0;   // fused workgroups per cell: 0 = by batch, 1 = never split, S = S parts
  int last_split = 1;  // parts per cell of the most recent apply (LINCOLL_INFO_FUSED_SPLIT)
  double tuned_ms = 0.0;
  int tuned_cached = 0;
  int last_path = 0;          // path of the most recent apply (LINCOLL_INFO_LAST_PATH)
  int opt_check_finite = 0;   // LINCOLL_OPT_CHECK_FINITE
  int* d_flag = nullptr;      // its device flag
  std::string arch;           // gcnArchName of the plan's device (key of the tuner's cache)
  // replayable graph of the last apply (opt_graph)
  unsigned long alloc_gen = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphKey {
    const void* h;
    void* out;
    int batch, Bc, fused, per_cu, project;
    unsigned long gen;
  } gkey{};
  // time stepping (lincoll_rk4): work buffers and the recorded step
  int cap_rk = 0;
  void* d_rk_k = nullptr;
  void* d_rk_tmp = nullptr;
  void* d_rk_acc = nullptr;
  hipGraphExec_t rk_gexec = nullptr;
  GraphKey rk_key{};
  double rk_dt = 0.0;
  // binary operator (quadcoll_apply): hemisphere rule, tables, work volumes
  int sphere_polar = 8, sphere_azim = 16;
  int cap_qc = 0;
  double* d_Ws = nullptr;
  double* d_qV = nullptr;
  double2 *d_qF = nullptr, *d_qGp = nullptr, *d_qGm = nullptr, *d_qC = nullptr, *d_qS = nullptr, *d_qQ = nullptr;
  double2* d_qPh = nullptr;   // azimuth phase tables of the hemisphere rule
  long cap_qph = 0;           // complex values held by d_qPh
  int quad_fix = 0;           // mass fix of quadcoll_apply (LINCOLL_OPT_QUAD_FIX)
  double* d_qOs = nullptr;    // fix 2: loss weight [n][n][n] for the rule (qos_polar, qos_azim)
  double* d_qGW = nullptr;    // fix 2: (g_j, W_j) [J][2]
  double* d_qRule = nullptr;  // fix 2: hemisphere rule [M][4]
  long cap_qrule = 0;
  int qos_polar = 0, qos_azim = 0;
  // steady solver work memory (plan_steady_work)
  void* d_steady = nullptr;
  size_t cap_steady = 0;
};

namespace {

size_t esize(int dtype) { return dtype == LINCOLL_F64 ? sizeof(double) : sizeof(float); }

// Last HIP error seen on this thread (plan creation destroys a failed plan,
// so its code is kept here as well).
thread_local int g_last_hip = 0;

// Failure injection for tests of the out-of-memory paths: when positive, the
// k-th dalloc call from now fails with hipErrorOutOfMemory (the k - 1 before
// it succeed); set by lincoll_debug_fail_alloc.
int g_fail_alloc_after = 0;

int hip_fail(lincoll_plan_t pl, hipError_t e) {
  if (pl) pl->last_hip = (int)e;
  g_last_hip = (int)e;
  return e == hipErrorOutOfMemory ? LINCOLL_ENOMEM : LINCOLL_EHIP;
}

// (Re)allocates *ptr.  The old buffer is freed first, so after a failure
// *ptr is null; every caller then zeroes the capacities that describe the
// buffers it was growing, and the next call allocates them again (or reports
// LINCOLL_ENOTREADY) instead of launching kernels on null pointers.
template <typename P>
hipError_t dalloc(lincoll_plan_t pl, P** ptr, size_t bytes) {
  if (*ptr) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
  }
  ++pl->alloc_gen;   // device pointers changed: a captured graph is stale
  if (g_fail_alloc_after > 0 && --g_fail_alloc_after == 0) return hipErrorOutOfMemory;
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, bytes);
  if (e == hipSuccess) {
    *ptr = static_cast<P*>(v);
    pl->bytes += bytes;
  }
  return e;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

int validate(const lincoll_params_t* p) {
  if (!p) return LINCOLL_EINVAL;
  if (p->dtype != LINCOLL_F64 && p->dtype != LINCOLL_F32 && p->dtype != LINCOLL_BF16X3) return LINCOLL_EINVAL;
  if (!(p->n == 8 || p->n == 16 || p->n == 32 || p->n == 64)) return LINCOLL_EINVAL;
  if (!(p->L > 0.0) || !std::isfinite(p->L)) return LINCOLL_EINVAL;
  if (!(p->omega >= 0.5 && p->omega <= 1.0)) return LINCOLL_EINVAL;
  if (!(p->C > 0.0) || !std::isfinite(p->C)) return LINCOLL_EINVAL;
  if (!std::isfinite(p->R)) return LINCOLL_EINVAL;
  if (p->J < 0 || p->J > 256) return LINCOLL_EINVAL;
  if (!(p->eps >= 0.0) || !(p->eps < 1.0)) return LINCOLL_EINVAL;
  if (p->quad_rule != 0 && p->quad_rule != 1) return LINCOLL_EINVAL;
  if (p->project != 0 && p->project != 1) return LINCOLL_EINVAL;
  if (p->max_batch < 0) return LINCOLL_EINVAL;
  if (p->path < 0 || p->path > 2) return LINCOLL_EINVAL;
  if (p->path == LINCOLL_PATH_FUSED && !fused_supported(p->n, p->dtype)) return LINCOLL_EINVAL;
  if (!staged_supported(p->n, p->dtype)) return LINCOLL_EINVAL;
  return LINCOLL_OK;
}

lincoll_params_t resolved(const lincoll_params_t* in) {
  lincoll_params_t p = *in;
  if (p.R <= 0.0) p.R = 4.0 * p.L / (3.0 + std::sqrt(2.0));
  if (p.J <= 0) p.J = p.n / 2 + 1;
  return p;
}

// Accumulator chunks the fused kernel keeps in registers: the plan's option,
// else the default for n (the fastest measured on MI355X).
int fused_keep(const lincoll_plan_s* pl) {
  if (pl->opt_keep >= 0) return pl->opt_keep;
  return fused_default_keep(pl->p.n, pl->p.dtype);
}

// Path of an apply of `batch` cells.  AUTO takes the fused kernels where
// they exist.  Split over several workgroups per cell, they beat the staged
// kernels from one cell on; with one workgroup per cell (splitting switched
// off, or two pencils per thread) a small batch leaves most of the chip idle,
// and the staged kernels, which spread even one cell over many CUs, are
// faster at n = 32 below 16 cells in F32 and 128 in F64 (measured on MI355X).
int fused_auto_min_batch(const lincoll_plan_s* pl) {
  const bool can_split = pl->opt_ppt == 1 && pl->opt_split != 1;
  if (pl->p.n == 16 || can_split) return 1;
  return pl->p.dtype == LINCOLL_F64 ? 128 : 16;
}

bool use_fused(const lincoll_plan_s* pl, int batch) {
  if (pl->p.path == LINCOLL_PATH_STAGED) return false;
  if (pl->p.path == LINCOLL_PATH_FUSED) return true;
  return fused_supported(pl->p.n, pl->p.dtype) && batch >= fused_auto_min_batch(pl);
}

// Workgroups per cell of a fused apply of `batch` cells: the plan's option,
// else enough parts to spread a small batch over the chip (one workgroup per
// cell once the batch fills it).  The two-pencil kernel does not split.
int fused_split(const lincoll_plan_s* pl, int batch) {
  if (pl->opt_ppt != 1 || pl->opt_split == 1) return 1;
  if (pl->opt_split > 1) return std::min(pl->opt_split, pl->t.J);
  return fused_auto_split(pl->p.n, pl->t.J, batch, pl->cus);
}

// The batch a path query refers to: the Maxwellian batch when it is per
// cell, otherwise a large batch.
int info_batch(const lincoll_plan_s* pl) { return pl->Bc > 1 ? pl->Bc : 1 << 30; }

int ensure_cells(lincoll_plan_t pl, int B) {
  if (B <= pl->cap_cells) return LINCOLL_OK;
  const int n = pl->p.n, P = n / 2 + 1, J = pl->t.J, MW = (n + 31) / 32;
  const size_t n3 = (size_t)n * n * n, P3 = (size_t)P * P * P, es = esize(pl->p.dtype);
  hipError_t e;
  if ((e = dalloc(pl, &pl->d_params, (size_t)B * 5 * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_fac64, (size_t)B * 6 * n * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_pref64, (size_t)B * 2 * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_gfac64, (size_t)B * P * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_Ainv, (size_t)B * 25 * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_facT, (size_t)B * 6 * n * es)) || (e = dalloc(pl, &pl->d_prefT, (size_t)B * 2 * es)) ||
      (e = dalloc(pl, &pl->d_mask, (size_t)B * n * n * MW * sizeof(uint32_t))) ||
      (e = dalloc(pl, &pl->d_Kh, (size_t)B * J * kh_stride(n) * sizeof(double))) || (e = dalloc(pl, &pl->d_nu, (size_t)B * n3 * es))) {
    pl->cap_cells = 0;
    pl->Bc = 0;          // the Maxwellian cache is gone: applies report ENOTREADY
    return hip_fail(pl, e);
  }
  pl->cap_cells = B;
  // Setup scratch, in chunks of cells bounded to ~256 MiB per buffer.  Per
  // cell, tmpA holds the J kernel-mode octants (J P^3 doubles) and later the
  // FP64 loss frequency nu (n^3 doubles); small J makes the second larger.
  const size_t per_cell = std::max<size_t>((size_t)J * P3, n3) * sizeof(double);
  int chunk = (int)std::max<size_t>(1, (size_t)(256u << 20) / per_cell);
  if (chunk > B) chunk = B;
  if (chunk > pl->setup_chunk) {
    if ((e = dalloc(pl, &pl->d_tmpA, (size_t)chunk * per_cell)) || (e = dalloc(pl, &pl->d_tmpB, (size_t)chunk * per_cell)) ||
        (e = dalloc(pl, &pl->d_planes64, (size_t)chunk * P * n * n * 2 * sizeof(double)))) {
      pl->setup_chunk = 0;
      pl->cap_cells = 0;
      pl->Bc = 0;
      return hip_fail(pl, e);
    }
    pl->setup_chunk = chunk;
  }
  return LINCOLL_OK;
}

int ensure_work(lincoll_plan_t pl, int B) {
  const int n = pl->p.n, P = n / 2 + 1;
  const size_t es = esize(pl->p.dtype);
  hipError_t e;
  if (pl->p.project && B > pl->cap_pin) {
    if ((e = dalloc(pl, &pl->d_pin, (size_t)B * n * n * n * es))) {
      pl->cap_pin = 0;
      return hip_fail(pl, e);
    }
    pl->cap_pin = B;
  }
  if (use_fused(pl, B)) {
    const int S = fused_split(pl, B);
    const size_t need =
        S > 1 ? fused_split_scratch_bytes(n, fused_slots(n, B * (S + fused_loss_item(n, B, S, pl->cus)), pl->opt_per_cu,
                                                      pl->cus),
                                          B, S, pl->p.dtype)
              : fused_scratch_bytes(n, fused_slots(n, B, pl->opt_per_cu, pl->cus), pl->opt_ppt, pl->p.dtype);
    if (need > pl->R_bytes || !pl->d_R) {
      pl->cap_work = 0;
      if ((e = dalloc(pl, &pl->d_R, need))) {
        pl->R_bytes = 0;
        return hip_fail(pl, e);
      }
      pl->R_bytes = need;
    }
    return LINCOLL_OK;
  }
  const size_t vol = (size_t)B * P * n * n * 2 * es, vol64 = (size_t)B * P * n * n * 2 * sizeof(double);
  if (B <= pl->cap_work && pl->d_H && pl->R_bytes >= vol64) return LINCOLL_OK;
  if ((e = dalloc(pl, &pl->d_R, vol64)) || (e = dalloc(pl, &pl->d_H, vol)) || (e = dalloc(pl, &pl->d_W, vol64)) ||
      (e = dalloc(pl, &pl->d_Wq, vol)) || (e = dalloc(pl, &pl->d_Lp, vol))) {
    pl->cap_work = 0;
    pl->R_bytes = 0;
    return hip_fail(pl, e);
  }
  pl->R_bytes = vol64;
  pl->cap_work = B;
  return LINCOLL_OK;
}

int do_set_maxwellians(lincoll_plan_t pl, const double* params, int batch) {
  int st = ensure_cells(pl, batch);
  if (st) return st;
  hipError_t e = hipMemcpyAsync(pl->d_params, params, (size_t)batch * 5 * sizeof(double), hipMemcpyDeviceToDevice,
                                pl->stream);
  if (e) {
    pl->Bc = 0;
    return hip_fail(pl, e);
  }
  SetupCtx c;
  c.n = pl->p.n;
  c.J = pl->t.J;
  c.Q = pl->t.Q;
  c.Bc = batch;
  c.dtype = pl->p.dtype;
  c.L = pl->p.L;
  c.eps = pl->p.eps;
  c.stream = pl->stream;
  c.params = pl->d_params;
  c.phi = pl->d_phi;
  c.Cdct = pl->d_Cdct;
  c.Om64 = pl->d_Om64;
  c.fac64 = pl->d_fac64;
  c.pref64 = pl->d_pref64;
  c.gfac64 = pl->d_gfac64;
  c.Ainv = pl->d_Ainv;
  c.facT = pl->p.dtype == LINCOLL_F64 ? (void*)pl->d_fac64 : pl->d_facT;
  c.prefT = pl->p.dtype == LINCOLL_F64 ? (void*)pl->d_pref64 : pl->d_prefT;
  c.mask = pl->d_mask;
  c.Kh = pl->d_Kh;
  c.nu = pl->d_nu;
  c.tmpA = pl->d_tmpA;
  c.tmpB = pl->d_tmpB;
  c.planes64 = pl->d_planes64;
  c.chunk = pl->setup_chunk;
  e = setup_cells(c);
  if (e) {
    pl->Bc = 0;
    return hip_fail(pl, e);
  }
  pl->Bc = batch;
  return LINCOLL_OK;
}

}  // namespace

extern "C" {

void lincoll_params_default(lincoll_params_t* p, int n, double L_domain, double vhs_omega, int dtype) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n = n;
  p->L = L_domain;
  p->omega = vhs_omega;
  p->C = 1.0 / (4.0 * M_PI);
  p->R = 0.0;
  p->J = 0;
  p->eps = 1e-9;
  p->quad_rule = 0;
  p->project = 0;
  p->max_batch = 0;
  p->dtype = dtype;
  p->path = LINCOLL_PATH_AUTO;
}

const char* lincoll_strerror(int s) {
  switch (s) {
    case LINCOLL_OK: return "success";
    case LINCOLL_EINVAL: return "invalid argument";
    case LINCOLL_ENOMEM: return "device out of memory";
    case LINCOLL_EHIP: return "HIP runtime error";
    case LINCOLL_ENOTREADY: return "Maxwellians not set for this batch";
    case LINCOLL_ENOTIMPL: return "not implemented";
    case LINCOLL_EDIVERGED: return "iteration diverged";
    case LINCOLL_ENONFINITE: return "non-finite values in the output";
  }
  return "unknown status";
}

long long lincoll_plan_tables(const lincoll_params_t* pin, int table, double* out, long long count) {
  if (!pin) return LINCOLL_EINVAL;
  lincoll_params_t q = *pin;
  if (q.path == LINCOLL_PATH_FUSED || q.dtype == LINCOLL_BF16X3) q.path = LINCOLL_PATH_STAGED, q.dtype = LINCOLL_F32;
  if (validate(&q)) return LINCOLL_EINVAL;
  const lincoll_params_t p = resolved(pin);
  HostTables t;
  TableParams tp{p.n, p.L, p.omega, p.C, p.R, p.J, p.quad_rule};
  if (!build_tables(tp, t)) return LINCOLL_EINVAL;
  const std::vector<double>* v = nullptr;
  switch (table) {
    case LINCOLL_TABLE_G: v = &t.g; break;
    case LINCOLL_TABLE_W: v = &t.W; break;
    case LINCOLL_TABLE_PHI: v = &t.Phi; break;
    case LINCOLL_TABLE_OMEGA: v = &t.Omega; break;
    case LINCOLL_TABLE_PHIJ: v = &t.phi; break;
    default: return LINCOLL_EINVAL;
  }
  const long long need = (long long)v->size();
  if (out) {
    if (count < need) return LINCOLL_EINVAL;
    std::memcpy(out, v->data(), (size_t)need * sizeof(double));
  }
  return need;
}

int lincoll_plan_ex(const lincoll_params_t* pin, lincoll_plan_t* out) {
  if (!out) return LINCOLL_EINVAL;
  *out = nullptr;
  int st = validate(pin);
  if (st) return st;
  lincoll_plan_t pl = new (std::nothrow) lincoll_plan_s();
  if (!pl) return LINCOLL_ENOMEM;
  pl->p = resolved(pin);
  TableParams tp{pl->p.n, pl->p.L, pl->p.omega, pl->p.C, pl->p.R, pl->p.J, pl->p.quad_rule};
  if (!build_tables(tp, pl->t)) {
    delete pl;
    return LINCOLL_EINVAL;
  }
  hipError_t e = hipGetDevice(&pl->device);
  if (!e) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, pl->device) == hipSuccess && v > 0) pl->cus = v;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) pl->arch = prop.gcnArchName;
  }
  if (e) {
    pl->last_hip = (int)e;
    delete pl;
    return LINCOLL_EHIP;
  }
  const int n = pl->p.n, P = n / 2 + 1, J = pl->t.J, Q = pl->t.Q;
  const double s3 = 1.0 / ((double)n * n * n);
  const int QS = phi_stride(n);
  std::vector<double> phis((size_t)J * QS, 0.0), oms(pl->t.Omega);
  for (int j = 0; j < J; ++j)
    for (int q = 0; q < Q; ++q) phis[(size_t)j * QS + q] = pl->t.Phi[(size_t)j * Q + q] * s3;
  for (auto& v : oms) v *= s3;
  const size_t es = esize(pl->p.dtype);
  auto upload = [&](void* dst, const std::vector<double>& src, bool asf) -> hipError_t {
    if (!asf) return hipMemcpy(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice);
    std::vector<float> f(src.begin(), src.end());
    return hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
  };
  const bool asf = pl->p.dtype != LINCOLL_F64;
  if ((e = dalloc(pl, &pl->d_Phi, (size_t)J * QS * es)) || (e = dalloc(pl, &pl->d_Om, (size_t)Q * es)) ||
      (e = dalloc(pl, &pl->d_Om64, (size_t)Q * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_phi, (size_t)J * P * P * P * sizeof(double))) ||
      (e = dalloc(pl, &pl->d_Cdct, (size_t)P * P * sizeof(double))) || (e = upload(pl->d_Phi, phis, asf)) ||
      (e = upload(pl->d_Om, oms, asf)) || (e = upload(pl->d_Om64, oms, false)) ||
      (e = upload(pl->d_phi, pl->t.phi, false)) || (e = upload(pl->d_Cdct, pl->t.Cdct, false))) {
    int rc = hip_fail(pl, e);
    lincoll_destroy(pl);
    return rc;
  }
  // default Maxwellian (1, 0, 1)
  double* dpar = nullptr;
  const double def[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  if ((e = hipMalloc(&dpar, sizeof(def))) || (e = hipMemcpy(dpar, def, sizeof(def), hipMemcpyHostToDevice))) {
    dfree(dpar);
    int rc = hip_fail(pl, e);
    lincoll_destroy(pl);
    return rc;
  }
  st = do_set_maxwellians(pl, dpar, 1);
  if (!st && (e = hipStreamSynchronize(pl->stream))) st = hip_fail(pl, e);
  dfree(dpar);
  if (st) {
    lincoll_destroy(pl);
    return st;
  }
  *out = pl;
  return LINCOLL_OK;
}

int lincoll_plan(int n, double L_domain, double vhs_omega, int dtype, lincoll_plan_t* out) {
  lincoll_params_t p;
  lincoll_params_default(&p, n, L_domain, vhs_omega, dtype);
  return lincoll_plan_ex(&p, out);
}

int lincoll_set_stream(lincoll_plan_t pl, void* s) {
  if (!pl) return LINCOLL_EINVAL;
  pl->stream = static_cast<hipStream_t>(s);
  return LINCOLL_OK;
}

int lincoll_set_maxwellians(lincoll_plan_t pl, const double* params, int batch) {
  if (!pl || !params || batch < 1) return LINCOLL_EINVAL;
  if (pl->p.max_batch > 0 && batch > pl->p.max_batch) return LINCOLL_EINVAL;
  return do_set_maxwellians(pl, params, batch);
}

namespace {

hipError_t launch_project(lincoll_plan_t pl, const void* x, void* y, int batch, hipStream_t stream,
                          const int* gate = nullptr) {
  ProjectCtx c;
  c.gate = gate;
  c.n = pl->p.n;
  c.batch = batch;
  c.Bc = pl->Bc;
  c.dtype = pl->p.dtype == LINCOLL_F64 ? 0 : 1;
  c.L = pl->p.L;
  c.stream = stream;
  c.x = x;
  c.y = y;
  c.fac64 = pl->d_fac64;
  c.pref64 = pl->d_pref64;
  c.Ainv = pl->d_Ainv;
  return project_cells(c);
}

}  // namespace

int lincoll_project(lincoll_plan_t pl, const void* x, void* y, int batch) {
  if (!pl || !x || !y || batch < 1) return LINCOLL_EINVAL;
  if (pl->Bc != 1 && pl->Bc != batch) return LINCOLL_ENOTREADY;
  hipError_t e = launch_project(pl, x, y, batch, pl->stream);
  return e ? hip_fail(pl, e) : LINCOLL_OK;
}

namespace {

ApplyCtx apply_ctx(lincoll_plan_t pl, const void* hin, void* out, int batch, hipStream_t stream) {
  ApplyCtx c;
  c.n = pl->p.n;
  c.J = pl->t.J;
  c.Q = pl->t.Q;
  c.batch = batch;
  c.Bc = pl->Bc;
  c.cus = pl->cus;
  c.per_cu = pl->opt_per_cu;
  c.zblk = pl->opt_zblk;
  c.fused_ppt = pl->opt_ppt;
  c.fused_keep = fused_keep(pl);
  c.fused_split = use_fused(pl, batch) ? fused_split(pl, batch) : 1;
  c.plane_tile = pl->opt_tile;
  c.dtype = pl->p.dtype;
  c.stream = stream;
  c.h = hin;
  c.out = out;
  c.Phi = pl->d_Phi;
  c.Om = pl->d_Om;
  c.fac = pl->p.dtype == LINCOLL_F64 ? (const void*)pl->d_fac64 : pl->d_facT;
  c.pref = pl->p.dtype == LINCOLL_F64 ? (const void*)pl->d_pref64 : pl->d_prefT;
  c.fac64 = pl->d_fac64;
  c.pref64 = pl->d_pref64;
  c.mask = pl->d_mask;
  c.Kh = pl->d_Kh;
  c.nu = pl->d_nu;
  c.R = pl->d_R;
  c.H = pl->d_H;
  c.W = pl->d_W;
  c.Wq = pl->d_Wq;
  c.Lp = pl->d_Lp;
  return c;
}

// Every launch of one apply, on `stream` (the plan's stream, or the capture
// stream while a replayable graph is recorded).  Work buffers must exist.
hipError_t launch_apply(lincoll_plan_t pl, const void* h, void* out, int batch, hipStream_t stream,
                        const int* gate = nullptr) {
  hipError_t e;
  const void* hin = h;
  if (pl->p.project) {
    if ((e = launch_project(pl, h, pl->d_pin, batch, stream, gate))) return e;
    hin = pl->d_pin;
  }
  ApplyCtx c = apply_ctx(pl, hin, out, batch, stream);
  c.gate = gate;
  const bool fused = use_fused(pl, batch);
  pl->last_path = fused ? LINCOLL_PATH_FUSED : LINCOLL_PATH_STAGED;
  pl->last_split = fused ? c.fused_split : 1;
  if ((e = fused ? fused_apply(c) : staged_apply(c))) return e;
  if (pl->p.project) return launch_project(pl, out, out, batch, stream, gate);
  return hipSuccess;
}

void drop_graph(lincoll_plan_t pl) {
  if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
  pl->gexec = nullptr;
}

// Records the launches of one apply into a graph on the plan's own capture
// stream and instantiates it; later applies with the same key replay it with
// a single hipGraphLaunch.  The graph holds kernel nodes only.
hipError_t capture_apply(lincoll_plan_t pl, const void* h, void* out, int batch,
                         const lincoll_plan_s::GraphKey& key) {
  drop_graph(pl);
  hipError_t e;
  if (!pl->cap_stream && (e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking))) return e;
  if ((e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal))) return e;
  const hipError_t el = launch_apply(pl, h, out, batch, pl->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(pl->cap_stream, &g);
  if (el) e = el;
  if (!e) e = hipGraphInstantiate(&pl->gexec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e) {
    pl->gexec = nullptr;
    return e;
  }
  pl->gkey = key;
  return hipSuccess;
}

int checked_apply_args(lincoll_plan_t pl, const void* h, void* out, int batch) {
  if (!pl || !h || !out || batch < 1) return LINCOLL_EINVAL;
  if (pl->p.max_batch > 0 && batch > pl->p.max_batch) return LINCOLL_EINVAL;
  const size_t bytes = (size_t)batch * pl->p.n * pl->p.n * pl->p.n * esize(pl->p.dtype);
  const char* a = static_cast<const char*>(h);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return LINCOLL_EINVAL;   // overlap
  if (pl->Bc != 1 && pl->Bc != batch) return LINCOLL_ENOTREADY;
  return LINCOLL_OK;
}

}  // namespace

namespace {

// LINCOLL_OPT_CHECK_FINITE: scan the output on the plan's stream and read the
// flag back (synchronises the stream).
int check_output(lincoll_plan_t pl, const void* out, int batch) {
  if (!pl->opt_check_finite) return LINCOLL_OK;
  hipError_t e;
  if (!pl->d_flag && (e = dalloc(pl, &pl->d_flag, sizeof(int)))) return hip_fail(pl, e);
  const long count = (long)batch * pl->p.n * pl->p.n * pl->p.n;
  int host = 0;
  if ((e = nonfinite_check(out, count, pl->p.dtype == LINCOLL_F64, pl->d_flag, pl->stream)) ||
      (e = hipMemcpyAsync(&host, pl->d_flag, sizeof(int), hipMemcpyDeviceToHost, pl->stream)) ||
      (e = hipStreamSynchronize(pl->stream)))
    return hip_fail(pl, e);
  return host ? LINCOLL_ENONFINITE : LINCOLL_OK;
}

}  // namespace

int lincoll_apply(lincoll_plan_t pl, const void* h, void* out, int batch) {
  int st = checked_apply_args(pl, h, out, batch);
  if (st) return st;
  if ((st = ensure_work(pl, batch))) return st;
  hipError_t e;
  if (!pl->opt_graph) {
    if ((e = launch_apply(pl, h, out, batch, pl->stream))) return hip_fail(pl, e);
    return check_output(pl, out, batch);
  }
  const lincoll_plan_s::GraphKey key{h, out, batch, pl->Bc, use_fused(pl, batch) ? 1 : 0, pl->opt_per_cu, pl->p.project,
                                     pl->alloc_gen};
  const lincoll_plan_s::GraphKey& k = pl->gkey;
  const bool same = pl->gexec && k.h == key.h && k.out == key.out && k.batch == key.batch && k.Bc == key.Bc &&
                    k.fused == key.fused && k.per_cu == key.per_cu && k.project == key.project && k.gen == key.gen;
  if (!same && (e = capture_apply(pl, h, out, batch, key))) return hip_fail(pl, e);
  if ((e = hipGraphLaunch(pl->gexec, pl->stream))) return hip_fail(pl, e);
  pl->last_path = key.fused ? LINCOLL_PATH_FUSED : LINCOLL_PATH_STAGED;
  pl->last_split = key.fused ? fused_split(pl, batch) : 1;
  return check_output(pl, out, batch);
}

int lincoll_apply_noalloc(lincoll_plan_t pl, const void* h, void* out, int batch) {
  int st = checked_apply_args(pl, h, out, batch);
  if (st) return st;
  if (!use_fused(pl, batch) || pl->p.project) return LINCOLL_EINVAL;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e) return hip_fail(pl, e);
  if (dev != pl->device) return LINCOLL_EINVAL;
  void* scr = nullptr;
  size_t bytes = 0;
  if ((e = fused_noalloc_scratch(dev, &scr, &bytes))) return hip_fail(pl, e);
  const size_t slot = fused_scratch_bytes(pl->p.n, 1, pl->opt_ppt, pl->p.dtype);
  if (slot == 0 || slot > bytes) return LINCOLL_EINVAL;
  ApplyCtx c = apply_ctx(pl, h, out, batch, pl->stream);
  c.R = scr;
  // The plan's split of this batch (as lincoll_apply takes it) where its
  // slots and partial sums fit the array; else one workgroup per cell, the
  // persistent workgroups capped to the slots the array holds.
  const int n = pl->p.n, S = c.fused_split;
  const size_t need =
      S > 1 ? fused_split_scratch_bytes(
                  n, fused_slots(n, batch * (S + fused_loss_item(n, batch, S, pl->cus)), pl->opt_per_cu, pl->cus),
                  batch, S, pl->p.dtype)
            : 0;
  if (S > 1 && need <= bytes) {
    c.max_slots = 0;
  } else {
    c.fused_split = 1;
    c.max_slots = (int)(bytes / slot);
  }
  if ((e = fused_apply(c))) return hip_fail(pl, e);
  pl->last_path = LINCOLL_PATH_FUSED;
  pl->last_split = c.fused_split;
  return LINCOLL_OK;
}

int lincoll_set_option(lincoll_plan_t pl, int key, int value) {
  if (!pl) return LINCOLL_EINVAL;
  switch (key) {
    case LINCOLL_OPT_GRAPH:
      if (value != 0 && value != 1) return LINCOLL_EINVAL;
      pl->opt_graph = value;
      break;
    case LINCOLL_OPT_FUSED_PER_CU:
      if (value < 0 || value > fused_max_per_cu(pl->p.n)) return LINCOLL_EINVAL;
      pl->opt_per_cu = value;
      break;
    case LINCOLL_OPT_SPHERE_POLAR:
      if (value < 2 || value > 64 || value % 2) return LINCOLL_EINVAL;
      pl->sphere_polar = value;
      break;
    case LINCOLL_OPT_SPHERE_AZIMUTH:
      if (value < 1 || value > 256) return LINCOLL_EINVAL;
      pl->sphere_azim = value;
      break;
    case LINCOLL_OPT_PROJECT:
      if (value != 0 && value != 1) return LINCOLL_EINVAL;
      pl->p.project = value;
      break;
    case LINCOLL_OPT_QUAD_FIX:
      if (value < 0 || value > 2) return LINCOLL_EINVAL;
      pl->quad_fix = value;
      break;
    case LINCOLL_OPT_ZBLOCK:
      if (value != 64 && value != 128 && value != 256) return LINCOLL_EINVAL;
      pl->opt_zblk = value;
      break;
    case LINCOLL_OPT_PLANE_TILE:
      if (value != 0 && value != 1) return LINCOLL_EINVAL;
      if (value == 1 && pl->p.n > 32) return LINCOLL_EINVAL;
      pl->opt_tile = value;
      break;
    case LINCOLL_OPT_FUSED_PPT:
      if (value != 1 && value != 2) return LINCOLL_EINVAL;
      if (value == 2 && pl->p.dtype != LINCOLL_F32) return LINCOLL_EINVAL;
      pl->opt_ppt = value;
      break;
    case LINCOLL_OPT_FUSED_KEEP:
      if (value != -1 && !fused_keep_valid(pl->p.n, pl->p.dtype, value)) return LINCOLL_EINVAL;
      pl->opt_keep = value;
      break;
    case LINCOLL_OPT_FUSED_SPLIT:
      if (value < 0 || value > pl->t.J) return LINCOLL_EINVAL;
      pl->opt_split = value;
      break;
    case LINCOLL_OPT_TUNE_CACHE:
      if (value != 0 && value != 1) return LINCOLL_EINVAL;
      pl->opt_tune_cache = value;
      break;
    case LINCOLL_OPT_CHECK_FINITE:
      if (value != 0 && value != 1) return LINCOLL_EINVAL;
      pl->opt_check_finite = value;
      break;
    case LINCOLL_OPT_PATH:
      if (value < LINCOLL_PATH_AUTO || value > LINCOLL_PATH_FUSED) return LINCOLL_EINVAL;
      if (value == LINCOLL_PATH_FUSED && !fused_supported(pl->p.n, pl->p.dtype)) return LINCOLL_EINVAL;
      if (value == LINCOLL_PATH_STAGED && !staged_supported(pl->p.n, pl->p.dtype)) return LINCOLL_EINVAL;
      pl->p.path = value;
      break;
    default:
      return LINCOLL_EINVAL;
  }
  drop_graph(pl);
  return LINCOLL_OK;
}

namespace {

// A launch configuration of the apply: path, fused workgroups per CU,
// staged tile (z-pass block size, in-plane tile) and graph replay.
struct Tuned {
  int path, per_cu, zblk, tile, graph, ppt, keep, split;
  double ms;
};

// Process-wide cache of tuned configurations, keyed by the device
// architecture, n, dtype, the batch rounded up to a power of two, the
// projection flag and whether the Maxwellians are per cell.
std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tune_cache;

std::string tune_key(const lincoll_plan_s* pl, int batch) {
  int bucket = 1;
  while (bucket < batch) bucket <<= 1;
  return pl->arch + "|n" + std::to_string(pl->p.n) + "|d" + std::to_string(pl->p.dtype) + "|b" +
         std::to_string(bucket) + "|p" + std::to_string(pl->p.project) + "|c" + std::to_string(pl->Bc > 1 ? 1 : 0);
}

void apply_tuned(lincoll_plan_t pl, const Tuned& t) {
  pl->p.path = t.path;
  pl->opt_per_cu = t.per_cu;
  pl->opt_zblk = t.zblk;
  pl->opt_tile = t.tile;
  pl->opt_graph = t.graph;
  pl->opt_ppt = t.ppt;
  pl->opt_keep = t.keep;
  pl->opt_split = t.split;
  pl->tuned_ms = t.ms;
  drop_graph(pl);
}

}  // namespace

int lincoll_autotune(lincoll_plan_t pl, const void* h, void* out, int batch, int reps) {
  int st = checked_apply_args(pl, h, out, batch);
  if (st) return st;
  if (reps < 1 || reps > 1000) return LINCOLL_EINVAL;
  const std::string key = tune_key(pl, batch);
  if (pl->opt_tune_cache) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      apply_tuned(pl, it->second);
      pl->tuned_cached = 1;
      return LINCOLL_OK;
    }
  }
  std::vector<Tuned> cands;
  const int n = pl->p.n, dt = pl->p.dtype;
  // workgroups per cell: the split chosen by batch, and (where that splits)
  // one workgroup per cell
  std::vector<int> splits{0};
  if (fused_auto_split(n, pl->t.J, batch, pl->cus) > 1) splits.push_back(1);
  for (int g = 0; g < 2; ++g) {
    if (staged_supported(n, dt))
      for (int zb : {64, 128, 256})
        for (int tile = 0; tile <= (n <= 32 ? 1 : 0); ++tile)
          cands.push_back({LINCOLL_PATH_STAGED, 0, zb, tile, g, 1, -1, 0, 0.0});
    if (fused_supported(n, dt))
      for (int pc = 1; pc <= fused_max_per_cu(n); ++pc) {
        for (int keep : {0, 4, 8, 16})
          if (fused_keep_valid(n, dt, keep))
            for (int sp : splits) cands.push_back({LINCOLL_PATH_FUSED, pc, 128, 0, g, 1, keep, sp, 0.0});
        if (dt == LINCOLL_F32) cands.push_back({LINCOLL_PATH_FUSED, pc, 128, 0, g, 2, -1, 0, 0.0});
      }
  }
  if (cands.empty()) return LINCOLL_EINVAL;
  const Tuned saved{pl->p.path, pl->opt_per_cu, pl->opt_zblk, pl->opt_tile, pl->opt_graph, pl->opt_ppt, pl->opt_keep,
                    pl->opt_split, pl->tuned_ms};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1))) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(pl, e);
  }
  double best = 1e300;
  int bi = -1;
  for (size_t i = 0; i < cands.size() && !st; ++i) {
    apply_tuned(pl, cands[i]);
    if ((st = lincoll_apply(pl, h, out, batch))) break;   // warm-up (allocates, captures)
    if ((e = hipEventRecord(e0, pl->stream))) { st = hip_fail(pl, e); break; }
    for (int r = 0; r < reps && !st; ++r) st = lincoll_apply(pl, h, out, batch);
    if (st) break;
    float ms = 0.f;
    if ((e = hipEventRecord(e1, pl->stream)) || (e = hipEventSynchronize(e1)) || (e = hipEventElapsedTime(&ms, e0, e1))) {
      st = hip_fail(pl, e);
      break;
    }
    cands[i].ms = ms / reps;
    if (cands[i].ms < best) {
      best = cands[i].ms;
      bi = (int)i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st || bi < 0) {
    apply_tuned(pl, saved);
    return st ? st : LINCOLL_EINVAL;
  }
  apply_tuned(pl, cands[bi]);
  pl->tuned_cached = 0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = cands[bi];
  return LINCOLL_OK;
}

int quadcoll_apply(lincoll_plan_t pl, const void* f, void* out, int batch) {
  if (!pl || !f || !out || batch < 1) return LINCOLL_EINVAL;
  if (!quadcoll_supported(pl->p.n)) return LINCOLL_ENOTIMPL;
  if (pl->p.max_batch > 0 && batch > pl->p.max_batch) return LINCOLL_EINVAL;
  const int n = pl->p.n, J = pl->t.J, Q = pl->t.Q;
  const size_t n3 = (size_t)n * n * n, bytes = (size_t)batch * n3 * sizeof(double);
  const char* a = static_cast<const char*>(f);
  const char* b = static_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return LINCOLL_EINVAL;   // overlap
  std::vector<double> mu, wmu;
  if (!hemisphere_polar(pl->sphere_polar, mu, wmu)) return LINCOLL_EINVAL;
  hipError_t e;
  if (!pl->d_Ws) {
    // W_j s_j(|k|^2) = Phi_j / (4 pi^2), FP64
    std::vector<double> ws(pl->t.Phi);
    for (auto& v : ws) v /= 4.0 * M_PI * M_PI;
    if ((e = dalloc(pl, &pl->d_Ws, ws.size() * sizeof(double))) ||
        (e = hipMemcpy(pl->d_Ws, ws.data(), ws.size() * sizeof(double), hipMemcpyHostToDevice))) {
      dfree(pl->d_Ws);
      pl->d_Ws = nullptr;
      return hip_fail(pl, e);
    }
  }
  if (batch > pl->cap_qc) {
    const size_t cb = (size_t)batch * n3 * sizeof(double2);
    if ((e = dalloc(pl, &pl->d_qV, bytes)) || (e = dalloc(pl, &pl->d_qF, cb)) || (e = dalloc(pl, &pl->d_qGp, cb)) ||
        (e = dalloc(pl, &pl->d_qGm, cb)) || (e = dalloc(pl, &pl->d_qC, cb)) || (e = dalloc(pl, &pl->d_qS, cb)) ||
        (e = dalloc(pl, &pl->d_qQ, cb))) {
      pl->cap_qc = 0;
      return hip_fail(pl, e);
    }
    pl->cap_qc = batch;
  }
  const long nph = quadcoll_phase_count(n, (int)mu.size(), pl->sphere_azim);
  if (nph > pl->cap_qph) {
    if ((e = dalloc(pl, &pl->d_qPh, (size_t)nph * sizeof(double2)))) {
      pl->cap_qph = 0;
      return hip_fail(pl, e);
    }
    pl->cap_qph = nph;
  }
  std::vector<double> st(mu.size());
  for (size_t i = 0; i < mu.size(); ++i) st[i] = std::sqrt(1.0 - mu[i] * mu[i]);
  if (pl->quad_fix == 2 && (!pl->d_qOs || pl->qos_polar != pl->sphere_polar || pl->qos_azim != pl->sphere_azim)) {
    // loss weight of eq. (16) for this hemisphere rule, built on the device
    const int na = pl->sphere_azim, M = (int)mu.size() * na;
    std::vector<double> rule((size_t)M * 4), gw((size_t)J * 2);
    for (size_t i = 0; i < mu.size(); ++i)
      for (int m = 0; m < na; ++m) {
        const double ph = 2.0 * M_PI * m / na;
        double* r = &rule[((size_t)i * na + m) * 4];
        r[0] = st[i] * std::cos(ph);
        r[1] = st[i] * std::sin(ph);
        r[2] = mu[i];
        r[3] = wmu[i] / na;
      }
    for (int j = 0; j < J; ++j) {
      gw[2 * j] = pl->t.g[j];
      gw[2 * j + 1] = pl->t.W[j];
    }
    pl->qos_polar = pl->qos_azim = 0;
    if (!pl->d_qOs && (e = dalloc(pl, &pl->d_qOs, n3 * sizeof(double)))) return hip_fail(pl, e);
    if (!pl->d_qGW && (e = dalloc(pl, &pl->d_qGW, (size_t)J * 2 * sizeof(double)))) return hip_fail(pl, e);
    if ((long)rule.size() > pl->cap_qrule) {
      if ((e = dalloc(pl, &pl->d_qRule, rule.size() * sizeof(double)))) {
        pl->cap_qrule = 0;
        return hip_fail(pl, e);
      }
      pl->cap_qrule = (long)rule.size();
    }
    if ((e = hipMemcpy(pl->d_qRule, rule.data(), rule.size() * sizeof(double), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(pl->d_qGW, gw.data(), gw.size() * sizeof(double), hipMemcpyHostToDevice)) ||
        (e = quadcoll_sph_table(n, pl->d_qOs, pl->d_qGW, J, pl->d_qRule, M, pl->p.L, pl->stream)))
      return hip_fail(pl, e);
    pl->qos_polar = pl->sphere_polar;
    pl->qos_azim = pl->sphere_azim;
  }
  QuadCtx c;
  c.n = n;
  c.J = J;
  c.Q = Q;
  c.batch = batch;
  c.L = pl->p.L;
  c.stream = pl->stream;
  c.f = static_cast<const double*>(f);
  c.out = static_cast<double*>(out);
  c.V = pl->d_qV;
  c.Fk = pl->d_qF;
  c.Gp = pl->d_qGp;
  c.Gm = pl->d_qGm;
  c.C = pl->d_qC;
  c.S = pl->d_qS;
  c.Qk = pl->d_qQ;
  c.Om64 = pl->d_Om64;
  c.Ws = pl->d_Ws;
  c.g = pl->t.g.data();
  c.mu = mu.data();
  c.st = st.data();
  c.wpolar = wmu.data();
  c.npolar = (int)mu.size();
  c.nazim = pl->sphere_azim;
  c.phase = pl->d_qPh;
  c.fix = pl->quad_fix;
  c.Osph = pl->d_qOs;
  if ((e = quadcoll_apply_fp64(c))) return hip_fail(pl, e);
  return LINCOLL_OK;
}

namespace {

// One step of the classical fourth-order Runge-Kutta scheme for
// df/dt = L[f]: k1 = L f, k2 = L(f + dt/2 k1), k3 = L(f + dt/2 k2),
// k4 = L(f + dt k3), f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4).
hipError_t rk4_step(lincoll_plan_t pl, void* f, int batch, double dt, hipStream_t s) {
  const long cnt = (long)batch * pl->p.n * pl->p.n * pl->p.n;
  const int dt_ = pl->p.dtype == LINCOLL_F64 ? 0 : 1;
  void *k = pl->d_rk_k, *tmp = pl->d_rk_tmp, *acc = pl->d_rk_acc;
  hipError_t e;
  if ((e = launch_apply(pl, f, k, batch, s)) || (e = rk_stage(dt_, f, k, acc, tmp, cnt, dt / 6, dt / 2, 1, s)) ||
      (e = launch_apply(pl, tmp, k, batch, s)) || (e = rk_stage(dt_, f, k, acc, tmp, cnt, dt / 3, dt / 2, 0, s)) ||
      (e = launch_apply(pl, tmp, k, batch, s)) || (e = rk_stage(dt_, f, k, acc, tmp, cnt, dt / 3, dt, 0, s)) ||
      (e = launch_apply(pl, tmp, k, batch, s)) || (e = rk_final(dt_, f, acc, k, cnt, dt / 6, s)))
    return e;
  return hipSuccess;
}

}  // namespace

int lincoll_rk4(lincoll_plan_t pl, void* f, int batch, double dt, int steps) {
  if (!pl || !f || batch < 1 || steps < 0 || !std::isfinite(dt)) return LINCOLL_EINVAL;
  if (pl->p.max_batch > 0 && batch > pl->p.max_batch) return LINCOLL_EINVAL;
  if (pl->Bc != 1 && pl->Bc != batch) return LINCOLL_ENOTREADY;
  int st = ensure_work(pl, batch);
  if (st) return st;
  hipError_t e;
  if (batch > pl->cap_rk) {
    const size_t bytes = (size_t)batch * pl->p.n * pl->p.n * pl->p.n * esize(pl->p.dtype);
    if ((e = dalloc(pl, &pl->d_rk_k, bytes)) || (e = dalloc(pl, &pl->d_rk_tmp, bytes)) ||
        (e = dalloc(pl, &pl->d_rk_acc, bytes))) {
      pl->cap_rk = 0;
      return hip_fail(pl, e);
    }
    pl->cap_rk = batch;
  }
  if (!pl->opt_graph) {
    for (int i = 0; i < steps; ++i)
      if ((e = rk4_step(pl, f, batch, dt, pl->stream))) return hip_fail(pl, e);
    return LINCOLL_OK;
  }
  // record one step once, replay it `steps` times
  const lincoll_plan_s::GraphKey key{f, nullptr, batch, pl->Bc, use_fused(pl, batch) ? 1 : 0, pl->opt_per_cu,
                                     pl->p.project, pl->alloc_gen};
  const lincoll_plan_s::GraphKey& k = pl->rk_key;
  const bool same = pl->rk_gexec && k.h == key.h && k.batch == key.batch && k.Bc == key.Bc && k.fused == key.fused &&
                    k.per_cu == key.per_cu && k.project == key.project && k.gen == key.gen && pl->rk_dt == dt;
  if (!same) {
    if (pl->rk_gexec) (void)hipGraphExecDestroy(pl->rk_gexec);
    pl->rk_gexec = nullptr;
    if (!pl->cap_stream && (e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking))) return hip_fail(pl, e);
    if ((e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal))) return hip_fail(pl, e);
    const hipError_t el = rk4_step(pl, f, batch, dt, pl->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(pl->cap_stream, &g);
    if (el) e = el;
    if (!e) e = hipGraphInstantiate(&pl->rk_gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e) {
      pl->rk_gexec = nullptr;
      return hip_fail(pl, e);
    }
    pl->rk_key = key;
    pl->rk_dt = dt;
  }
  for (int i = 0; i < steps; ++i)
    if ((e = hipGraphLaunch(pl->rk_gexec, pl->stream))) return hip_fail(pl, e);
  if (steps > 0) {
    pl->last_path = key.fused ? LINCOLL_PATH_FUSED : LINCOLL_PATH_STAGED;
    pl->last_split = key.fused ? fused_split(pl, batch) : 1;
  }
  return LINCOLL_OK;
}

}  // extern "C"

namespace lincoll {
int plan_apply_on(lincoll_plan_s* pl, const void* h, void* out, int batch, hipStream_t s, const int* gate) {
  int st = checked_apply_args(pl, h, out, batch);
  if (st) return st;
  if ((st = ensure_work(pl, batch))) return st;
  const hipError_t e = launch_apply(pl, h, out, batch, s, gate);
  return e ? hip_fail(pl, e) : LINCOLL_OK;
}

int plan_ensure_work(lincoll_plan_s* pl, int batch) { return ensure_work(pl, batch); }

hipError_t plan_capture_stream(lincoll_plan_s* pl, hipStream_t* s) {
  if (!pl->cap_stream) {
    const hipError_t e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    if (e) return e;
  }
  *s = pl->cap_stream;
  return hipSuccess;
}

int plan_graph_option(const lincoll_plan_s* pl) { return pl->opt_graph; }

void* plan_steady_work(lincoll_plan_s* pl, size_t bytes, int* status) {
  *status = LINCOLL_OK;
  if (bytes > pl->cap_steady || !pl->d_steady) {
    pl->cap_steady = 0;
    const hipError_t e = dalloc(pl, &pl->d_steady, bytes);
    if (e) {
      *status = hip_fail(pl, e);
      return nullptr;
    }
    pl->cap_steady = bytes;
  }
  return pl->d_steady;
}

hipStream_t plan_stream(const lincoll_plan_s* pl) { return pl->stream; }
const void* plan_nu(const lincoll_plan_s* pl) { return pl->d_nu; }
void plan_note_hip(lincoll_plan_s* pl, hipError_t e) {
  pl->last_hip = (int)e;
  g_last_hip = (int)e;
}
}  // namespace lincoll

extern "C" {

void lincoll_debug_fail_alloc(int after) { g_fail_alloc_after = after > 0 ? after : 0; }

int lincoll_get_info(lincoll_plan_t pl, int key, double* val) {
  if (!pl && val && key == LINCOLL_INFO_HIP_ERROR) {   // last HIP error of this thread
    *val = g_last_hip;
    return LINCOLL_OK;
  }
  if (!pl || !val) return LINCOLL_EINVAL;
  switch (key) {
    case LINCOLL_INFO_N: *val = pl->p.n; break;
    case LINCOLL_INFO_J: *val = pl->t.J; break;
    case LINCOLL_INFO_R: *val = pl->p.R; break;
    case LINCOLL_INFO_DTYPE: *val = pl->p.dtype; break;
    case LINCOLL_INFO_PATH: *val = use_fused(pl, info_batch(pl)) ? LINCOLL_PATH_FUSED : LINCOLL_PATH_STAGED; break;
    case LINCOLL_INFO_MAXW_BATCH: *val = pl->Bc; break;
    case LINCOLL_INFO_DEVICE_BYTES: *val = (double)pl->bytes; break;
    case LINCOLL_INFO_HIP_ERROR: *val = pl->last_hip; break;
    case LINCOLL_INFO_EPS: *val = pl->p.eps; break;
    case LINCOLL_INFO_GRAPH: *val = pl->opt_graph; break;
    case LINCOLL_INFO_FUSED_PER_CU:
      *val = pl->opt_per_cu > 0 ? pl->opt_per_cu : fused_max_per_cu(pl->p.n);
      break;
    case LINCOLL_INFO_TUNED_MS: *val = pl->tuned_ms; break;
    case LINCOLL_INFO_L: *val = pl->p.L; break;
    case LINCOLL_INFO_PROJECT: *val = pl->p.project; break;
    case LINCOLL_INFO_QUAD_FIX: *val = pl->quad_fix; break;
    case LINCOLL_INFO_ZBLOCK: *val = pl->opt_zblk; break;
    case LINCOLL_INFO_PLANE_TILE: *val = pl->opt_tile; break;
    case LINCOLL_INFO_TUNE_CACHED: *val = pl->tuned_cached; break;
    case LINCOLL_INFO_FUSED_PPT: *val = pl->opt_ppt; break;
    case LINCOLL_INFO_FUSED_KEEP: *val = fused_keep(pl); break;
    case LINCOLL_INFO_LAST_PATH: *val = pl->last_path; break;
    case LINCOLL_INFO_FUSED_SPLIT: *val = pl->last_split; break;
    default: return LINCOLL_EINVAL;
  }
  return LINCOLL_OK;
}

void lincoll_destroy(lincoll_plan_t pl) {
  if (!pl) return;
  (void)hipStreamSynchronize(pl->stream);
  drop_graph(pl);
  if (pl->rk_gexec) (void)hipGraphExecDestroy(pl->rk_gexec);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  void* ptrs[] = {pl->d_Phi,  pl->d_Om,    pl->d_Om64,  pl->d_phi,  pl->d_Cdct, pl->d_params, pl->d_fac64,
                  pl->d_pref64, pl->d_gfac64, pl->d_Ainv, pl->d_facT, pl->d_prefT, pl->d_mask,  pl->d_Kh,
                  pl->d_nu,   pl->d_tmpA,  pl->d_tmpB,  pl->d_planes64, pl->d_R, pl->d_H, pl->d_W, pl->d_Wq, pl->d_Lp, pl->d_pin,
                  pl->d_rk_k, pl->d_rk_tmp, pl->d_rk_acc, pl->d_Ws, pl->d_qV, pl->d_qF, pl->d_qGp,
                  pl->d_qGm, pl->d_qC, pl->d_qS, pl->d_qQ, pl->d_qPh, pl->d_qOs, pl->d_qGW, pl->d_qRule, pl->d_steady,
                  pl->d_flag};
  for (void* p : ptrs) dfree(p);
  delete pl;
}

}  // extern "C"
