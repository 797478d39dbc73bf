// Internal interfaces between the ABI layer and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

struct lincoll_plan_s;

namespace lincoll {

// Plan accessors for host code outside the ABI translation unit.
hipStream_t plan_stream(const lincoll_plan_s* pl);
void plan_note_hip(lincoll_plan_s* pl, hipError_t e);   // records e as the plan's last HIP error
// Loss collision frequency nu = iDFT[Omega DFT[M]] of the Maxwellians set,
// [Bc][n^3], double for LINCOLL_F64 plans and float otherwise.
const void* plan_nu(const lincoll_plan_s* pl);
// lincoll_apply's checks and launches on stream s, never through a recorded
// graph (so that a caller can record it into a graph of its own), with the
// fused kernel and the projections gated by *gate (nullptr: always run).
// Work buffers are allocated here if needed: call once outside any capture.
int plan_apply_on(lincoll_plan_s* pl, const void* h, void* out, int batch, hipStream_t s, const int* gate);
// The apply work buffers for batch cells (lincoll_apply allocates them on
// first use; a caller that records launches into a graph calls this first).
int plan_ensure_work(lincoll_plan_s* pl, int batch);
// A stream the plan owns for recording graphs (created on first use).
hipError_t plan_capture_stream(lincoll_plan_s* pl, hipStream_t* s);
// 1 if the plan replays recorded graphs (LINCOLL_OPT_GRAPH).
int plan_graph_option(const lincoll_plan_s* pl);
// Device work memory of the steady solver, owned by the plan and kept between
// calls (grown when a call needs more; freed with the plan).  Returns null and
// sets *status on failure.
void* plan_steady_work(lincoll_plan_s* pl, size_t bytes, int* status);

// Row strides of the device mode tables (K_j octants and Phi_j radial
// tables), padded to whole blocks of 512 values so that the fused kernel copies
// a row into LDS with the same fixed number of load instructions per wave.
constexpr int pad512(int x) { return (x + 511) / 512 * 512; }
constexpr int kh_stride(int n) { return pad512((n / 2 + 1) * (n / 2 + 1) * (n / 2 + 1)); }
constexpr int phi_stride(int n) { return pad512(3 * (n / 2) * (n / 2) + 1); }

// Everything one staged or fused apply needs (raw device pointers; element
// type is double for dtype 0 and float otherwise; complex = interleaved).
struct ApplyCtx {
  int n = 0, J = 0, Q = 0;
  int batch = 0, Bc = 0;       // cells in this call; cells in the Maxwellian cache (1 = broadcast)
  int cus = 256;               // compute units of the device
  int per_cu = 0;              // fused path: workgroups per compute unit (0 = default)
  int max_slots = 0;           // fused path: cap on the persistent workgroups (0 = none)
  int fused_ppt = 1;           // fused path: pencils per thread (1: k_fused, 2: k_fused2)
  int fused_keep = 0;          // k_fused: accumulator chunks kept in registers (fused_keep_valid)
  int fused_split = 1;         // fused path: workgroups per cell (1: k_fused; S > 1: k_fused_split, k_fused_finish)
  int zblk = 128;              // staged path: threads per block of the z-pass kernels (64, 128, 256)
  int plane_tile = 0;          // staged path: 0 = 64-thread in-plane blocks, 1 = 32-thread (n <= 32)
  const int* gate = nullptr;   // fused path: the kernel does nothing unless *gate != 0 (device flag)
  int dtype = 0;
  hipStream_t stream = nullptr;
  const void* h = nullptr;
  void* out = nullptr;
  const void* Phi = nullptr;   // [J][phi_stride(n)]  Phi_j(|k|^2) / n^3
  const void* Om = nullptr;    // [Q]     Omega(|k|^2) / n^3
  const void* fac = nullptr;   // [Bc][6][n]: exp(-(v-u_d)^2/(2 theta)), d = 1..3; then exp(-(v-u_d)^2/theta)
  const void* pref = nullptr;  // [Bc][2]: rho (2 pi theta)^-3/2, rho (pi theta)^-3/2
  const double* fac64 = nullptr;   // the same two in FP64
  const double* pref64 = nullptr;
  const uint32_t* mask = nullptr;  // [Bc][n*n][(n+31)/32] cutoff bits along z
  const void* Kh = nullptr;    // [Bc][J][kh_stride(n)]  K_j / n^3 on the octant [P][P][P], P = n/2+1, double
  const void* nu = nullptr;    // [Bc][n^3]
  void* R = nullptr;           // work, complex [batch][P][n][n] each; R and W in double
  void* H = nullptr;
  void* W = nullptr;
  void* Wq = nullptr;
  void* Lp = nullptr;
};

// Per-cell FP64 setup context.
struct SetupCtx {
  int n = 0, J = 0, Q = 0;
  int Bc = 0;
  int dtype = 0;
  double L = 0.0, eps = 0.0;
  hipStream_t stream = nullptr;
  const double* params = nullptr;  // [Bc][5]
  const double* phi = nullptr;     // [J][P^3]
  const double* Cdct = nullptr;    // [P][P]
  const double* Om64 = nullptr;    // [Q] Omega / n^3, FP64
  double* fac64 = nullptr;         // [Bc][6][n]
  double* pref64 = nullptr;        // [Bc][2]
  double* gfac64 = nullptr;        // [Bc][P]
  double* Ainv = nullptr;          // [Bc][25]
  void* facT = nullptr;            // copies in the apply dtype
  void* prefT = nullptr;
  uint32_t* mask = nullptr;
  void* Kh = nullptr;              // [Bc][J][kh_stride(n)] double for every dtype (octant [P][P][P] first)
  void* nu = nullptr;              // [Bc][n^3] apply dtype
  double* tmpA = nullptr;          // scratch, [chunk][J][P^3] FP64 each
  double* tmpB = nullptr;
  double* planes64 = nullptr;      // scratch, complex double [chunk][P][n][n]
  int chunk = 0;                   // cells per scratch pass
};

struct ProjectCtx {
  int n = 0, batch = 0, Bc = 0, dtype = 0;
  double L = 0.0;
  hipStream_t stream = nullptr;
  const void* x = nullptr;
  void* y = nullptr;
  const double* fac64 = nullptr;
  const double* pref64 = nullptr;
  const double* Ainv = nullptr;
  const int* gate = nullptr;       // nothing is done unless *gate != 0
};

// Binary operator Q(f, f) (eq. (14)), FP64.
struct QuadCtx {
  int n = 0, J = 0, Q = 0, batch = 0;
  double L = 0.0;
  hipStream_t stream = nullptr;
  const double* f = nullptr;     // [batch][n^3] physical
  double* out = nullptr;         // [batch][n^3]
  double* V = nullptr;           // [batch][n^3] loss field
  double2 *Fk = nullptr, *Gp = nullptr, *Gm = nullptr, *C = nullptr, *S = nullptr, *Qk = nullptr;   // [batch][n^3]
  const double* Om64 = nullptr;  // [Q] Omega / n^3
  const double* Ws = nullptr;    // [J][Q] W_j s_j(|k|^2)
  const double* g = nullptr;     // host [J]
  const double* mu = nullptr;    // host [npolar] polar cosines
  const double* st = nullptr;    // host [npolar] sqrt(1 - mu^2)
  const double* wpolar = nullptr;   // host [npolar] polar weights
  int npolar = 0, nazim = 0;
  double2* phase = nullptr;      // [npolar][nazim/2+1][4][n] phase tables of one g-node (quadcoll_phase_count)
  int fix = 0;                   // mass fix of Sec. 2.3: 0 none, 1 Q^_0 = 0 (eq. (15)), 2 sinc estimated (eq. (16))
  const double* Osph = nullptr;  // fix 2: [n][n][n] loss weight (quadcoll_sph_table)
};
// The loss weight of the second mass fix into tab [n][n][n] (natural order,
// [kz][kx][ky]); gw = device [J][2] (g_j, W_j), rule = device [nsph][4].
hipError_t quadcoll_sph_table(int n, double* tab, const double* gw, int J, const double* rule, int nsph, double L,
                              hipStream_t s);
// complex values of the phase tables of QuadCtx::phase
inline long quadcoll_phase_count(int n, int npolar, int nazim) { return (long)npolar * (nazim / 2 + 1) * 4 * n; }
bool quadcoll_supported(int n);
hipError_t quadcoll_apply_fp64(const QuadCtx& c);

hipError_t staged_apply(const ApplyCtx& c);
hipError_t setup_cells(const SetupCtx& c);
hipError_t project_cells(const ProjectCtx& c);
bool staged_supported(int n, int dtype);
bool fused_supported(int n, int dtype);
hipError_t fused_apply(const ApplyCtx& c);
// BF16x3 matrix-core forward plane transform of the gain loop (n = 32, 64):
// out = (first ? 0 : out) + Phi_j * DFT2(in) over the planes [nplanes][n][n].
hipError_t plane_fwd_bf16x3(int n, const float2* in, float2* out, const float* table, int j, int nplanes, int first,
                            int cus, hipStream_t s);
// RK4 stage combinations (double arithmetic on the dtype's storage)
hipError_t rk_stage(int dtype, const void* f, const void* k, void* acc, void* tmp, long count, double a, double b,
                    int first, hipStream_t s);
hipError_t rk_final(int dtype, void* f, const void* acc, const void* k, long count, double a, hipStream_t s);
size_t fused_scratch_bytes(int n, int nslots, int ppt, int dtype);
bool fused_keep_valid(int n, int dtype, int keep);
// Sets *flag (device int) to 1 if any of x[0 .. count) is NaN or infinite,
// else 0 (double if dtype_f64, float otherwise); enqueued on s.
hipError_t nonfinite_check(const void* x, long count, int dtype_f64, int* flag, hipStream_t s);
int fused_default_keep(int n, int dtype);
// The fixed device scratch of lincoll_apply_noalloc on `device` (which must
// be current): its address and size.
hipError_t fused_noalloc_scratch(int device, void** ptr, size_t* bytes);
int fused_max_per_cu(int n);
int fused_slots(int n, int batch, int per_cu, int cus);
// Parts per cell that spread a batch of n-point cells over the chip (at most
// one work item per resident workgroup, one of a cell's kept for its loss
// term where possible, and J parts; the fewest parts with the shortest
// longest part); 1 once the batch alone fills it.
int fused_auto_split(int n, int J, int batch, int cus);
// Bytes of R a split apply needs: the slots of its workgroups, then the
// partial gain sums of batch * S work items (256-byte aligned).
size_t fused_split_scratch_bytes(int n, int nslots, int batch, int S, int dtype);
// 1 if a split apply gives the loss term a work item of its own (S + 1 items
// per cell), which it does while that many items still fit the chip at once.
int fused_loss_item(int n, int batch, int S, int cus);
size_t fused_partial_offset(int n, int nslots, int dtype);

}  // namespace lincoll
