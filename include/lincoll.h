/*
 * lincoll: the linearized Boltzmann collision operator for VHS gases by the
 * fast Fourier spectral method of Yin, Cai and Wang (arXiv 2503.09580),
 * on AMD Instinct MI355X (gfx950).
 *
 * Operator (Sec. 2.1, eq. (5)):  L[h] = Q(M,h) + Q(h,M)  about a Maxwellian
 *   M(v) = rho (2 pi theta)^(-3/2) exp(-|v-u|^2 / (2 theta)),
 * VHS kernel B(g) = C g^(2(1-omega)) (eq. (4)), truncated at g <= R.
 * Discretisation (Sec. 2.3, Sec. 3.2 eqs. (20), (23), (24), Algorithm 1):
 * n points per velocity axis on the periodic box [-L, L)^3,
 *   v_i = -L + i * 2L/n,  i = 0..n-1,
 * g-quadrature by a Jacobi-Gauss-Radau rule with J = n/2 + 1 nodes, and the
 * cutoff r = h/M only where M/rho >= eps (eq. (25)).  Each application costs
 * O(J n^3 log n) with no sum over sphere points.
 *
 * Conventions shared by every entry point
 *   - Arrays h, out, x are device memory, row-major [batch][n][n][n]
 *     (last index fastest, index i <-> velocity -L + i*2L/n).  Element type
 *     is double for LINCOLL_F64 and float for LINCOLL_F32 / LINCOLL_BF16X3.
 *   - Maxwellian parameters are device memory, double [batch][5] holding
 *     (rho, u1, u2, u3, theta) per cell, rho > 0, theta > 0.
 *   - The caller owns h, out, x and the parameter array; the plan owns all
 *     tables, per-cell caches and scratch, and frees them in lincoll_destroy.
 *   - Every call is asynchronous on the plan's stream (lincoll_set_stream;
 *     the null stream until set).  Completion follows stream order.
 *   - A plan is not thread-safe; distinct plans are independent.
 *   - Functions return LINCOLL_OK (0) or a negative status; nothing throws
 *     across this interface.  Argument checks happen on the host before any
 *     device work is enqueued.
 */
#ifndef LINCOLL_H
#define LINCOLL_H

#ifdef __cplusplus
extern "C" {
#endif

#define LINCOLL_OK 0
#define LINCOLL_EINVAL -1    /* bad argument: n, L, omega, dtype, batch, null or aliased pointer */
#define LINCOLL_ENOMEM -2    /* device allocation failed */
#define LINCOLL_EHIP -3      /* a HIP runtime call failed (lincoll_get_info LINCOLL_INFO_HIP_ERROR) */
#define LINCOLL_ENOTREADY -4 /* batch does not match the Maxwellians set (neither 1 nor batch) */
#define LINCOLL_ENOTIMPL -5  /* operation not provided by this build */
#define LINCOLL_EDIVERGED -6 /* an iterate left the admissible set (density or temperature <= 0, non-finite values) */
#define LINCOLL_ENONFINITE -7 /* debug check (LINCOLL_OPT_CHECK_FINITE): the output holds NaN or infinite values */

typedef struct lincoll_plan_s* lincoll_plan_t;

typedef enum {
  LINCOLL_F64 = 0,   /* every step in double */
  LINCOLL_F32 = 1,   /* transforms and mode products in float; setup, mask and projection in double */
  LINCOLL_BF16X3 = 2 /* as F32, with the two in-plane forward DFT stages of the gain loop as split-bfloat16
                        (hi + lo, three products, FP32 accumulation) matrix-core GEMMs; staged path, n = 32, 64 */
} lincoll_dtype_t;

typedef enum {
  LINCOLL_PATH_AUTO = 0,    /* the fused kernels where they exist (F32 and F64 at n = 16, 32), for any batch:
                               batches smaller than the device's compute unit count are split over several
                               workgroups per cell (LINCOLL_OPT_FUSED_SPLIT).  With splitting switched off
                               (LINCOLL_OPT_FUSED_SPLIT = 1) or two pencils per thread, n = 32 takes the
                               staged kernels below 16 cells (F32) or 128 cells (F64).  Otherwise (n = 8,
                               64, BF16X3) the staged kernels */
  LINCOLL_PATH_STAGED = 1,  /* batched per-stage kernels (every n and dtype) */
  LINCOLL_PATH_FUSED = 2    /* persistent workgroups, one per cell or S per cell (LINCOLL_OPT_FUSED_SPLIT)
                               (F32 and F64 at n = 16, 32) */
} lincoll_path_t;

typedef struct {
  int n;            /* points per velocity axis (the paper's 2N): 8, 16, 32 or 64 (BF16X3: 32, 64) */
  double L;         /* half-width of the periodic velocity box, > 0 */
  double omega;     /* VHS viscosity index, 1/2 <= omega <= 1 (eq. (4)) */
  double C;         /* kernel constant of B(g) = C g^(2(1-omega)); default 1/(4 pi) (eq. (26)) */
  double R;         /* kernel cutoff; <= 0 selects 4L/(3+sqrt 2), the largest de-aliased value (Sec. 2.3) */
  int J;            /* g-quadrature nodes; <= 0 selects n/2 + 1 (exact to degree n, Sec. 4.1) */
  double eps;       /* cutoff of eq. (25); default 1e-9; 0 disables it */
  int quad_rule;    /* 0: Radau weight (1+x)^(4-2 omega) absorbs g^2 B(g); 1: weight (1+x)^2 times B(g_j) */
  int project;      /* 1: lincoll_apply returns P L P (exact conservation), see lincoll_project */
  int max_batch;    /* upper bound on batch accepted by apply (0: unbounded) */
  int dtype;        /* lincoll_dtype_t */
  int path;         /* lincoll_path_t */
} lincoll_params_t;

/* Fills *p with the defaults above for (n, L, omega, dtype). */
void lincoll_params_default(lincoll_params_t* p, int n, double L_domain, double vhs_omega, int dtype);

/* Creates a plan: host FP64 precomputation of Algorithm 1 (quadrature, the
 * kernel-mode tables s_j, Phi_j, Omega and phi_j = iDFT[s_j]), upload, and the
 * default Maxwellian (rho, u, theta) = (1, 0, 1) for one cell.  Synchronous. */
int lincoll_plan(int n, double L_domain, double vhs_omega, int dtype, lincoll_plan_t* out);
int lincoll_plan_ex(const lincoll_params_t* p, lincoll_plan_t* out);

/* Sets the HIP stream (a hipStream_t passed as void*) for all later calls. */
int lincoll_set_stream(lincoll_plan_t plan, void* hip_stream);

/* Per-cell Maxwellians (Algorithm 1, first loop; the modified Newton
 * operator of Sec. 5.2, eq. (modified_lin_eq), uses one local Maxwellian per
 * spatial cell).  params: device double [batch][5].  Computes
 * in FP64 on the device: the cutoff mask, the kernel modes
 * K_j = DFT[G phi_j] with G = rho (pi theta)^(-3/2) exp(-|v|^2/theta) (eq. (24)),
 * nu = iDFT[Omega DFT[M]] (eq. (20)) and the invariant Gram matrix.  batch = 1
 * is broadcast to every cell of a later apply.  Asynchronous. */
int lincoll_set_maxwellians(lincoll_plan_t plan, const double* params, int batch);

/* out[b] = L[h[b]] about Maxwellian b (or the broadcast one) for b < batch
 * (eq. (20) + eq. (23), Algorithm 1).  h and out must not overlap.
 * batch >= 1 and, when the plan sets max_batch, batch <= max_batch (else
 * LINCOLL_EINVAL, nothing enqueued); batch must equal the Maxwellian batch or
 * the Maxwellian batch must be 1 (else LINCOLL_ENOTREADY). */
int lincoll_apply(lincoll_plan_t plan, const void* h, void* out, int batch);

/* lincoll_apply without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and argument checks as
 * lincoll_apply.  A batch that the plan splits over several workgroups per
 * cell (LINCOLL_OPT_FUSED_SPLIT) is split the same way when its slots and
 * partial sums fit the array (one cell at n = 32 needs about 10 MiB); the
 * output is then bitwise identical to lincoll_apply's on the same plan, as
 * it is for an unsplit batch.  A split batch that does not fit runs one
 * workgroup per cell and agrees with lincoll_apply to rounding.  It calls no
 * hipMalloc, hipFree or other allocating routine and never records a
 * graph: the fused kernels' per-workgroup scratch (the spectrum of r and the
 * L+ accumulator) and a split's partial sums live in a fixed 96 MiB device
 * array of the library, one per GPU, held until the process ends, which
 * limits the persistent workgroups to 256 at n = 32 and 1024 at n = 16 for
 * F32 plans, 192 and 1536 for F64 (whose accumulator is double); any batch
 * is processed, the workgroups loop over cells.  Nothing in that array needs
 * to start at zero.  All calls on one GPU share it: calls that overlap in
 * time on one GPU (other streams, other plans, other threads) race and give
 * wrong results; serialise them.  Requirements beyond lincoll_apply's: the
 * plan's apply of this batch takes the fused path (LINCOLL_F32 or
 * LINCOLL_F64, n = 16 or 32, path FUSED or AUTO; see LINCOLL_PATH_AUTO),
 * project = 0, the Maxwellians already set (lincoll_set_maxwellians
 * allocates), and the plan's device current; otherwise LINCOLL_EINVAL. */
int lincoll_apply_noalloc(lincoll_plan_t plan, const void* h, void* out, int batch);

/* y[b] = P x[b]: removes the collision-invariant part in the inner product
 * <a,b> = sum a b / M, i.e. y = x - M sum_a phi_a (A^-1 m[x])_a with
 * phi_a in {1, v1, v2, v3, |v|^2}, A_ab = sum M phi_a phi_b, m_a = sum x phi_a.
 * Then sum y phi_a = 0 and P(phi_a M) = 0.  Reductions in FP64 for every
 * dtype.  x == y is allowed. */
int lincoll_project(lincoll_plan_t plan, const void* x, void* y, int batch);

/* out[b] = Q(f[b], f[b]), the binary collision operator by the spectral
 * method of Sec. 2.3, eq. (14) (the mass fix of LINCOLL_OPT_QUAD_FIX, none by
 * default), with the plan's
 * g-quadrature (W_j, g_j, as for the linearized operator) and a product rule
 * on the hemisphere: the positive nodes of the LINCOLL_OPT_SPHERE_POLAR-point
 * Gauss-Legendre rule (default 8, i.e. 4 polar cosines) times
 * LINCOLL_OPT_SPHERE_AZIMUTH equispaced azimuths (default 16); 64 points by
 * default.  Always FP64, whatever the plan's dtype: f and out are device
 * double [batch][n][n][n], not overlapping.  Independent of the Maxwellians.
 * Work volumes (7 n^3 doubles complex per cell) belong to the plan.  Cost:
 * per cell 2 J M + J + 4 complex 3-D transforms (M hemisphere points).
 * n = 8, 16, 32; other n give LINCOLL_ENOTIMPL. */
int quadcoll_apply(lincoll_plan_t plan, const void* f, void* out, int batch);

#define LINCOLL_INFO_N 0
#define LINCOLL_INFO_J 1
#define LINCOLL_INFO_R 2
#define LINCOLL_INFO_DTYPE 3
#define LINCOLL_INFO_PATH 4          /* path an apply of the Maxwellian batch takes (of a large batch when the
                                        Maxwellians are broadcast or not yet set), as lincoll_path_t */
#define LINCOLL_INFO_MAXW_BATCH 5    /* batch of the Maxwellians currently set */
#define LINCOLL_INFO_DEVICE_BYTES 6  /* device memory held by the plan */
#define LINCOLL_INFO_HIP_ERROR 7     /* last hipError_t seen (0 if none) */
#define LINCOLL_INFO_EPS 8
#define LINCOLL_INFO_GRAPH 9         /* 1 if applies replay a captured graph (LINCOLL_OPT_GRAPH) */
#define LINCOLL_INFO_FUSED_PER_CU 10 /* fused-path workgroups per compute unit in effect */
#define LINCOLL_INFO_TUNED_MS 11     /* ms per apply of the configuration lincoll_autotune chose (0 if never run) */
#define LINCOLL_INFO_L 12            /* half-width L of the velocity box */
#define LINCOLL_INFO_PROJECT 13      /* 1 if applies return P L P */
#define LINCOLL_INFO_QUAD_FIX 14     /* mass fix of quadcoll_apply (LINCOLL_OPT_QUAD_FIX) */
#define LINCOLL_INFO_ZBLOCK 15       /* staged path: threads per block of the z-pass kernels */
#define LINCOLL_INFO_PLANE_TILE 16   /* staged path: in-plane tile (0: 64 threads, 1: 32 threads per block) */
#define LINCOLL_INFO_TUNE_CACHED 17  /* 1 if the last lincoll_autotune took its result from the cache */
#define LINCOLL_INFO_FUSED_PPT 18    /* fused path: pencils per thread (LINCOLL_OPT_FUSED_PPT) */
#define LINCOLL_INFO_FUSED_KEEP 19   /* fused path: accumulator chunks kept in registers, in effect */
#define LINCOLL_INFO_LAST_PATH 20    /* path the most recent apply (of any batch) took; 0 before the first.  Set
                                        when the launches are enqueued (or recorded into a graph) */
#define LINCOLL_INFO_FUSED_SPLIT 21  /* workgroups per cell of the most recent apply: S > 1 when it took the
                                        fused path split S ways (LINCOLL_OPT_FUSED_SPLIT), else 1 */
/* Reads one plan property into *val.  With plan == NULL only
 * LINCOLL_INFO_HIP_ERROR is accepted: the last HIP error seen on this thread
 * (for a lincoll_plan/lincoll_plan_ex that failed with LINCOLL_EHIP). */
int lincoll_get_info(lincoll_plan_t plan, int key, double* val);

/* Execution options (batching row of the design: launch shape and launch
 * mechanism of the persistent path).  Every change drops a captured graph.
 *   LINCOLL_OPT_GRAPH        0 | 1.  With 1, an apply records its launches
 *                            once into a hipGraph (kernel nodes only, on a
 *                            stream the plan owns) and replays it with one
 *                            hipGraphLaunch on the plan's stream for as long
 *                            as h, out, batch, the Maxwellian batch, the
 *                            options and the plan's buffers stay the same;
 *                            otherwise it records again.  Leave it 0 when
 *                            the caller captures lincoll_apply into a graph
 *                            of its own.
 *   LINCOLL_OPT_FUSED_PER_CU workgroups of the fused path per compute unit:
 *                            0 = default (the maximum), n = 16: 1..4,
 *                            n = 32: 1.
 *   LINCOLL_OPT_PATH         a lincoll_path_t the plan's n and dtype support.
 *   LINCOLL_OPT_SPHERE_POLAR, LINCOLL_OPT_SPHERE_AZIMUTH
 *                            hemisphere rule of quadcoll_apply.
 * Returns LINCOLL_EINVAL for an unknown key or an unsupported value. */
#define LINCOLL_OPT_GRAPH 0
#define LINCOLL_OPT_FUSED_PER_CU 1
#define LINCOLL_OPT_PATH 2
#define LINCOLL_OPT_SPHERE_POLAR 3    /* quadcoll: Gauss-Legendre order on [-1,1] (even, 2..64; positive nodes used) */
#define LINCOLL_OPT_SPHERE_AZIMUTH 4  /* quadcoll: azimuths (1..256) */
#define LINCOLL_OPT_PROJECT 5         /* 0 | 1: as lincoll_params_t.project */
#define LINCOLL_OPT_ZBLOCK 7          /* staged path: threads per block of the z-pass kernels, 64 | 128 (default) | 256 */
#define LINCOLL_OPT_PLANE_TILE 8      /* staged path: in-plane kernels with 64 (0, default) or 32 (1, n <= 32)
                                         threads per block, i.e. 64/n or 32/n planes per block */
#define LINCOLL_OPT_TUNE_CACHE 9      /* 1 (default): lincoll_autotune reuses a cached result; 0: always times */
#define LINCOLL_OPT_CHECK_FINITE 12   /* debug: 1 = after each lincoll_apply, scan the output for NaN or infinite
                                         values on the plan's stream and read the result back (the call then
                                         synchronises the stream); returns LINCOLL_ENONFINITE if any, the output
                                         as computed.  Not for callers that capture lincoll_apply into a graph
                                         (the read-back cannot be captured).  0 (default): no check */
#define LINCOLL_OPT_FUSED_PPT 10      /* fused path: pencils per thread, 1 (default: two waves per SIMD, the L+^
                                         accumulator partly streamed through the workgroup's scratch slot every
                                         node, see LINCOLL_OPT_FUSED_KEEP) or 2 (one wave per SIMD with the whole
                                         register file per lane; the accumulator stays in registers).  The same
                                         arithmetic; results agree to float rounding (the two kernels are
                                         compiled separately and may contract differently).  F32 plans only */
#define LINCOLL_OPT_FUSED_KEEP 11     /* fused path, one pencil per thread: how many chunks of each thread's
                                         L+^ accumulator stay in registers across the quadrature nodes instead of
                                         making a round trip through LDS or the scratch slot.  F32 (chunks of two
                                         complex floats): 0, 4, 8 (all at n = 16), 16 (n = 32, all); default 8.
                                         F64 (chunks of one complex double): n = 16: 0, 8, 16 (all), default 16;
                                         n = 32: 0, 4, 8, default 0.  -1 restores the default.  The same
                                         additions in the same order for every value: F32 results are bitwise
                                         equal; F64 results agree to a few units in the last place (the compiler
                                         may contract the M^h product into the next addition differently in
                                         each compiled instance) */
#define LINCOLL_OPT_FUSED_SPLIT 13    /* fused path, one pencil per thread: workgroups per cell.  The gain loop of
                                         Algorithm 1 is partitioned: part p of a cell takes the nodes j = p, p + S,
                                         ..., computes its own spectrum of r, and writes its partial sum of
                                         Phi_j Q_j to the plan's work memory (part 0 also writes the loss term);
                                         two more kernels add the S parts in order and apply the final inverse
                                         transform.  Where the chip holds S + 1 work items per cell at once,
                                         the loss term gets an item of its own and runs beside the gain parts.
                                         0 (default): by batch -- a batch with fewer cells than the device holds
                                         workgroups at once (one per compute unit at n = 32, four at n = 16) is
                                         split into at most J parts and at most (resident workgroups / batch)
                                         work items per cell, one kept for the loss where that leaves two parts:
                                         the fewest parts whose longest part has the fewest nodes (one cell at
                                         n = 32: 17 parts; 16 cells: 9 parts of at most 2 nodes; 64 cells: 3
                                         parts), so that small batches use the whole chip; 1: never split;
                                         S = 2..J: S parts.  Results agree with the
                                         unsplit kernel to rounding (the gain sum is associated differently).
                                         lincoll_apply_noalloc always runs unsplit */
#define LINCOLL_OPT_QUAD_FIX 6        /* quadcoll: mass fix of Sec. 2.3 -- 0 none (default); 1 Q^_0 = 0 (eq. (15)),
                                         the per-cell mean of Q removed; 2 the sinc of the loss term replaced by
                                         its estimate on the hemisphere rule (eq. (16)), a [n]^3 FP64 table the
                                         plan builds on the device once per rule */
int lincoll_set_option(lincoll_plan_t plan, int key, int value);

/* Launch-configuration tuner: times `reps` applies of every supported
 * configuration on the caller's h/out/batch (after one warm-up each): path;
 * on the fused path the workgroups per CU, the pencils per thread
 * (LINCOLL_OPT_FUSED_PPT), the accumulator split (LINCOLL_OPT_FUSED_KEEP)
 * and, for a batch that AUTO splits, split or not (LINCOLL_OPT_FUSED_SPLIT
 * 0 or 1); on the staged path the z-pass
 * block size (64, 128, 256) and the in-plane tile (LINCOLL_OPT_ZBLOCK,
 * LINCOLL_OPT_PLANE_TILE); graph replay on and off.  Keeps the fastest as the
 * plan's configuration, records its time (LINCOLL_INFO_TUNED_MS) and stores
 * it in a process-wide cache keyed by (device architecture, n, dtype, batch
 * rounded up to a power of two, projection flag, per-cell or broadcast
 * Maxwellians); a later call with the same key takes the cached result
 * without timing (LINCOLL_INFO_TUNE_CACHED = 1) unless LINCOLL_OPT_TUNE_CACHE
 * is 0.  No configuration changes the arithmetic of a path beyond the
 * association of sums (the split).  Synchronises the
 * plan's stream; out holds L[h] afterwards (after a cache hit it is not
 * written).  Same argument rules as lincoll_apply; reps in [1, 1000]. */
int lincoll_autotune(lincoll_plan_t plan, const void* h, void* out, int batch, int reps);

/* Advances f[b] in place by `steps` steps of the classical fourth-order
 * Runge-Kutta scheme with step dt for the spatially homogeneous linearized
 * equation df/dt = L[f] about the plan's Maxwellians (Sec. 4.2; four applies
 * per step).  f: device [batch][n][n][n] in the apply dtype; the stage
 * buffers belong to the plan.  With LINCOLL_OPT_GRAPH one whole step is
 * recorded once (for this f, batch and dt) and replayed.  Same batch rules
 * as lincoll_apply; steps >= 0. */
int lincoll_rk4(lincoll_plan_t plan, void* f, int batch, double dt, int steps);

/* ---- Steady 1-D problem with diffuse walls (Sec. 5, Appendix B) ----------
 * v1 d_x f = Q(f,f)/Kn on x in (x_l, x_r), first-order upwind finite volumes
 * (eq. (discrete_eq)) on nx cells, the plan's velocity grid, fully
 * accommodating walls (eq. (maxwell_bc)) through ghost cells, and the
 * total-mass constraint dx h_v^3 sum f = C (eq. (total_mass)).
 * Readings this library takes where the printed scheme leaves a choice:
 *   - wall densities make the discrete mass flux through each wall exactly
 *     zero: ghost f_0 = rho_L E_L with rho_L = -sum v1- f_1 / sum v1+ E_L,
 *     E_W(v) = exp(-|v-u_W|^2/(2 theta_W)), and the mirror image at x_r (the
 *     printed constants are the continuum limit of this normalisation);
 *   - the residual r = T[f] - Q(f,f)/Kn uses Q with the mass fix Q^_0 = 0
 *     (Sec. 2.3), i.e. Q minus its mean over the velocity grid, per cell;
 *   - the modified Newton operator (eq. (modified_Newton)) is
 *     A g = T[g] - P L P g / Kn with L about each cell's local Maxwellian
 *     (its discrete density, velocity and temperature) and P the invariant
 *     projection of lincoll_project, so every Krylov vector keeps zero mass;
 *   - every Newton iterate, and the initial guess of eq. (initial), is
 *     rescaled to the discrete mass C.
 * Norms: sqrt(dx h_v^3 sum r^2) (Appendix B).
 * Arrays f, r, g, out: device double [nx][n][n][n] (cell-major; the plan's
 * velocity layout inside a cell).  The plan supplies n, L, the collision
 * kernel, the hemisphere rule of quadcoll_apply (residual, FP64 always) and
 * the apply dtype of the Newton operator; these calls replace its Maxwellians
 * with the local ones of f and use its stream.  Work memory is allocated per
 * call and freed before return; every call synchronises the plan's stream. */
/* Learned correction of the inner solves: a small FP32 network (see the
 * lincoll_mlp_* functions below). */
typedef struct lincoll_mlp_s* lincoll_mlp_t;

typedef struct {
  int nx;                   /* cells, >= 1 (and <= the plan's max_batch if set) */
  double x_l, x_r;          /* slab ends, x_l < x_r (default -0.5, 0.5) */
  double kn;                /* Knudsen number > 0 (default 0.1) */
  double mass;              /* C > 0 (default 1) */
  double theta_l, theta_r;  /* wall temperatures > 0 (default 1, 1.5) */
  double u_l[3], u_r[3];    /* wall velocities (default 0) */
  double tol;               /* Newton stops when the residual norm < tol (default 1e-5) */
  double inner_rtol;        /* inner stop: residual <= inner_rtol * |r| ... (default 1e-3) */
  double inner_atol;        /* ... or <= min(inner_atol, tol / 100) (default 1e-7) (Sec. 5.3) */
  int max_newton;           /* Newton steps, >= 0 (default 30) */
  int max_inner;            /* inner iterations per Newton step, >= 1 (default 2000) */
  int restart;              /* GMRES cycle length, 1..64 (default 30) */
  int init;                 /* 1: start from eq. (initial); 0: from f as passed (default 1) */
  int precond;              /* right preconditioner of the inner GMRES, lincoll_precond_t (default SWEEP) */
  int inner;                /* inner solver, lincoll_inner_t (default GMRES) */
  int backtrack;            /* 1 (default): a Newton step that does not lower the residual is halved, at most
                               three times (f = f_prev - lambda g, lambda = 1/2, 1/4, 1/8); 0: full steps */
  lincoll_mlp_t mlp;        /* network of LINCOLL_PRECOND_LEARNED (else unused; default NULL) */
  float* rec_X;             /* optional device [rec_cap][LINCOLL_MLP_IN]: training features, one row per cell */
  float* rec_T;             /* ... device [rec_cap][LINCOLL_MLP_OUT]: training targets (both NULL: no recording) */
  int rec_cap;              /* rows available in rec_X / rec_T */
} lincoll_steady_params_t;

typedef enum {
  LINCOLL_INNER_GMRES = 0,   /* restarted flexible GMRES with sp->precond */
  LINCOLL_INNER_SOURCE = 1   /* source iteration (Sec. 5.2, eq. (source_iteration)): g <- g + M^-1 (r - A g)
                                from g = 0 with M^-1 the zero-mass sweep, i.e. (T + nu/Kn) g' =
                                (P L P + nu) g / Kn + r; one operator application per iteration */
} lincoll_inner_t;

typedef enum {
  LINCOLL_PRECOND_NONE = 0,  /* plain GMRES */
  LINCOLL_PRECOND_SWEEP = 1, /* one transport sweep z = (T + diag(nu)/Kn)^-1 y: the upwind recurrence of the
                                source iteration (Sec. 5.2) with nu(v) the loss collision frequency of each
                                cell's L; left wall ghost from z, right ghost empty; then the total of z is
                                removed along the current iterate, so corrections keep zero mass */
  LINCOLL_PRECOND_LEARNED = 2 /* SWEEP inside GMRES, and each inner solve starts from a z + alpha Delta with
                                 z = sweep(r), Delta the correction of mlp(features(z)) and (a, alpha)
                                 minimising the start's residual (two extra operator applications, counted
                                 as inner iterations): a nonlinear preconditioner applied to the residual */
} lincoll_precond_t;

typedef struct {
  int newton_iters;         /* Newton steps taken (= binary-operator evaluations - 1) */
  int inner_iters;          /* linearized-operator evaluations, all steps */
  int converged;            /* 1 if the residual fell below tol */
  double residual;          /* final residual norm */
  double mass;              /* final discrete mass */
  double res_history[65];   /* residual norm before step k, k = 0..min(newton_iters, 64) */
  int inner_history[64];    /* inner iterations of step k */
  double ms_total, ms_residual, ms_inner;   /* wall clock: whole solve, residuals, inner solves */
  int rec_rows;             /* training rows written to rec_X / rec_T */
  int backtracks;           /* step halvings taken (each costs one residual evaluation) */
} lincoll_steady_report_t;

/* Fills *sp with the defaults above for nx cells. */
void lincoll_steady_default(lincoll_steady_params_t* sp, int nx);

/* r = T[f] - (Q(f,f) - mean Q)/Kn per cell (eq. (discrete_eq) as a
 * residual); *norm (host, may be NULL) = its norm.  r may be NULL to get the
 * norm only.  f and r must not overlap.  Synchronous. */
int lincoll_steady_residual(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f, double* r,
                            double* norm);

/* out = T[g] - P L P g / Kn with L about the local Maxwellians of f (the
 * modified Newton operator, eq. (modified_Newton)); the plan's Maxwellians
 * are set to those of f.  g and out must not overlap.  Synchronous. */
int lincoll_steady_newton_apply(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                                const double* g, double* out);

/* z = M^-1 y, the inner solver's preconditioner sp->precond (NONE: z = y;
 * SWEEP and LEARNED: the zero-mass transport sweep) about the local
 * Maxwellians of f; the plan's Maxwellians are set to those of f.  y and z
 * must not overlap.  Synchronous. */
int lincoll_steady_precondition(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                                const double* y, double* z);

/* Modified Newton iteration (Sec. 5.2): f <- f - g with A g = r(f) solved by
 * restarted flexible GMRES from g = 0 (right preconditioner sp->precond,
 * classical Gram-Schmidt, FP64 vectors, the plan's apply dtype inside A) to
 * the inner tolerances; stops at the
 * residual tolerance or after max_newton steps.  f is overwritten with the
 * last iterate; rep (host, may be NULL) receives the history.  Returns
 * LINCOLL_OK also when not converged (see rep->converged). */
int lincoll_steady_solve(lincoll_plan_t plan, const lincoll_steady_params_t* sp, double* f,
                         lincoll_steady_report_t* rep);

/* With rec_X / rec_T set, every Newton step appends nx training rows after
 * its inner solve: features of z = sweep(r) and targets m(g - z)/s, g the
 * step's correction (solve the inner systems tightly for clean targets).
 * Rows beyond rec_cap are not written. */

/* ---- Learned correction of the inner solves ----------------------------
 * Per cell c with local Maxwellian (rho, u, theta) the Hermite functions
 *   psi_0 = 1, psi_d = (v_d - u_d)/sqrt(theta), psi_4 = (|v-u|^2/theta - 3)/sqrt 6
 * (orthonormal under M/rho) give moments m_a(c) = h^3 sum z psi_a / rho.
 * Features, 26 per cell, with s = sqrt(mean m^2) (1 if 0), ms = m/s and
 * x_c = (c+1/2)/nx: ms (5), (sum_{c'<=c} ms - ms/2)/nx (5),
 * (sum_{c'>=c} ms - ms/2)/nx (5), sum_{c'<=c} ms x_c'/nx (5),
 * sum_{c'>=c} ms x_c'/nx (5), x_c.  The network Y = tanh(X W1 + b1) W2 + b2
 * (26 -> 128 -> 5, FP32) predicts m(g - z)/s, and the correction is
 * Delta_c = sum_a s Y_a(c) M_c psi_a.  Weights: one packed float array
 * W1 [26][128], b1 [128], W2 [128][5], b2 [5] (row-major). */
#define LINCOLL_MLP_IN 26
#define LINCOLL_MLP_HIDDEN 128
#define LINCOLL_MLP_OUT 5
#define LINCOLL_MLP_WEIGHTS (26 * 128 + 128 + 128 * 5 + 5)

/* Creates a network on the current device with Glorot-uniform weights from
 * a seeded generator (splitmix64) and zero biases.  Synchronous. */
int lincoll_mlp_create(unsigned long long seed, lincoll_mlp_t* out);
void lincoll_mlp_destroy(lincoll_mlp_t mlp);
int lincoll_mlp_set_stream(lincoll_mlp_t mlp, void* hip_stream);
/* Copies the packed weights to (write = 0) or from (write = 1) the host array
 * w of count = LINCOLL_MLP_WEIGHTS floats; writing resets the optimiser.
 * Synchronous. */
int lincoll_mlp_weights(lincoll_mlp_t mlp, float* w, long long count, int write);
/* Y [rows][5] = network(X [rows][26]); device float arrays.  Asynchronous. */
int lincoll_mlp_forward(lincoll_mlp_t mlp, const float* X, float* Y, int rows);
/* loss = mean((Y - T)^2) over all rows x 5 entries (host, may be NULL) and
 * its gradient with respect to the packed weights into grad (device
 * [LINCOLL_MLP_WEIGHTS], may be NULL).  Synchronous. */
int lincoll_mlp_loss_grad(lincoll_mlp_t mlp, const float* X, const float* T, int rows, float* grad, double* loss);
/* steps full-batch Adam steps (beta 0.9, 0.999, eps 1e-8, step size lr) on
 * the loss above; *loss (may be NULL) = the loss before the last step.
 * Synchronous. */
int lincoll_mlp_train(lincoll_mlp_t mlp, const float* X, const float* T, int rows, int steps, double lr,
                      double* loss);
/* X [nx][26] (device float) and *s (host) = features of the field z about
 * the local Maxwellians of f (both device double [nx][n][n][n]).  Synchronous. */
int lincoll_learned_features(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                             const double* z, float* X, double* s);
/* out = Delta: sum_a s Y_a(c) M_c psi_a about the local Maxwellians of f
 * (Y device float [nx][5], out device double).  Synchronous. */
int lincoll_learned_correction(lincoll_plan_t plan, const lincoll_steady_params_t* sp, const double* f,
                               const float* Y, double s, double* out);

/* Releases everything the plan owns (waits for its stream first). */
void lincoll_destroy(lincoll_plan_t plan);

/* Static string for a status code. */
const char* lincoll_strerror(int status);

/* Testing hook for the out-of-memory paths (not a paper operation): with
 * after = k > 0, the k-th device allocation the library attempts from now
 * on fails as if hipMalloc returned out-of-memory (the k - 1 before it
 * proceed); after <= 0 switches injection off.  A call that fails this way
 * returns LINCOLL_ENOMEM and leaves the plan usable: its capacities are
 * reset, so the next call allocates again, and a plan whose Maxwellian cache
 * was lost reports LINCOLL_ENOTREADY until lincoll_set_maxwellians succeeds.
 * Process-wide, not thread-safe. */
void lincoll_debug_fail_alloc(int after);

#define LINCOLL_TABLE_G 0      /* g_j, [J] */
#define LINCOLL_TABLE_W 1      /* W_j = w_j^g B(g_j), [J] */
#define LINCOLL_TABLE_PHI 2    /* Phi_j(q) = 4 pi^2 W_j sinc(pi g_j sqrt(q)/(2L)), [J][3(n/2)^2+1], q = |k|^2 */
#define LINCOLL_TABLE_OMEGA 3  /* Omega(q) = 16 pi^2 sum_j W_j sinc(pi g_j sqrt(q)/L), [3(n/2)^2+1] */
#define LINCOLL_TABLE_PHIJ 4   /* phi_j(|d1|,|d2|,|d3|) = iDFT[sigma_j], octant [J][n/2+1]^3 */
/* Host-only (no device is touched): writes `count` doubles of one
 * precomputed table for the parameters *p into out.  Returns the table's
 * element count, or a negative status (count too small, bad parameters). */
long long lincoll_plan_tables(const lincoll_params_t* p, int table, double* out, long long count);

#ifdef __cplusplus
}
#endif
#endif /* LINCOLL_H */
