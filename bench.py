"""Benchmark: batched applications of the linearized VHS collision operator
L[h] = Q(M,h) + Q(h,M) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64|bf16x3]
                    [--path auto|staged|fused] [--config C3|C2|C1] [--no-cpu]

A step is one call of lincoll_apply over the whole batch of the workload
(configuration C3 by default: n = 32 points per velocity axis, box [-8,8)^3,
VHS omega = 0.74, 4096 cells along a 1-D grid, each with its own local
Maxwellian), with the inputs and the per-cell Maxwellian setup resident in
HBM before timing starts.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks.  Packed FP32 instructions are kept out of these
# kernels, so plain FP32 and FP64 vector FMAs both issue at
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s.
PEAK_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def alg_flops_per_cell(n, J):
    """Algorithmic work of one cell-apply: (2J + 4) real 3-D transforms at
    2.5 N log2 N (N = n^3), 4J n^3 for the mode products and ~60 n^3 for the
    Maxwellians, the cutoff division and the loss combination."""
    N3 = n ** 3
    return (2 * J + 4) * 2.5 * N3 * math.log2(N3) + 4 * J * N3 + 60 * N3


def alg_bytes_per_cell(n, elem):
    """Compulsory HBM traffic of one cell-apply: h in, L out, 5 parameters."""
    return 2 * n ** 3 * elem + 40


# Sources whose compiled code is the fused kernel; a counter record is only
# used while their hash matches.
KERNEL_SOURCES = {
    "fused": ["paper_2503_09580_amd/csrc/fused.hip", "paper_2503_09580_amd/csrc/fused_body.inc",
              "paper_2503_09580_amd/csrc/fft.h",
              "paper_2503_09580_amd/csrc/twiddles.h", "paper_2503_09580_amd/csrc/internal.h"],
}
def fused_kernel_name(n, ppt, keep, dtype, split=1):
    """Name of the fused kernel instance a plan launches (as in the profiles);
    a split apply is three launches."""
    tl = "double" if dtype == "f64" else "float"
    if ppt == 2:
        return f"k_fused2<{n}>"
    if split > 1:
        return f"k_fused_split<{n}, {keep}, {tl}> + k_fused_sum + k_fused_finish<{n}, {tl}>"
    return f"k_fused<{n}, {keep}, {tl}>"


def kernel_source_hash(path):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(path, []):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(kernel, cfg, dtype, path):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a device copy of known size), or None when no record exists
    or the kernel sources changed since the counters were taken."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    want = kernel_source_hash(path)
    for name in sorted(os.listdir(d)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(d, name)) as fh:
            for line in fh:
                m = re.match(r"^traffic-record: (\{.*\})\s*$", line)
                if not m:
                    continue
                r = json.loads(m.group(1))
                if (r.get("kernel") == kernel and r.get("config") == cfg and r.get("dtype") == dtype
                        and r.get("source_sha256") == want):
                    return r
    return None


def copy_calibration(torch, dev, stream, mib):
    """A plain device-to-device copy of known size, so that counter runs see a
    reference kernel whose true HBM traffic is mib MiB read + mib MiB written."""
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        for _ in range(3):
            dst.copy_(src)
    stream.synchronize()
    del src, dst


def workload(cfg):
    from paper_2503_09580_amd import workloads as wl
    if cfg == "C3":
        h, p = wl.c3()
    elif cfg == "C2":
        h, p = wl.c2()
    elif cfg == "C1":
        h, p = wl.c1()
    elif cfg == "C5":
        h, p = wl.c5()
    else:
        raise SystemExit(f"unknown config {cfg}")
    c = wl.CONFIGS[cfg]
    return h, p, c


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


_POOL = {}    # inputs shared with forked workers (copy-on-write)


def _pool_init():
    from oracle import fast_direct
    c = _POOL["c"]
    _POOL["plan"] = fast_direct.make_plan(c["n"], c["L"], c["omega"])


def _oracle_cells(rng):
    """Worker of the all-core baseline: the oracle on cells [b0, b1)."""
    from oracle import alg1
    b0, b1 = rng
    h, params = _POOL["h"], _POOL["params"]
    p = params[b0:b1] if params.shape[0] > 1 else params
    alg1.apply_batch(_POOL["plan"], h[b0:b1], p)
    return b1 - b0


def cpu_baseline(cfg, h, params, c, budget_s=8.0):
    """The oracle (Algorithm 1 with numpy's FFT, FP64) on a bounded sample of
    the same cells, timed on this host: one thread, then one process per
    core (at most 16, the CPU share of one GPU) each on its own cells, the
    same oracle code in every process.  Runs before the GPU is touched."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp

    from oracle import alg1, fast_direct
    plan = fast_direct.make_plan(c["n"], c["L"], c["omega"])
    alg1.apply_batch(plan, h[:1], params[:1])          # warm
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < budget_s and done < h.shape[0]:
        b = done
        alg1.apply_batch(plan, h[b:b + 1], params[b:b + 1] if params.shape[0] > 1 else params)
        done += 1
    dt = time.perf_counter() - t0
    single = done / dt
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    workers = max(1, min(16, cores))
    per = max(1, min(h.shape[0] // workers, int(single * budget_s)))
    _POOL.update(h=h, params=params, c=c)
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork"), initializer=_pool_init) as ex:
        list(ex.map(_oracle_cells, [(w, w + 1) for w in range(workers)]))     # every worker up, plan built
        t0 = time.perf_counter()
        cells = sum(ex.map(_oracle_cells, [(w * per, (w + 1) * per) for w in range(workers)]))
        wall = time.perf_counter() - t0
    _POOL.clear()
    return {"value": cells / wall, "unit": "applies/s", "cores": workers, "kind": "oracle",
            "single_thread_value": single,
            "cpu_model": cpu_model(), "host_cores_visible": cores,
            "sample": f"{cfg}: {done} cells on one thread ({dt:.1f} s), then {cells} cells in {workers} processes "
                      f"of {per} cells each ({wall:.1f} s wall), FP64 Algorithm 1 with numpy's FFT"}


def quadcoll_flops_per_cell(n, J, M):
    """(2 J M + J + 4) complex 3-D transforms at 5 N log2 N (N = n^3) plus
    ~10 n^3 per hemisphere point and node for phases and products."""
    N3 = n ** 3
    return (2 * J * M + J + 4) * 5.0 * N3 * math.log2(N3) + 10.0 * J * M * N3


def bench_quadcoll(a, torch, lincoll, dev):
    """Q(f, f) (eq. (14), 64-point hemisphere rule, FP64) over 256 cells at
    n = 32 (the cell count of the steady-state workload): f = local
    Maxwellian + perturbation of the C3 generator's first 256 cells."""
    from paper_2503_09580_amd import workloads as wl
    B = 256
    h, params = wl.c3(batch=4096, cells=np.arange(B))
    n, L, om = 32, 8.0, 0.74
    f = h + np.stack([wl.maxwellian(n, L, q[0], q[1:4], q[4]) for q in params])
    ft = torch.from_numpy(f).to(dev, torch.float64)
    out = torch.empty_like(ft)
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        plan = lincoll.Plan(n, L, om, "f64")
        J = int(plan.info("J"))
        for _ in range(max(1, a.warmup)):
            plan.quadcoll(ft, out)
        stream.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = min(a.steps, 5)
        ev0.record(stream)
        for _ in range(steps):
            plan.quadcoll(ft, out)
        ev1.record(stream)
        ev1.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    M = 64
    fl = quadcoll_flops_per_cell(n, J, M) * B
    ach = fl / (ms / 1e3) / 1e12
    rec = {"metric": "Q(f,f) applies/sec at N=32 (FP64, 64 hemisphere points)", "value": B / (ms / 1e3),
           "unit": "applies/s", "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{B} cells, n={n}, box [-{L:g},{L:g})^3, VHS omega={om}, J={J}, "
                                  f"hemisphere 4 polar x 16 azimuths", "cells": B, "n": n},
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_VALU_TFLOPS, "traffic": None,
                        "kernel": "quadcoll_apply (all launches of one step)"}}
    if not a.no_cpu:
        from oracle import binary, fast_direct, quadrature
        plan = fast_direct.make_plan(n, L, om)
        sph = quadrature.hemisphere_product_rule(8, 16)
        t0 = time.perf_counter()
        binary.q_binary(plan, sph, f[0], f[0], method="fast")
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": 1.0 / dt, "unit": "applies/s", "cores": 1, "kind": "oracle",
                               "sample": f"cell 0, binary-method oracle with library FFT, FP64, {dt:.1f} s"}
    print(json.dumps(rec))


def bench_rk4(a, torch, lincoll, dev):
    """The paper's timed workload (Table 5): 100 RK4 steps (dt = 0.1) of
    df/dt = L[f], n = 32 (N = 16), R = 6, L = (3 + sqrt 2) R / 4, one
    homogeneous cell about the standard Maxwellian, cutoff 1e-9; FP64 unless
    --dtype says otherwise.  --case 1: Maxwell molecules (omega = 1) from the
    mass-1 f^(1); --case 2: B2 = g^0.56/(4 pi) (omega = 0.72) from f^(2).
    After the timed 100 steps another 100 run untimed, and the line reports
    the L2 distance to M at t = 10 and t = 20 next to Table 4's printed value
    (t = 20) and the mass drift."""
    from paper_2503_09580_amd import workloads as wl
    n, R = 32, 6.0
    L = (3.0 + math.sqrt(2.0)) * R / 4.0
    dtype = a.dtype if a.dtype in ("f64", "f32") else "f64"
    td = torch.float64 if dtype == "f64" else torch.float32
    case = a.case
    omega = 1.0 if case == 1 else 0.72
    f0 = (wl.paper_f1(n, L, unit_mass=True) if case == 1 else wl.paper_f2(n, L))[None]
    stream = torch.cuda.Stream(device=dev)
    steps = 100
    with torch.cuda.stream(stream):
        plan = lincoll.Plan(n, L, omega, dtype, R=R)
        plan.set_option("graph", 1)
        f = torch.from_numpy(f0).to(dev, td)
        plan.rk4(f, 0.1, max(1, a.warmup))
        stream.synchronize()
        f = torch.from_numpy(f0).to(dev, td)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        plan.rk4(f, 0.1, steps)
        ev1.record(stream)
        ev1.synchronize()
        path = "fused" if plan.info("last_path") == 2 else "staged"   # the path the timed applies took
        f10 = f.double().cpu().numpy()[0]
        plan.rk4(f, 0.1, steps)
        stream.synchronize()
        f20 = f.double().cpu().numpy()[0]
    ms = ev0.elapsed_time(ev1)
    h3 = (2.0 * L / n) ** 3
    M = wl.maxwellian(n, L, 1.0, (0, 0, 0), 1.0)
    m0 = h3 * f0.sum()
    table4 = {"dist_t10": math.sqrt(h3 * np.sum((f10 - M) ** 2)), "dist_t20": math.sqrt(h3 * np.sum((f20 - M) ** 2)),
              "paper_t20": 3.09e-5 if case == 1 else 4.25e-4,
              "mass_drift_t10": abs(h3 * f10.sum() - m0) / m0, "mass_drift_t20": abs(h3 * f20.sum() - m0) / m0}
    J = n // 2 + 1
    paper_s = 2.81          # Table 5, linearized operator, double, 100 steps, one CPU thread (both cases)
    value = steps / (ms / 1e3)
    fl = 4 * alg_flops_per_cell(n, J) * steps
    ach = fl / (ms / 1e3) / 1e12
    rec = {"metric": f"RK4 steps/sec of df/dt = L[f] (Table 5, Case {case})", "value": value, "unit": "steps/s",
           "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": ms / steps, "higher_is_better": True,
           "scaling": "strong", "vs_baseline": value / (100.0 / paper_s),
           "vs_baseline_note": "paper: 100 steps in 2.81 s on one Intel i7-13800H thread, FP64 (other hardware)",
           "dtype": dtype, "data": f"synthetic (closed-form f^({case}))",
           "config": {"workload": f"1 cell, n={n}, R={R:g}, L={L:.4f}, omega={omega:g}, "
                                  f"f^({case}), dt=0.1, 100 steps", "path": path, "graph": 1},
           "table4": table4,
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_VALU_TFLOPS, "traffic": None,
                        "kernel": "lincoll_rk4 (one recorded graph per step)",
                        "note": "one cell cannot fill 256 CUs: latency-bound by construction"}}
    if not a.no_cpu:
        from oracle import fast_direct, timestep
        plan = fast_direct.make_plan(n, L, omega, R=R)
        p = np.array([[1.0, 0, 0, 0, 1.0]])
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 10.0 and k < 20:
            timestep.rk4(plan, f0, p, 0.1, 1)
            k += 1
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": k / dt, "unit": "steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{k} RK4 steps of the same problem by the oracle (Algorithm 1, FP64)"}
    print(json.dumps(rec))


def bench_steady(a, torch, lincoll, dev):
    """Newton solve wall-time of the steady 1-D heat-transfer problem (Sec. 5.3.2,
    Fourier flow; scheme of Appendix B): 256 cells on [-0.5, 0.5], walls at
    temperature 1 and 1.5, Kn = 0.1, mass 1, n = 32, box [-8,8)^3,
    VHS omega = 0.74; residuals by quadcoll_apply (FP64), Newton operator with
    applies in --dtype (default f32) inside sweep-preconditioned flexible
    GMRES; Newton tolerance 1e-5, inner 1e-3 relative / 1e-7 absolute.  A step
    is one whole solve from the initial guess of eq. (initial)."""
    from paper_2503_09580_amd import workloads as wl
    c = wl.CONFIGS["C4"]
    n, L, om, nx = c["n"], c["L"], c["omega"], c["nx"]
    dtype = a.dtype or "f32"
    precond = a.precond
    sp = lincoll.steady_params(nx, kn=c["kn"], theta_l=c["theta_l"], theta_r=c["theta_r"], mass=c["mass"],
                               precond=precond, inner=a.inner)
    stream = torch.cuda.Stream(device=dev)
    steps = max(1, min(a.steps, 5))
    extra = {}
    with torch.cuda.stream(stream):
        plan = lincoll.Plan(n, L, om, dtype)
        graph = 1 if a.graph is None else a.graph     # each GMRES cycle replays one recorded graph
        plan.set_option("graph", graph)
        f = torch.empty((nx, n, n, n), dtype=torch.float64, device=dev)
        if precond == "learned":
            # training data from plain solves at wall temperatures spread over [1.1, 2.0],
            # away from the timed case (1.5)
            t0 = time.perf_counter()
            thetas = np.array([1.1, 1.3, 1.7, 2.0])
            rows = len(thetas) * 8 * nx
            RX = torch.zeros((rows, 26), dtype=torch.float32, device=dev)
            RT = torch.zeros((rows, 5), dtype=torch.float32, device=dev)
            used = 0
            for th in thetas:
                rsp = lincoll.steady_params(nx, kn=c["kn"], theta_l=c["theta_l"], theta_r=float(th), mass=c["mass"],
                                            inner_rtol=1e-8, inner_atol=0.0, rec_X=RX[used:], rec_T=RT[used:])
                used += plan.steady_solve(rsp, f)["rec_rows"]
            net = lincoll.MLP(seed=7)
            loss = net.train(RX[:used].contiguous(), RT[:used].contiguous(), steps=3000, lr=2e-3)
            stream.synchronize()
            sp = lincoll.steady_params(nx, kn=c["kn"], theta_l=c["theta_l"], theta_r=c["theta_r"], mass=c["mass"],
                                       precond="learned", mlp=net)
            extra = {"train_rows": used, "train_loss": loss, "train_thetas": [round(float(t), 4) for t in thetas],
                     "train_s": time.perf_counter() - t0}
            # the same solver without the network (sweep preconditioner, same dtype), timed alike:
            # what the learned start gains or loses by itself
            sps = lincoll.steady_params(nx, kn=c["kn"], theta_l=c["theta_l"], theta_r=c["theta_r"], mass=c["mass"])
            plan.steady_solve(sps, f)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                reps_s = plan.steady_solve(sps, f)
            stream.synchronize()
            extra["sweep_same_dtype_s"] = (time.perf_counter() - t0) / steps
            extra["sweep_same_dtype_inner_iters"] = reps_s["inner_iters"]
            extra["sweep_same_dtype_residual"] = reps_s["residual"]
            # the plain FP64 solver (sweep preconditioner) on the same problem, timed alike
            plan64 = lincoll.Plan(n, L, om, "f64")
            plan64.set_option("graph", graph)
            sp64 = lincoll.steady_params(nx, kn=c["kn"], theta_l=c["theta_l"], theta_r=c["theta_r"], mass=c["mass"])
            plan64.steady_solve(sp64, f)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                rep64 = plan64.steady_solve(sp64, f)
            stream.synchronize()
            extra["plain_f64_s"] = (time.perf_counter() - t0) / steps
            extra["plain_f64_inner_iters"] = rep64["inner_iters"]
            extra["plain_f64_residual"] = rep64["residual"]
        for _ in range(max(1, a.warmup)):
            plan.steady_solve(sp, f)
        stream.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(steps):
            reps.append(plan.steady_solve(sp, f))
        stream.synchronize()
        wall = (time.perf_counter() - t0) / steps
        J = int(plan.info("J"))
    rep = reps[-1]
    evals = rep["newton_iters"] + 1
    M = 64
    q_ms = sum(r["ms_residual"] for r in reps) / steps
    ach = quadcoll_flops_per_cell(n, J, M) * nx * evals / (q_ms / 1e3) / 1e12
    rec = {"metric": "Newton solve wall-time (steady 1-D heat transfer, Table 8 case theta_R=1.5, Kn=0.1)",
           "value": wall, "unit": "s", "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": wall * 1e3,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (closed-form initial guess)",
           "config": {"workload": f"{nx} cells x n={n}^3 velocities, box [-{L:g},{L:g})^3, omega={om}, Kn={c['kn']}, "
                                  f"walls theta 1/1.5, tol 1e-5", "precond": precond, "inner": a.inner,
                      "graph": graph,
                      "newton_iters": rep["newton_iters"], "inner_iters": rep["inner_iters"],
                      "residual": rep["residual"], "res_history": rep["res_history"],
                      "ms_residual": rep["ms_residual"], "ms_inner": rep["ms_inner"], "ms_total": rep["ms_total"],
                      "converged": rep["converged"], **extra},
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_VALU_TFLOPS, "traffic": None,
                        "kernel": "quadcoll_apply inside the residuals (the dominant part of a solve)"}}
    if not a.no_cpu:
        from oracle import alg1, binary, fast_direct, quadrature
        fh = f[:1].cpu().numpy()
        oplan = fast_direct.make_plan(n, L, om)
        sph = quadrature.hemisphere_product_rule(8, 16)
        t0 = time.perf_counter()
        binary.q_binary(oplan, sph, fh[0], fh[0], fix=1)
        tq = time.perf_counter() - t0
        p = np.array([[1.0, 0.0, 0.0, 0.0, 1.2]])
        t0 = time.perf_counter()
        alg1.apply_batch(oplan, fh, p)
        tl = time.perf_counter() - t0
        est = evals * nx * tq + rep["inner_iters"] * nx * tl
        rec["cpu_baseline"] = {"value": est, "unit": "s", "cores": alg1.threads_used(), "kind": "oracle",
                               "sample": f"one cell's binary Q ({tq:.2f} s) and one linearized apply ({tl:.2f} s) "
                                         f"by the oracle, scaled by the solve's {evals} x {nx} residual cells and "
                                         f"{rep['inner_iters']} x {nx} operator cells"}
    print(json.dumps(rec))


# Table 7: Couette-flow solve times (total, s) on an 11th-gen Intel Core i7
# with 8 threads; 200 cells, n = 32, Maxwell molecules, FP64.
PAPER_TABLE7 = {0.1: {0.1: 174.8, 1.0: 127.1, 10.0: 121.6}, 0.2: {0.1: 242.3, 1.0: 134.0, 10.0: 124.7},
                0.3: {0.1: 254.9, 1.0: 136.5, 10.0: 134.9}, 0.4: {0.1: 254.9, 1.0: 180.9, 10.0: 136.7},
                0.5: {0.1: 256.5, 1.0: 199.6, 10.0: 153.1}}


def bench_couette(a, torch, lincoll, dev):
    """The paper's Couette flow (Sec. 5.3.1; walls at -+u_W, theta = 1): 200
    cells on [-0.5, 0.5], n = 32, Maxwell molecules, R = 3.5 and
    L = (3 + sqrt 2) R / 4, mass 1, Newton tolerance 1e-5, inner 1e-3 / 1e-7.
    A step is one whole solve from the initial guess of eq. (initial)."""
    kn, uw = a.kn, a.uw
    nx, n, R = 200, 32, 3.5
    L = (3.0 + math.sqrt(2.0)) * R / 4.0
    dtype = a.dtype or "f32"
    sp = lincoll.steady_params(nx, kn=kn, theta_l=1.0, theta_r=1.0, u_l=(0.0, -uw, 0.0), u_r=(0.0, uw, 0.0))
    stream = torch.cuda.Stream(device=dev)
    steps = max(1, min(a.steps, 5))
    with torch.cuda.stream(stream):
        plan = lincoll.Plan(n, L, 1.0, dtype, R=R)
        f = torch.empty((nx, n, n, n), dtype=torch.float64, device=dev)
        for _ in range(max(1, a.warmup)):
            plan.steady_solve(sp, f)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rep = plan.steady_solve(sp, f)
        stream.synchronize()
        wall = (time.perf_counter() - t0) / steps
        J = int(plan.info("J"))
    paper = PAPER_TABLE7.get(round(uw, 1), {}).get(kn)
    ach = quadcoll_flops_per_cell(n, J, 64) * nx * (rep["newton_iters"] + 1) / (rep["ms_residual"] / 1e3) / 1e12
    rec = {"metric": "Newton solve wall-time (Couette flow, Table 7 workload)", "value": wall, "unit": "s",
           "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": wall * 1e3, "higher_is_better": False,
           "scaling": "strong", "vs_baseline": wall / paper if paper else None,
           "vs_baseline_note": "value / the paper's Table 7 total on an 8-thread Intel Core i7, FP64 (other hardware)"
           if paper else None,
           "dtype": dtype, "data": "synthetic (closed-form initial guess)",
           "config": {"workload": f"Couette u_W={uw}, Kn={kn}: {nx} cells x n={n}^3, R={R}, L={L:.4f}, Maxwell molecules",
                      "newton_iters": rep["newton_iters"], "inner_iters": rep["inner_iters"],
                      "residual": rep["residual"], "converged": rep["converged"], "paper_s": paper,
                      "ms_residual": rep["ms_residual"], "ms_inner": rep["ms_inner"]},
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_VALU_TFLOPS, "traffic": None,
                        "kernel": "quadcoll_apply inside the residuals (the dominant part of a solve)"}}
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default=None, help="f32 (default for apply), f64 (default for rk4), bf16x3")
    ap.add_argument("--path", default="auto")
    ap.add_argument("--config", default="C3")
    ap.add_argument("--case", type=int, default=1, choices=[1, 2], help="rk4: Sec. 4.2 case")
    ap.add_argument("--inner", default="gmres", choices=["gmres", "source"], help="steady: inner solver")
    ap.add_argument("--kn", type=float, default=1.0, help="couette: Knudsen number")
    ap.add_argument("--uw", type=float, default=0.5, help="couette: wall speed")
    ap.add_argument("--precond", default="sweep", choices=["sweep", "none", "learned"],
                    help="steady: inner preconditioner (learned: trains the network first, untimed)")
    ap.add_argument("--op", default="apply", choices=["apply", "quadcoll", "rk4", "steady", "couette"],
                    help="apply: batched L[h] (default); quadcoll: binary Q(f,f); rk4: Table 5 time stepping; "
                         "steady: Newton solve of the 256-cell heat-transfer problem; couette: the paper's "
                         "Table 7 workload (--kn, --uw)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-configuration tuner (lincoll_autotune) before timing")
    ap.add_argument("--graph", type=int, default=None, help="force graph replay off (0) or on (1)")
    ap.add_argument("--fused-ppt", type=int, default=None, choices=[1, 2],
                    help="fused path: force one or two pencils per thread (skips the tuner)")
    ap.add_argument("--fused-keep", type=int, default=None, choices=[0, 4, 8, 16],
                    help="fused path: force the accumulator chunks kept in registers (skips the tuner)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run a device copy of this many MiB first (reference kernel for counter runs)")
    a = ap.parse_args()
    if a.dtype is None:
        a.dtype = "f64" if a.op == "rk4" else "f32"
    if a.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; per-cell work has no cross-GPU traffic, "
                                   "so N GPUs would each run this workload on their own share of cells",
                          "n_gpus": a.gpus}))
        sys.exit(2)

    cpu = None
    if a.op == "apply" and not a.no_cpu:
        h0, p0, c0 = workload(a.config)
        cpu = cpu_baseline(a.config, h0, p0, c0)    # before anything touches the GPU (the pool forks)
        del h0, p0

    import torch
    from paper_2503_09580_amd import lincoll

    dev = torch.device("cuda:0")
    if a.op == "quadcoll":
        return bench_quadcoll(a, torch, lincoll, dev)
    if a.op == "rk4":
        return bench_rk4(a, torch, lincoll, dev)
    if a.op == "steady":
        return bench_steady(a, torch, lincoll, dev)
    if a.op == "couette":
        return bench_couette(a, torch, lincoll, dev)
    h, params, c = workload(a.config)
    n, L, om, B = c["n"], c["L"], c["omega"], h.shape[0]
    td = torch.float64 if a.dtype == "f64" else torch.float32
    elem = 8 if a.dtype == "f64" else 4
    ht = torch.from_numpy(h).to(dev, td)
    pt = torch.from_numpy(params).to(dev, torch.float64)
    out = torch.empty_like(ht)
    stream = torch.cuda.Stream(device=dev)
    if a.copy_calib_mib > 0:
        copy_calibration(torch, dev, stream, a.copy_calib_mib)
    with torch.cuda.stream(stream):
        plan = lincoll.Plan(n, L, om, a.dtype, path=a.path)
        plan.set_maxwellians(pt)
        # per-cell setup (Maxwellian factors, cutoff mask, K_j, nu, Gram
        # inverse) of all B cells, timed on a second call (buffers exist)
        es0, es1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        es0.record(stream)
        plan.set_maxwellians(pt)
        es1.record(stream)
        es1.synchronize()
        setup_ms = es0.elapsed_time(es1)
        J = int(plan.info("J"))
        tuned_ms = None
        if a.fused_ppt is not None:
            plan.set_option("fused_ppt", a.fused_ppt)
            a.no_tune = True
        if a.fused_keep is not None:
            plan.set_option("fused_keep", a.fused_keep)
            a.no_tune = True
        if not a.no_tune and a.path == "auto":
            tuned_ms = plan.autotune(ht, out, reps=3)   # untimed; picks path, workgroups/CU, graph replay
        if a.graph is not None:
            plan.set_option("graph", a.graph)
        plan.apply(ht, out)   # one untimed apply, so that the plan reports the path this batch takes
        stream.synchronize()
        path = "fused" if plan.info("last_path") == 2 else "staged"
        launch = {"path": path, "graph": int(plan.info("graph")), "tuned_ms": tuned_ms,
                  "fused_per_cu": int(plan.info("fused_per_cu")) if path == "fused" else None,
                  "fused_pencils_per_thread": int(plan.info("fused_ppt")) if path == "fused" else None,
                  "fused_accumulator_chunks_in_registers": int(plan.info("fused_keep"))
                  if path == "fused" and plan.info("fused_ppt") == 1 else None,
                  "fused_workgroups_per_cell": int(plan.info("fused_split")) if path == "fused" else None,
                  "staged_zblock": int(plan.info("zblock")) if path == "staged" else None,
                  "staged_plane_tile": int(plan.info("plane_tile")) if path == "staged" else None,
                  "tuner": "lincoll_autotune over path x workgroups/CU x fused pencils per thread x fused "
                           "accumulator split x fused workgroups per cell x staged tiles x graph"}
        for _ in range(a.warmup):
            plan.apply(ht, out)
        stream.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(a.steps):
            plan.apply(ht, out)
        ev1.record(stream)
        ev1.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / a.steps
    value = B * a.steps / (gpu_ms / 1e3)

    rec = {
        "metric": f"L[h] applies/sec at N={n} ({a.dtype.upper()})",
        "value": value,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "wall_s_timed": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32+f64", "bf16x3": "bf16x3"}.get(a.dtype, a.dtype),
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {B} cells, n={n}, box [-{L:g},{L:g})^3, VHS omega={om}, "
                               f"J={J}, eps=1e-9, per-cell Maxwellians"
                               + (", theta log-uniform in [0.5, 2]" if a.config == "C5" else "")
                               if a.config in ("C3", "C5") else
                               f"{a.config}: {B} cells, n={n}, box [-{L:g},{L:g})^3, VHS omega={om}, J={J}",
                   "cells": B, "n": n, "path": path, "launch": launch},
        "setup": {"ms": setup_ms, "cells_per_s": B / (setup_ms / 1e3),
                  "what": "lincoll_set_maxwellians for all cells (FP64 per-cell setup), untimed in value"},
    }
    # Roofline of the dominant kernel.  On the fused path a step is exactly one
    # launch of the fused kernel on `stream` (three for a split apply: the
    # parts, their sum, the inverse), so the event-timed step is that kernel's
    # average launch duration; the staged path is reported as a whole.
    fl = alg_flops_per_cell(n, J) * B
    by = alg_bytes_per_cell(n, elem) * B
    achieved = fl / (ms_per_step / 1e3) / 1e12
    split = int(plan.info("fused_split")) if path == "fused" else 1
    kname = (fused_kernel_name(n, int(plan.info("fused_ppt")), int(plan.info("fused_keep")), a.dtype, split)
             if path == "fused" else "lincoll_apply (all launches of one step)")
    tr = traffic_record(kname, a.config, a.dtype, path) if path == "fused" else None
    rec["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_VALU_TFLOPS,
                       "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None,
                       "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                       "kernel": kname, "launches_per_step": (3 if split > 1 else 1) if path == "fused" else None,
                       "alg_flops_per_launch": fl, "alg_bytes_per_launch": by,
                       "hbm_GBs_compulsory": by / (ms_per_step / 1e3) / 1e9}
    if tr:
        rec["roofline"]["traffic_GBs"] = (tr["fetch_bytes"] + tr["write_bytes"]) / (ms_per_step / 1e3) / 1e9
        rec["roofline"]["traffic_source"] = tr["summary"]
    if not a.no_check:
        # accuracy of this result against the FP64 path on the same GPU and
        # the same (rounded) inputs
        with torch.cuda.stream(stream):
            ref_plan = lincoll.Plan(n, L, om, "f64", path="staged")
            ref_plan.set_maxwellians(pt)
            h64 = ht.double()
            ref = ref_plan.apply(h64)
            stream.synchronize()
        def errs(x):
            dd = (x.double() - ref).reshape(B, -1)
            r2 = ref.reshape(B, -1)
            l2 = dd.norm(dim=1) / r2.norm(dim=1)
            mx = dd.abs().amax(dim=1) / r2.abs().amax(dim=1)
            return {"max": float(l2.max()), "median": float(l2.median()), "elementwise_max": float(mx.max())}

        rec["rel_err_vs_fp64"] = errs(out)
        # the paper's precision and the matrix-core variant on the same cells,
        # timed the same way (event-bracketed applies after one warm-up)
        others = {}
        if a.config in ("C3", "C5"):
            def timed(p, x, y, reps=5):
                p.apply(x, y)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    p.apply(x, y)
                e1.record(stream)
                e1.synchronize()
                return e0.elapsed_time(e1) / reps

            with torch.cuda.stream(stream):
                # the paper's precision on the path an F64 plan takes by default
                # (the fused kernel at n <= 32), and on the staged kernels
                p64 = lincoll.Plan(n, L, om, "f64")
                p64.set_maxwellians(pt)
                o64 = torch.empty_like(h64)
                ms64 = timed(p64, h64, o64)
                path64 = "fused" if p64.info("last_path") == 2 else "staged"
                ms64s = timed(ref_plan, h64, torch.empty_like(h64)) if path64 == "fused" else ms64
                d64 = errs(o64)
                others["f64"] = {"ms_per_step": ms64, "applies_per_s": B / (ms64 / 1e3), "path": path64,
                                 "staged_ms_per_step": ms64s, "staged_applies_per_s": B / (ms64s / 1e3),
                                 "max_rel_diff_vs_staged": max(d64["max"], d64["elementwise_max"])}
                del p64, o64
                if a.dtype != "bf16x3":
                    bp = lincoll.Plan(n, L, om, "bf16x3")
                    bp.set_maxwellians(pt)
                    hb = ht if ht.dtype == torch.float32 else ht.float()
                    ob = torch.empty_like(hb)
                    msb = timed(bp, hb, ob)
                    stream.synchronize()
                    others["bf16x3"] = {"ms_per_step": msb, "applies_per_s": B / (msb / 1e3), "path": "staged",
                                        "rel_err_vs_fp64": errs(ob)}
                    del bp, hb, ob
            rec["other_dtypes"] = others
        del ref_plan, ref, h64
    if cpu is not None:
        rec["cpu_baseline"] = cpu
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
