"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs, element by element.

Bars (tests/parity_util.py): per cell, both the relative l2 error and the
largest element-wise error relative to max |ref| stay below 1e-12 for FP64
and 1e-5 for FP32 against the FP64 oracle (the tolerances the specification
states).  Sizes span several tiles and ragged batch counts; full-size
configurations are checked on sampled cells the oracle computes one by one,
and the FP32 headline configuration on every cell against the GPU FP64 path
(itself checked against the oracle)."""
import math

import numpy as np
import pytest

from oracle import alg1, fast_direct as fd, projection
from paper_2503_09580_amd import workloads as wl
from parity_util import check, check_batch, check_cells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
DEV = torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def run(plan, h, params, dtype):
    td = torch.float64 if dtype == "f64" else torch.float32
    ht = torch.from_numpy(np.ascontiguousarray(h)).to(DEV, td)
    pt = torch.from_numpy(np.ascontiguousarray(params)).to(DEV, torch.float64)
    plan.set_maxwellians(pt)
    out = plan.apply(ht)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def oracle_cells(n, L, omega, h, params, **kw):
    p = fd.make_plan(n, L, omega, **kw)
    return alg1.apply_batch(p, h, params)


def mixed_inputs(n, L, batch, seed, per_cell=True, degree=4):
    rng = np.random.default_rng(seed)
    keep = np.array([a + b + c <= degree for a, b, c in wl.MONOMIALS])
    params = np.empty((batch if per_cell else 1, 5))
    for b in range(params.shape[0]):
        params[b] = [rng.uniform(0.7, 1.3), *rng.uniform(-0.3, 0.3, 3), rng.uniform(0.7, 1.4)]
    h = np.empty((batch, n, n, n))
    for b in range(batch):
        q = params[b if per_cell else 0]
        h[b] = wl.maxwellian(n, L, q[0], q[1:4], q[4]) * wl.poly_eval(n, L, wl.poly_coeffs(rng) * keep, q[1:4],
                                                                     math.sqrt(q[4]))
    return h, params


@pytest.mark.parametrize("n,L,omega,batch", [(8, 4.0, 1.0, 3), (16, 8.0, 0.5, 5), (16, 8.0, 0.74, 7),
                                             (32, 8.0, 0.74, 3)])
def test_fp64_staged_matches_oracle(n, L, omega, batch):
    h, params = mixed_inputs(n, L, batch, seed=1000 + n)
    plan = lc.Plan(n, L, omega, "f64", path="staged")
    got = run(plan, h, params, "f64")
    ref = oracle_cells(n, L, omega, h, params)
    check_cells(got, ref, 1e-12, tag="f64 staged")


@pytest.mark.parametrize("n,L,omega,batch", [(16, 8.0, 0.74, 7), (32, 8.0, 0.74, 5), (16, 8.0, 1.0, 300)])
def test_fp64_fused_matches_oracle_and_staged(n, L, omega, batch):
    """The fused kernel on an F64 plan (double after the product with M^h as
    well) against the oracle, and against the staged FP64 path on every cell;
    the 300-cell case runs several cells per persistent workgroup."""
    h, params = mixed_inputs(n, L, batch, seed=1100 + n + batch)
    plan = lc.Plan(n, L, omega, "f64", path="fused")
    assert plan.info("path") == 2
    got = run(plan, h, params, "f64")
    sample = [0, batch // 2, batch - 1] if batch > 10 else list(range(batch))
    ref = oracle_cells(n, L, omega, h[sample], params[sample])
    check_cells(got, ref, 1e-12, cells=sample, tag="f64 fused vs oracle")
    staged = run(lc.Plan(n, L, omega, "f64", path="staged"), h, params, "f64")
    check_batch(got, staged, 1e-12, tag="f64 fused vs staged")


def test_fp64_matches_direct_sum_oracle():
    """Against O1 (dense DFT + naive convolution) as well, n = 16."""
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 2, seed=7)
    plan = lc.Plan(n, L, om, "f64", path="staged")
    got = run(plan, h, params, "f64")
    p = fd.make_plan(n, L, om)
    for b in range(2):
        ref = fd.apply(p, h[b], params[b, 0], params[b, 1:4], params[b, 4])
        check(got[b], ref, 1e-12, tag=b)


def test_c1_hard_spheres_and_invariant_inputs():
    """Configuration C1 (n=16, L=8, hard spheres, unit Maxwellian) plus the
    collision-invariant inputs M, v M, |v|^2 M.  L of an invariant is a
    cancellation of two O(1) terms down to the discretisation error, so its
    error is measured against the loss term ||L-[h]|| (reading R13)."""
    cfg = wl.CONFIGS["C1"]
    n, L, om = cfg["n"], cfg["L"], cfg["omega"]
    h, params = wl.c1()
    inv = wl.invariant_inputs(n, L)
    hh = np.concatenate([h, inv])
    plan = lc.Plan(n, L, om, "f64")
    got = run(plan, hh, params, "f64")
    ref = oracle_cells(n, L, om, hh, params)
    check(got[0], ref[0], 1e-12)
    p = fd.make_plan(n, L, om)
    for b in range(1, hh.shape[0]):
        _, _, Lm = fd.apply(p, hh[b], 1.0, (0, 0, 0), 1.0, parts=True)
        check(got[b], ref[b], 1e-12, scale=Lm, tag=b)
        assert np.linalg.norm(ref[b]) < 0.1 * np.linalg.norm(Lm)    # it is near zero


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_fp64_cutoff_variants(eps):
    """Without the cutoff r = h/M spans the whole box; a quadratic p keeps
    its range moderate so that the FFT round-off (relative to max |r|, the
    issue of Sec. 3.3) stays below the 1e-12 bar on both sides."""
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 2, seed=55, degree=2)
    plan = lc.Plan(n, L, om, "f64", eps=eps)
    got = run(plan, h, params, "f64")
    ref = oracle_cells(n, L, om, h, params, eps=eps)
    check_cells(got, ref, 1e-12, tag=eps)


def test_quadrature_rule_1():
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 2, seed=56)
    plan = lc.Plan(n, L, om, "f64", quad_rule=1)
    got = run(plan, h, params, "f64")
    ref = oracle_cells(n, L, om, h, params, rule=1)
    check_cells(got, ref, 1e-12)


def test_c2_fp64_and_fp32_sampled():
    """Configuration C2 (n=32, omega=0.74, bi-Maxwellian perturbations, one
    Maxwellian broadcast), full batch of 64 on the GPU, 6 sampled cells in
    the oracle; FP64 <= 1e-12, FP32 <= 1e-5."""
    cfg = wl.CONFIGS["C2"]
    n, L, om = cfg["n"], cfg["L"], cfg["omega"]
    h, params = wl.c2()
    sample = [0, 1, 17, 31, 48, 63]
    ref = oracle_cells(n, L, om, h[sample], params)
    for dt, tol in [("f64", 1e-12), ("f32", 1e-5)]:
        plan = lc.Plan(n, L, om, dt)
        hin = h if dt == "f64" else h.astype(np.float32).astype(np.float64)
        got = run(plan, hin, params, dt)
        refd = ref if dt == "f64" else oracle_cells(n, L, om, hin[sample], params)
        check_cells(got, refd, tol, cells=sample, tag=dt)


@pytest.mark.parametrize("dt,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_c3_full_batch_sampled(dt, tol):
    """Configuration C3 at its full size (4096 cells, each its own
    Maxwellian), sampled cells checked against the oracle one by one."""
    cfg = wl.CONFIGS["C3"]
    n, L, om, B = cfg["n"], cfg["L"], cfg["omega"], cfg["batch"]
    h, params = wl.c3(batch=B)
    plan = lc.Plan(n, L, om, dt)
    got = run(plan, h, params, dt)
    sample = [0, 1, 777, 2048, 4094, 4095]
    hin = h[sample] if dt == "f64" else h[sample].astype(np.float32).astype(np.float64)
    ref = oracle_cells(n, L, om, hin, params[sample])
    check_cells(got, ref, tol, cells=sample, tag=dt)


def test_batched_equals_single_cell_and_broadcast():
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 9, seed=77)
    plan = lc.Plan(n, L, om, "f64")
    full = run(plan, h, params, "f64")
    for b in (0, 4, 8):
        one = run(plan, h[b:b + 1], params[b:b + 1], "f64")
        assert np.array_equal(one[0], full[b])
    # one Maxwellian broadcast to all cells equals the same Maxwellian repeated
    rep = np.repeat(params[:1], 9, axis=0)
    a = run(plan, h, params[:1], "f64")
    b = run(plan, h, rep, "f64")
    assert np.array_equal(a, b)


def test_repeat_is_bitwise_deterministic():
    n, L, om = 32, 8.0, 0.74
    h, params = mixed_inputs(n, L, 4, seed=78)
    for dt in ("f64", "f32"):
        plan = lc.Plan(n, L, om, dt)
        a = run(plan, h, params, dt)
        b = run(plan, h, params, dt)
        assert np.array_equal(a, b)


def test_projection_kernel_and_exact_conservation():
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 3, seed=79)
    plan = lc.Plan(n, L, om, "f64")
    pt = torch.from_numpy(params).to(DEV)
    plan.set_maxwellians(pt)
    x = torch.from_numpy(h).to(DEV)
    y = plan.project(x).cpu().numpy()
    phis = projection.invariants(n, L)
    for b in range(3):
        M = fd.maxwellian_fields(fd.make_plan(n, L, om), params[b, 0], params[b, 1:4], params[b, 4])[0]
        ref = projection.project(h[b], M, phis)
        check(y[b], ref, 1e-12, tag=b)
    # with the projection flag, L_cons = P L P conserves and annihilates exactly
    pplan = lc.Plan(n, L, om, "f64", project=1)
    got = run(pplan, h, params, "f64")
    for b in range(3):
        m = projection.moments(got[b], phis)
        assert np.max(np.abs(m)) <= 1e-12 * np.max(np.abs(got[b])) * n ** 3
    inv = np.stack([wl.invariant_inputs(n, L, params[0, 0], params[0, 1:4], params[0, 4])[a] for a in range(5)])
    got = run(pplan, inv, params[:1], "f64")
    assert np.max(np.abs(got)) <= 1e-12 * np.max(np.abs(inv))


def test_ragged_and_single_cell_batches():
    n, L, om = 16, 8.0, 0.74
    for B in (1, 2, 33):
        h, params = mixed_inputs(n, L, B, seed=90 + B)
        for dt, tol in [("f64", 1e-12), ("f32", 1e-5)]:
            plan = lc.Plan(n, L, om, dt)
            hin = h if dt == "f64" else h.astype(np.float32).astype(np.float64)
            got = run(plan, hin, params, dt)
            for b in sorted({0, B // 2, B - 1}):
                ref = oracle_cells(n, L, om, hin[b:b + 1], params[b:b + 1])[0]
                check(got[b], ref, tol, tag=(B, dt, b))


def test_abi_errors_on_device():
    n, L, om = 8, 4.0, 1.0
    plan = lc.Plan(n, L, om, "f64")
    x = torch.zeros((2, n, n, n), dtype=torch.float64, device=DEV)
    lib = lc.library()
    import ctypes
    p = ctypes.c_void_p(x.data_ptr())
    assert lib.lincoll_apply(plan._h, p, p, 2) == lc.EINVAL            # aliased
    q = ctypes.c_void_p(x.data_ptr() + 8 * n ** 3)
    assert lib.lincoll_apply(plan._h, p, q, 2) == lc.EINVAL            # overlapping
    params = torch.tensor([[1, 0, 0, 0, 1.0]] * 3, dtype=torch.float64, device=DEV)
    plan.set_maxwellians(params)
    y = torch.zeros_like(x)
    assert lib.lincoll_apply(plan._h, p, ctypes.c_void_p(y.data_ptr()), 2) == lc.ENOTREADY
    assert lib.quadcoll_apply(plan._h, p, ctypes.c_void_p(y.data_ptr()), 2) == lc.OK   # binary operator, FP64
    assert plan.info("J") == n // 2 + 1
    assert plan.info("maxw_batch") == 3


@pytest.mark.parametrize("dtype,n,path", [("f32", 32, "fused"), ("f64", 16, "fused"), ("f32", 16, "staged")])
def test_nonfinite_debug_check(dtype, n, path):
    """LINCOLL_OPT_CHECK_FINITE: a NaN in one cell's input makes that cell's
    output non-finite and the apply report LINCOLL_ENONFINITE (the output is
    still written); finite input passes; without the option the same NaN
    input returns OK.  Eager and graph replay."""
    L, om, B = 8.0, 0.74, 20
    h, params = mixed_inputs(n, L, B, seed=2700 + n)
    td = torch.float32 if dtype == "f32" else torch.float64
    for graph in (0, 1):
        plan = lc.Plan(n, L, om, dtype, path=path)
        plan.set_option("graph", graph)
        plan.set_maxwellians(dev(params, torch.float64))
        x = dev(h, td)
        out = torch.empty_like(x)
        plan.set_option("check_finite", 1)
        plan.apply(x, out)                                  # finite: OK
        assert bool(torch.isfinite(out).all())
        bad = x.clone()
        bad[7, 3, 4, 5] = float("nan")
        with pytest.raises(lc.LincollError) as err:
            plan.apply(bad, out)
        assert err.value.status == lc.ENONFINITE
        assert not bool(torch.isfinite(out[7]).all())
        assert bool(torch.isfinite(out[6]).all())           # other cells unaffected
        plan.set_option("check_finite", 0)
        plan.apply(bad, out)                                # no check: OK
        torch.cuda.synchronize()
        plan.close()


def test_empty_and_oversized_batches_are_rejected():
    """An empty batch is an argument error (LINCOLL_EINVAL) for apply,
    project and quadcoll, through the C ABI with valid pointers and through
    the binding with a zero-length tensor; so is a batch above the plan's
    max_batch.  The output is left untouched."""
    import ctypes
    n, L, om = 8, 4.0, 1.0
    lib = lc.library()
    plan = lc.Plan(n, L, om, "f64", max_batch=2)
    plan.set_maxwellians(torch.tensor([[1, 0, 0, 0, 1.0]], dtype=torch.float64, device=DEV))
    x = torch.ones((3, n, n, n), dtype=torch.float64, device=DEV)
    y = torch.full_like(x, 7.0)
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    for fn in (lib.lincoll_apply, lib.lincoll_project, lib.quadcoll_apply):
        assert fn(plan._h, px, py, 0) == lc.EINVAL
        assert fn(plan._h, px, py, -1) == lc.EINVAL
    assert lib.lincoll_apply(plan._h, px, py, 3) == lc.EINVAL        # above max_batch
    assert lib.lincoll_apply(plan._h, px, py, 2) == lc.OK
    torch.cuda.synchronize()
    assert torch.all(y[2] == 7.0)
    with pytest.raises(lc.LincollError) as err:
        plan.apply(torch.empty((0, n, n, n), dtype=torch.float64, device=DEV))
    assert err.value.status == lc.EINVAL


@pytest.mark.parametrize("n,L", [(16, 8.0), (32, 8.0)])
def test_fp32_fused_and_staged_match_oracle(n, L):
    """Both FP32 paths (the fused per-cell kernel and the staged kernels)
    against the oracle, per-cell Maxwellians, ragged batch of 37."""
    om = 0.74
    h, params = mixed_inputs(n, L, 37, seed=500 + n)
    hin = h.astype(np.float32).astype(np.float64)
    sample = [0, 5, 18, 36]
    ref = oracle_cells(n, L, om, hin[sample], params[sample])
    for path in ("fused", "staged"):
        plan = lc.Plan(n, L, om, "f32", path=path)
        assert plan.info("path") == (2 if path == "fused" else 1)
        got = run(plan, hin, params, "f32")
        check_cells(got, ref, 1e-5, cells=sample, tag=path)


def test_c3_fp32_fused_every_cell():
    """Configuration C3 at full size through the fused FP32 kernel: every one
    of the 4096 cells against the GPU FP64 path on the same (float-rounded)
    input, and 64 cells spread over the batch against the oracle."""
    cfg = wl.CONFIGS["C3"]
    n, L, om, B = cfg["n"], cfg["L"], cfg["omega"], cfg["batch"]
    h, params = wl.c3(batch=B)
    hin = h.astype(np.float32).astype(np.float64)
    del h
    plan = lc.Plan(n, L, om, "f32", path="fused")
    got = run(plan, hin, params, "f32")
    plan.close()
    sample = list(range(0, B, B // 64))[:64]
    ref = oracle_cells(n, L, om, hin[sample], params[sample])
    l2o, mxo = check_cells(got, ref, 1e-5, cells=sample, tag="oracle")
    ref64 = lc.Plan(n, L, om, "f64", path="staged")
    full = run(ref64, hin, params, "f64")
    ref64.close()
    # the GPU FP64 result is itself the oracle's on the sampled cells
    check_cells(full, ref[::8], 1e-12, cells=sample[::8], tag="f64 vs oracle")
    l2, mx = check_batch(got, full, 1e-5, tag="f32 vs gpu f64")
    print(f"C3 FP32, 4096 cells vs GPU FP64: worst l2 {l2:.3e}, worst element-wise {mx:.3e}; "
          f"64 cells vs oracle: {l2o:.3e}, {mxo:.3e}")


@pytest.mark.parametrize("n,path", [(16, "fused"), (32, "fused"), (32, "staged")])
def test_fp32_without_cutoff(n, path):
    """FP32 with eps = 0 (no cutoff: r = h/M over the whole box).  A
    quadratic p keeps r moderate, as for the FP64 variant.  The library runs
    with subnormal floats flushed to zero, so the float input is flushed the
    same way before it reaches the oracle."""
    L, om = 8.0, 0.74
    h, params = mixed_inputs(n, L, 5, seed=2300 + n, degree=2)
    h32 = h.astype(np.float32)
    h32[np.abs(h32) < np.finfo(np.float32).tiny] = 0.0
    hin = h32.astype(np.float64)
    plan = lc.Plan(n, L, om, "f32", path=path, eps=0.0)
    got = run(plan, hin, params, "f32")
    ref = oracle_cells(n, L, om, hin, params, eps=0.0)
    check_cells(got, ref, 1e-5, tag=(n, path))


@pytest.mark.parametrize("n,J,dtype,path", [(8, 2, "f32", "staged"), (16, 3, "f32", "fused"), (32, 4, "f32", "fused"),
                                            (32, 4, "f32", "staged"), (16, 3, "f64", "staged"), (16, 3, "f64", "fused"),
                                            (32, 4, "f64", "fused")])
def test_small_quadrature_counts(n, J, dtype, path):
    """Few g-nodes (J P^3 < n^3 with P = n/2 + 1): the per-cell setup scratch
    must still hold the FP64 loss frequency of n^3 values per cell.  Per-cell
    Maxwellians over several setup cells, against the oracle with the same J."""
    L, om = 8.0, 0.74
    h, params = mixed_inputs(n, L, 6, seed=2400 + n + J)
    hin = h if dtype == "f64" else h.astype(np.float32).astype(np.float64)
    plan = lc.Plan(n, L, om, dtype, J=J, path=path)
    assert plan.info("J") == J
    got = run(plan, hin, params, dtype)
    ref = oracle_cells(n, L, om, hin, params, J=J)
    check_cells(got, ref, 1e-12 if dtype == "f64" else 1e-5, tag=(n, J, path))
