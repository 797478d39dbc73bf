"""Launch mechanics of the persistent path: graph replay, workgroups per CU
and the launch-configuration tuner, through the C ABI.

A replayed graph must give exactly the eager result (same kernels, same
order), on every replay, with unrelated eager GPU work and synchronisations
between the replays, and it must be re-recorded when the buffers, the batch
or the plan's allocations change.  Tuned configurations must still meet the
FP32 bar against the oracle."""
import ctypes

import numpy as np
import pytest

from oracle import alg1, fast_direct as fd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
from test_gpu_parity import mixed_inputs  # noqa: E402
from parity_util import check_batch, check_cells  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def eager_result(n, L, om, dtype, path, h, params, **opts):
    td = torch.float64 if dtype == "f64" else torch.float32
    plan = lc.Plan(n, L, om, dtype, path=path)
    for k, v in opts.items():
        plan.set_option(k, v)
    plan.set_maxwellians(dev(params, torch.float64))
    out = plan.apply(dev(h, td))
    torch.cuda.synchronize()
    return out.cpu()


def busy_work():
    """Unrelated eager GPU work between graph replays."""
    a = torch.randn(512, 512, device=DEV)
    b = (a @ a.T).sum()
    other = lc.Plan(8, 4.0, 1.0, "f64")
    x = torch.randn(3, 8, 8, 8, dtype=torch.float64, device=DEV)
    other.apply(x)
    torch.cuda.synchronize()
    return float(b)


@pytest.mark.parametrize("n,dtype,path,batch", [(16, "f64", "staged", 5), (32, "f32", "fused", 9),
                                                (32, "f32", "staged", 4), (16, "f32", "fused", 11),
                                                (32, "bf16x3", "staged", 3), (64, "f32", "staged", 2),
                                                (64, "bf16x3", "staged", 2)])
def test_graph_replay_is_bitwise_eager(n, dtype, path, batch):
    L, om = 8.0, 0.74
    td = torch.float64 if dtype == "f64" else torch.float32
    h, params = mixed_inputs(n, L, batch, seed=700 + n + batch)
    ref = eager_result(n, L, om, dtype, path, h, params)
    plan = lc.Plan(n, L, om, dtype, path=path)
    plan.set_option("graph", 1)
    assert plan.info("graph") == 1
    plan.set_maxwellians(dev(params, torch.float64))
    ht = dev(h, td)
    out = torch.empty_like(ht)
    for rep in range(4):
        out.fill_(float("nan"))
        plan.apply(ht, out)          # first call records, later calls replay
        torch.cuda.synchronize()
        assert torch.equal(out.cpu(), ref), (rep, "replay differs from the eager apply")
        busy_work()
    # a different output buffer is recorded again
    out2 = torch.empty_like(ht)
    plan.apply(ht, out2)
    torch.cuda.synchronize()
    assert torch.equal(out2.cpu(), ref)
    # new Maxwellians of the same batch: same buffers, the replay reads them
    params2 = params.copy()
    params2[:, 4] *= 1.1
    plan.set_maxwellians(dev(params2, torch.float64))
    plan.apply(ht, out2)
    torch.cuda.synchronize()
    assert torch.equal(out2.cpu(), eager_result(n, L, om, dtype, path, h, params2))


def test_last_path_follows_every_entry_point():
    """LINCOLL_INFO_LAST_PATH names the path of the most recent apply, also
    when it was a graph replay (of an apply or of RK4 steps) or the
    no-allocation entry point.  One Maxwellian serves every batch; an AUTO
    FP32 plan at n = 32 takes the staged kernels for 2 cells and the fused
    kernel for 16."""
    n, L, om = 32, 8.0, 0.74
    staged, fused = lc.PATHS["staged"], lc.PATHS["fused"]
    plan = lc.Plan(n, L, om, "f32")
    plan.set_option("fused_split", 1)        # as lincoll_apply_noalloc, so that the two agree bitwise
    assert plan.info("last_path") == 0
    _, params = mixed_inputs(n, L, 1, seed=811)
    plan.set_maxwellians(dev(params, torch.float64))
    small = dev(mixed_inputs(n, L, 2, seed=812)[0], torch.float32)
    big = dev(mixed_inputs(n, L, 16, seed=813)[0], torch.float32)
    plan.apply(small)
    assert plan.info("last_path") == staged
    out = plan.apply(big)
    assert plan.info("last_path") == fused
    plan.set_option("graph", 1)
    plan.apply(big, out)                     # records
    f = small.clone()
    plan.rk4(f, 1e-3, 2)                     # records and replays RK4 steps on 2 cells
    assert plan.info("last_path") == staged
    plan.apply(big, out)                     # replays the recorded apply
    assert plan.info("last_path") == fused
    plan.rk4(f, 1e-3, 1)                     # replays the recorded RK4 step
    assert plan.info("last_path") == staged
    out2 = torch.empty_like(big)
    plan.apply_noalloc(big, out2)
    assert plan.info("last_path") == fused
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), out2.cpu())
    assert torch.isfinite(f).all()
    # the split: a replay reports the split of its own batch
    plan.set_option("fused_split", 0)        # by batch again (drops the recorded graphs)
    plan.apply(big, out)                     # records: 16 cells split
    split16 = plan.info("fused_split")
    assert split16 > 1
    plan.rk4(f, 1e-3, 1)                     # records an RK4 step on 2 cells: split further
    assert plan.info("fused_split") > split16
    plan.apply(big, out)                     # replays the recorded apply
    assert plan.info("fused_split") == split16
    plan.apply_noalloc(big, out2)            # the same split in the fixed array
    assert plan.info("fused_split") == split16
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), out2.cpu())


def test_graph_rerecords_after_reallocation():
    """A larger batch reallocates the plan's buffers; the replay must not use
    the old pointers."""
    n, L, om = 16, 8.0, 0.74
    plan = lc.Plan(n, L, om, "f32", path="staged")
    plan.set_option("graph", 1)
    for batch in (3, 9, 4):
        h, params = mixed_inputs(n, L, batch, seed=800 + batch)
        plan.set_maxwellians(dev(params, torch.float64))
        ht = dev(h, torch.float32)
        out = plan.apply(ht)
        out = plan.apply(ht, out)    # replay
        torch.cuda.synchronize()
        assert torch.equal(out.cpu(), eager_result(n, L, om, "f32", "staged", h, params))


@pytest.mark.parametrize("per_cu", [1, 2, 3, 4])
def test_fused_workgroups_per_cu_do_not_change_results(per_cu):
    n, L, om, batch = 16, 8.0, 0.74, 23
    h, params = mixed_inputs(n, L, batch, seed=900)
    ref = eager_result(n, L, om, "f32", "fused", h, params)
    got = eager_result(n, L, om, "f32", "fused", h, params, fused_per_cu=per_cu)
    assert torch.equal(got, ref)


@pytest.mark.parametrize("n,batch,dtype", [(16, 23, "f32"), (32, 19, "f32"), (16, 23, "f64"), (32, 19, "f64")])
def test_fused_kept_accumulator_is_bitwise_identical(n, batch, dtype):
    """Every split of the L+^ accumulator between registers, LDS and the
    scratch slot (LINCOLL_OPT_FUSED_KEEP) adds the same values in the same
    order.  F32: bitwise equal results.  F64: equal to 1e-14 (each split is
    compiled on its own, and without the rounding to float after the product
    with M^h the compiler may fuse that product into the next addition in one
    instance and not another).  One split is checked against the oracle,
    including the packed plane's partner correction of the K_j product
    (cells with drift, so that plane is not symmetric)."""
    L, om = 8.0, 0.74
    h, params = mixed_inputs(n, L, batch, seed=1300 + n)
    hin = h.astype(np.float32).astype(np.float64) if dtype == "f32" else h
    if dtype == "f32":
        keeps = [0, 4, 8] + ([16] if n == 32 else [])
    else:
        keeps = [0, 8, 16] if n == 16 else [0, 4, 8]
    # one workgroup per cell, so that every accumulator chunk makes its trip
    # across all J nodes (a split batch gives each part only a few)
    outs = [eager_result(n, L, om, dtype, "fused", hin, params, fused_keep=k, fused_split=1) for k in keeps]
    for k, o in zip(keeps[1:], outs[1:]):
        if dtype == "f32":
            assert torch.equal(o, outs[0]), k
        else:
            check_batch(o.numpy(), outs[0].numpy(), 1e-14, tag=("keep", k))
    sample = [0, batch // 2, batch - 1]
    orc = alg1.apply_batch(fd.make_plan(n, L, om), hin[sample], params[sample])
    check_cells(outs[-1].double().numpy(), orc, 1e-5 if dtype == "f32" else 1e-12, cells=sample)


def test_option_errors():
    lib = lc.library()
    plan = lc.Plan(32, 8.0, 0.74, "f32")
    assert lib.lincoll_set_option(plan._h, lc.OPTIONS["fused_per_cu"], 2) == lc.EINVAL   # n = 32 fits one
    assert lib.lincoll_set_option(plan._h, lc.OPTIONS["graph"], 2) == lc.EINVAL
    assert lib.lincoll_set_option(plan._h, 99, 0) == lc.EINVAL
    for bad in (-2, 2, 12, 32):
        assert lib.lincoll_set_option(plan._h, lc.OPTIONS["fused_keep"], bad) == lc.EINVAL
    assert lib.lincoll_set_option(plan._h, lc.OPTIONS["fused_keep"], 16) == lc.OK
    assert plan.info("fused_keep") == 16
    assert lib.lincoll_set_option(plan._h, lc.OPTIONS["fused_keep"], -1) == lc.OK
    p16 = lc.Plan(16, 8.0, 0.74, "f32")
    assert lib.lincoll_set_option(p16._h, lc.OPTIONS["fused_keep"], 16) == lc.EINVAL   # 8 chunks at n = 16
    d32 = lc.Plan(32, 8.0, 0.74, "f64")
    assert d32.info("path") == 2 and d32.info("fused_keep") == 0
    assert lib.lincoll_set_option(d32._h, lc.OPTIONS["fused_keep"], 16) == lc.EINVAL
    assert lib.lincoll_set_option(d32._h, lc.OPTIONS["fused_ppt"], 2) == lc.EINVAL    # two pencils: F32 only
    pbf = lc.Plan(32, 8.0, 0.74, "bf16x3")
    assert lib.lincoll_set_option(pbf._h, lc.OPTIONS["path"], lc.PATHS["fused"]) == lc.EINVAL   # staged only
    x = torch.zeros((2, 32, 32, 32), dtype=torch.float32, device=DEV)
    p = ctypes.c_void_p(x.data_ptr())
    assert lib.lincoll_autotune(plan._h, p, p, 2, 3) == lc.EINVAL                        # aliased
    y = torch.zeros_like(x)
    assert lib.lincoll_autotune(plan._h, p, ctypes.c_void_p(y.data_ptr()), 2, 0) == lc.EINVAL


@pytest.mark.parametrize("n,batch", [(16, 37), (32, 64)])
def test_autotune_picks_a_valid_configuration(n, batch):
    L, om = 8.0, 0.74
    h, params = mixed_inputs(n, L, batch, seed=1000 + n)
    hin = h.astype(np.float32).astype(np.float64)
    plan = lc.Plan(n, L, om, "f32")
    plan.set_maxwellians(dev(params, torch.float64))
    ht = dev(hin, torch.float32)
    ms = plan.autotune(ht, reps=2)
    assert ms > 0 and plan.info("tuned_ms") == ms
    assert plan.info("path") in (1, 2)
    assert 1 <= plan.info("fused_per_cu") <= (4 if n == 16 else 1)
    out = plan.apply(ht)
    out = plan.apply(ht, out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    sample = [0, batch // 2, batch - 1]
    ref = alg1.apply_batch(fd.make_plan(n, L, om), hin[sample], params[sample])
    check_cells(got, ref, 1e-5, cells=sample)


@pytest.mark.parametrize("n,L,dtype", [(16, 8.0, "f32"), (32, 8.0, "f32"), (32, 8.0, "f64"), (64, 10.0, "f32")])
def test_staged_tiles_are_bitwise_identical(n, L, dtype):
    """Every staged tile the tuner searches (z-pass blocks of 64, 128, 256
    threads; 64- or 32-thread in-plane blocks) gives bitwise the same result,
    and that result meets the bar against the oracle (sampled cells)."""
    om = 0.74
    B = 5 if n < 64 else 3
    h, params = mixed_inputs(n, L, B, seed=3000 + n)
    hin = h if dtype == "f64" else h.astype(np.float32).astype(np.float64)
    td = torch.float64 if dtype == "f64" else torch.float32
    ref = None
    for zb in (128, 64, 256):
        for tile in ((0, 1) if n <= 32 else (0,)):
            got = eager_result(n, L, om, dtype, "staged", hin, params, zblock=zb, plane_tile=tile).double().numpy()
            if ref is None:
                ref = got
            else:
                assert np.array_equal(got, ref), (zb, tile)
    sample = [0, B - 1]
    orc = alg1.apply_batch(fd.make_plan(n, L, om), hin[sample], params[sample])
    check_cells(ref, orc, 1e-12 if dtype == "f64" else 1e-5, cells=sample)


def test_autotune_cache_by_key():
    """lincoll_autotune stores its choice under (arch, n, dtype, batch bucket,
    projection, per-cell Maxwellians): a second plan with the same key takes
    it without timing, a different batch bucket or a disabled cache times."""
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 7, seed=3100)
    ht = dev(h, torch.float64)
    keys = ("path", "fused_per_cu", "zblock", "plane_tile", "graph")
    plans = []
    for _ in range(2):
        p = lc.Plan(n, L, om, "f64")
        p.set_maxwellians(dev(params, torch.float64))
        plans.append(p)
    plans[0].set_option("tune_cache", 0)
    plans[0].autotune(ht, reps=1)
    assert plans[0].info("tune_cached") == 0
    plans[1].autotune(ht, reps=1)
    assert plans[1].info("tune_cached") == 1
    assert [plans[0].info(k) for k in keys] == [plans[1].info(k) for k in keys]
    assert plans[1].info("tuned_ms") == plans[0].info("tuned_ms")
    p3 = lc.Plan(n, L, om, "f64")
    p3.set_maxwellians(dev(params[:3], torch.float64))
    p3.autotune(dev(h[:3], torch.float64), reps=1)      # batch bucket 4, not 8
    assert p3.info("tune_cached") == 0


@pytest.mark.parametrize("n,batch", [(16, 21), (32, 37)])
def test_fused_two_pencils_per_thread(n, batch):
    """The fused kernel with two pencils per thread (one wave per SIMD, the
    L+^ accumulator in registers) against the one-pencil kernel on the same
    inputs (the same arithmetic in the same order) and against the oracle."""
    L, om = 8.0, 0.74
    h, params = mixed_inputs(n, L, batch, seed=3200 + n)
    hin = h.astype(np.float32).astype(np.float64)
    one = eager_result(n, L, om, "f32", "fused", hin, params, fused_ppt=1).double().numpy()
    two = eager_result(n, L, om, "f32", "fused", hin, params, fused_ppt=2).double().numpy()
    d = np.max(np.abs(two - one)) / np.max(np.abs(one))
    print(f"n={n}: max |two - one| / max |one| = {d:.3e}")
    assert d <= 1e-6, d
    sample = [0, batch // 2, batch - 1]
    orc = alg1.apply_batch(fd.make_plan(n, L, om), hin[sample], params[sample])
    check_cells(two, orc, 1e-5, cells=sample)
