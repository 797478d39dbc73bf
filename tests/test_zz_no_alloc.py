"""lincoll_apply_noalloc (the entry point that allocates nothing) through the
C ABI against lincoll_apply on the same plan: bitwise equal outputs on two
calls in a row, the second with a smaller input; no allocation attempted
(an injected allocation failure stays unused, the plan's and torch's device
memory unchanged); unsupported configurations rejected."""
import ctypes
import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
from test_gpu_parity import mixed_inputs  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


@pytest.mark.parametrize("n,big,small,dtype", [(32, 300, 37, "f32"), (16, 1500, 5, "f32"), (32, 250, 37, "f64"),
                                               (16, 1700, 5, "f64")])
def test_noalloc_matches_apply_twice(n, big, small, dtype):
    """The F64 cases exceed the array's 192 (n = 32) and 1536 (n = 16) F64
    slots, so the persistent workgroups loop over several cells each."""
    L, om = 8.0, 0.74
    lib = lc.library()
    h, params = mixed_inputs(n, L, big, seed=2900 + n)
    # F64 at n = 32 takes the fused path under AUTO only from 128 cells on
    plan = lc.Plan(n, L, om, dtype, path="fused" if (dtype, n) == ("f64", 32) else "auto")
    plan.set_option("fused_split", 1)   # lincoll_apply_noalloc runs one workgroup per cell
    assert plan.info("path") == 2
    td = torch.float32 if dtype == "f32" else torch.float64
    for B in (big, small):
        print(f"noalloc n={n} dtype={dtype} batch={B}", flush=True)
        plan.set_maxwellians(dev(params[:B], torch.float64))
        x = dev(h[:B], td)
        ref = plan.apply(x)
        out = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        # tensors of earlier tests freed by the cycle collector would change
        # torch's count in between: collect first, and not during the call
        gc.collect()
        gc.disable()
        try:
            held = plan.info("device_bytes")
            torch_held = torch.cuda.memory_allocated(DEV)
            lib.lincoll_debug_fail_alloc(1)     # any library allocation now fails
            try:
                st = lib.lincoll_apply_noalloc(plan._h, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), B)
            finally:
                lib.lincoll_debug_fail_alloc(0)
            assert st == lc.OK, lc.library().lincoll_strerror(st)
            torch.cuda.synchronize()
            assert plan.info("device_bytes") == held
            assert torch.cuda.memory_allocated(DEV) == torch_held
        finally:
            gc.enable()
        assert torch.equal(out, ref), float((out - ref).abs().max())


def test_noalloc_rejects_unsupported_plans():
    lib = lc.library()
    n, L, om = 16, 8.0, 0.74
    x = torch.zeros((2, n, n, n), dtype=torch.float32, device=DEV)
    y = torch.zeros_like(x)
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    for kw in (dict(path="staged"), dict(project=1)):
        plan = lc.Plan(n, L, om, "f32", **kw)
        assert lib.lincoll_apply_noalloc(plan._h, px, py, 2) == lc.EINVAL
    p64 = lc.Plan(n, L, om, "f64", path="staged")                     # not on the fused path
    assert lib.lincoll_apply_noalloc(p64._h, px, py, 2) == lc.EINVAL
    p32 = lc.Plan(32, L, om, "f32")                                    # AUTO without splitting: two cells
    p32.set_option("fused_split", 1)                                   # take the staged path
    p32.set_maxwellians(torch.tensor([[1, 0, 0, 0, 1.0]] * 2, dtype=torch.float64, device=DEV))
    a32 = torch.zeros((2, 32, 32, 32), dtype=torch.float32, device=DEV)
    b32 = torch.zeros_like(a32)
    assert p32.info("path") == 1
    assert lib.lincoll_apply_noalloc(p32._h, ctypes.c_void_p(a32.data_ptr()), ctypes.c_void_p(b32.data_ptr()), 2) \
        == lc.EINVAL
    pbf = lc.Plan(32, L, om, "bf16x3")                                 # staged only
    x32 = torch.zeros((2, 32, 32, 32), dtype=torch.float32, device=DEV)
    y32 = torch.zeros_like(x32)
    assert lib.lincoll_apply_noalloc(pbf._h, ctypes.c_void_p(x32.data_ptr()), ctypes.c_void_p(y32.data_ptr()), 2) \
        == lc.EINVAL
    plan = lc.Plan(n, L, om, "f32")
    assert lib.lincoll_apply_noalloc(plan._h, px, px, 2) == lc.EINVAL       # aliased
    assert lib.lincoll_apply_noalloc(plan._h, px, py, 0) == lc.EINVAL       # empty
    plan.set_maxwellians(torch.tensor([[1, 0, 0, 0, 1.0]] * 3, dtype=torch.float64, device=DEV))
    assert lib.lincoll_apply_noalloc(plan._h, px, py, 2) == lc.ENOTREADY


@pytest.mark.parametrize("n,big,small,dtype", [(32, 3, 1, "f32"), (32, 2, 1, "f64"), (16, 40, 5, "f64")])
def test_noalloc_splits_small_batches_like_apply(n, big, small, dtype):
    """Batches the plan splits over several workgroups per cell run split in
    the array too (slots and partial sums fit): bitwise equal to
    lincoll_apply, no allocation, on two calls in a row, the second
    smaller."""
    L, om = 8.0, 0.74
    lib = lc.library()
    h, params = mixed_inputs(n, L, big, seed=3600 + n)
    plan = lc.Plan(n, L, om, dtype)
    td = torch.float32 if dtype == "f32" else torch.float64
    for B in (big, small):
        print(f"noalloc split n={n} dtype={dtype} batch={B}", flush=True)
        plan.set_maxwellians(dev(params[:B], torch.float64))
        x = dev(h[:B], td)
        ref = plan.apply(x)
        split = plan.info("fused_split")
        assert split > 1
        out = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        try:
            held = plan.info("device_bytes")
            torch_held = torch.cuda.memory_allocated(DEV)
            lib.lincoll_debug_fail_alloc(1)
            try:
                st = lib.lincoll_apply_noalloc(plan._h, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), B)
            finally:
                lib.lincoll_debug_fail_alloc(0)
            assert st == lc.OK, lc.library().lincoll_strerror(st)
            torch.cuda.synchronize()
            assert plan.info("device_bytes") == held
            assert torch.cuda.memory_allocated(DEV) == torch_held
        finally:
            gc.enable()
        assert plan.info("fused_split") == split
        assert torch.equal(out, ref), float((out - ref).abs().max())


def test_noalloc_split_that_does_not_fit_runs_unsplit():
    """64 cells at n = 32 split 3 ways with the loss item need 256 slots and
    their partial sums, more than the array holds: one workgroup per cell,
    agreeing with the split lincoll_apply to rounding."""
    n, L, om, B = 32, 8.0, 0.74, 64
    h, params = mixed_inputs(n, L, B, seed=3700)
    plan = lc.Plan(n, L, om, "f32")
    plan.set_maxwellians(dev(params, torch.float64))
    x = dev(h, torch.float32)
    ref = plan.apply(x)
    assert plan.info("fused_split") > 1
    out = torch.full_like(x, float("nan"))
    plan.apply_noalloc(x, out)
    torch.cuda.synchronize()
    assert plan.info("fused_split") == 1
    d = (out.double() - ref.double()).reshape(B, -1).abs().amax(dim=1)
    r = ref.double().reshape(B, -1).abs().amax(dim=1)
    assert float((d / r).max()) <= 5e-6
