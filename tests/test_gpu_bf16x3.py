"""BF16x3 variant (matrix-core forward DFT stages of the gain loop, n = 32
and 64) against the FP64 oracle and against the FP64 path on the same GPU.

Bar: a bfloat16 hi + lo pair carries 16 significant bits, so each split
operand is represented to within 2^-17 relative; the three-product form
drops a further term of relative size 2^-16.  With two GEMM stages per
transform this bounds the stage error by about 4 * 2^-16 = 6e-5 relative
to the plane's magnitude; the apply is checked at 5e-5 per cell (relative
l2), while the FP32 bar (1e-5) is not expected to hold for this dtype."""
import numpy as np
import pytest

from oracle import alg1, fast_direct as fd
from paper_2503_09580_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
from test_gpu_parity import mixed_inputs  # noqa: E402
from parity_util import check_batch, check_cells  # noqa: E402

DEV = torch.device("cuda:0")
BAR = 5e-5


def run(dtype, h, params, n=32, L=8.0, om=0.74):
    plan = lc.Plan(n, L, om, dtype)
    plan.set_maxwellians(torch.from_numpy(np.ascontiguousarray(params)).to(DEV, torch.float64))
    td = torch.float64 if dtype == "f64" else torch.float32
    out = plan.apply(torch.from_numpy(np.ascontiguousarray(h)).to(DEV, td))
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def test_bf16x3_c2_against_oracle():
    h, params = wl.c2()
    hin = h.astype(np.float32).astype(np.float64)
    got = run("bf16x3", hin, params)
    sample = [0, 13, 40, 63]
    ref = alg1.apply_batch(fd.make_plan(32, 8.0, 0.74), hin[sample], np.repeat(params, len(sample), 0))
    check_cells(got, ref, BAR, cells=sample)


def test_bf16x3_per_cell_maxwellians_ragged_batch():
    h, params = mixed_inputs(32, 8.0, 37, seed=1200)
    hin = h.astype(np.float32).astype(np.float64)
    got = run("bf16x3", hin, params)
    sample = [0, 17, 36]
    ref = alg1.apply_batch(fd.make_plan(32, 8.0, 0.74), hin[sample], params[sample])
    check_cells(got, ref, BAR, cells=sample)


def test_bf16x3_full_c3_batch_against_gpu_fp64():
    h, params = wl.c3()
    hin = h.astype(np.float32).astype(np.float64)
    got = run("bf16x3", hin, params)
    ref = run("f64", hin, params)
    check_batch(got, ref, BAR)


def test_bf16x3_n64_c5_cells_against_oracle():
    """n = 64 (box [-10, 10)^3): the four-wave matrix-core plane transform."""
    cells = [0, 300, 511]
    h, params = wl.c5(cells=cells)
    hin = h.astype(np.float32).astype(np.float64)
    got = run("bf16x3", hin, params, n=64, L=10.0)
    ref = alg1.apply_batch(fd.make_plan(64, 10.0, 0.74), hin, params)
    check_cells(got, ref, BAR)


def test_bf16x3_n64_full_c5_batch_against_gpu_fp64():
    h, params = wl.c5()
    hin = h.astype(np.float32).astype(np.float64)
    got = run("bf16x3", hin, params, n=64, L=10.0)
    ref = run("f64", hin, params, n=64, L=10.0)
    check_batch(got, ref, BAR)


def test_bf16x3_n64_ragged_batch():
    """A batch whose plane count (7 cells x 33 planes) is not a multiple of
    the grid, with per-cell Maxwellians."""
    h, params = mixed_inputs(64, 10.0, 7, seed=1310)
    hin = h.astype(np.float32).astype(np.float64)
    got = run("bf16x3", hin, params, n=64, L=10.0)
    ref = run("f64", hin, params, n=64, L=10.0)
    check_cells(got, ref, BAR)


def test_bf16x3_supported_at_n32_and_n64_only():
    import ctypes
    for n in (8, 16):
        p = lc.make_params(n, 8.0, 0.74, "bf16x3")
        h = ctypes.c_void_p()
        assert lc.library().lincoll_plan_ex(ctypes.byref(p), ctypes.byref(h)) == lc.EINVAL
    for n, L in ((32, 8.0), (64, 10.0)):
        plan = lc.Plan(n, L, 0.74, "bf16x3")
        assert plan.info("path") == 1        # staged path (the fused kernel has no BF16x3 stage)
