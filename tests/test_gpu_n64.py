"""n = 64 (configuration C5: box [-10, 10)^3, 512 cells, temperatures
log-uniform in [0.5, 2]) on the staged path against the oracle.  The 64-point
double pencils of the FP64 arithmetic live in registers and accumulation
registers at one wave per SIMD.  Bars as for smaller n: FP64 1e-12, FP32
1e-5 (relative l2 and element-wise relative to max |ref|, per cell)."""
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
from parity_util import check, check_cells  # noqa: E402

DEV = torch.device("cuda:0")
N, L, OM = 64, 10.0, 0.74


def run(dtype, h, params):
    plan = lc.Plan(N, L, OM, dtype)
    assert plan.info("path") == 1
    plan.set_maxwellians(torch.from_numpy(np.ascontiguousarray(params)).to(DEV, torch.float64))
    td = torch.float64 if dtype == "f64" else torch.float32
    out = plan.apply(torch.from_numpy(np.ascontiguousarray(h)).to(DEV, td))
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_c5_cells_against_oracle(dtype, tol):
    cells = [0, 97, 300, 511]
    h, params = wl.c5(cells=cells)
    hin = h if dtype == "f64" else h.astype(np.float32).astype(np.float64)
    got = run(dtype, hin, params)
    ref = alg1.apply_batch(fd.make_plan(N, L, OM), hin, params)
    check_cells(got, ref, tol, tag=dtype)


def test_c5_full_batch_sampled_fp32():
    h, params = wl.c5()
    got = run("f32", h, params)
    sample = [5, 255, 510]
    hin = h[sample].astype(np.float32).astype(np.float64)
    ref = alg1.apply_batch(fd.make_plan(N, L, OM), hin, params[sample])
    check_cells(got, ref, 1e-5, cells=sample)


def test_n64_per_cell_maxwellians_ragged():
    h, params = mixed_inputs(N, L, 7, seed=1300)
    got = run("f64", h, params)
    ref = alg1.apply_batch(fd.make_plan(N, L, OM), h[[0, 6]], params[[0, 6]])
    check(got[0], ref[0], 1e-12)
    check(got[6], ref[1], 1e-12)


def test_n64_rejects_fused():
    import ctypes
    for dt, path in [("f32", "fused"), ("bf16x3", "fused")]:
        p = lc.make_params(N, L, OM, dt, path=path)
        hnd = ctypes.c_void_p()
        assert lc.library().lincoll_plan_ex(ctypes.byref(p), ctypes.byref(hnd)) == lc.EINVAL
