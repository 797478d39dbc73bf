"""lincoll_rk4 (RK4 for df/dt = L[f], Sec. 4.2) through the C ABI against
the oracle's RK4 on the same inputs.  Bars: FP64 1e-12, FP32 1e-5 relative
l2 per cell after the steps; graph replay of a step equals the eager step.

FP64 evolves a full distribution f = M + h.  FP32 evolves the perturbation h:
for f = M + h the operator cancels the Maxwellian part (L[M] is at the
discretisation level), so each FP32 apply carries an error of order 1e-6
of |L-[f]| ~ |f|, which RK4 accumulates to ~1e-5 |f| over a few steps; the
perturbation form keeps the FP32 error relative to the evolving state.
Each step combines four applies with weights dt/6 (1, 2, 2, 1) and feeds
each stage's error through L into the next stage; bounding every apply's
error by the FP32 bar taken relative to the loss term |L-[f]| (the
cancellation-aware metric) gives, after S steps, the FP32 bar
1e-5 * (1 + 4 S dt |L-[f0]| / |f_S|)."""
import numpy as np
import pytest

from oracle import fast_direct as fd, timestep
from paper_2503_09580_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
from test_gpu_parity import mixed_inputs  # noqa: E402
from parity_util import check  # noqa: E402

DEV = torch.device("cuda:0")


def gpu_rk4(n, L, om, dtype, f, params, dt, steps, graph=0):
    plan = lc.Plan(n, L, om, dtype)
    plan.set_option("graph", graph)
    plan.set_maxwellians(torch.from_numpy(np.ascontiguousarray(params)).to(DEV, torch.float64))
    td = torch.float64 if dtype == "f64" else torch.float32
    ft = torch.from_numpy(np.ascontiguousarray(f)).to(DEV, td)
    plan.rk4(ft, dt, steps)
    torch.cuda.synchronize()
    return ft.double().cpu().numpy()


@pytest.mark.parametrize("n,dtype,tol", [(16, "f64", 1e-12), (16, "f32", 1e-5), (32, "f32", 1e-5)])
def test_rk4_matches_oracle(n, dtype, tol):
    L, om, dt, steps = 8.0, 0.74, 0.1, 3
    h, params = mixed_inputs(n, L, 3, seed=1400 + n)
    M = np.stack([wl.maxwellian(n, L, q[0], q[1:4], q[4]) for q in params])
    f = M + h if dtype == "f64" else h   # full distribution (FP64) or perturbation (FP32)
    fin = f if dtype == "f64" else f.astype(np.float32).astype(np.float64)
    got = gpu_rk4(n, L, om, dtype, fin, params, dt, steps)
    op = fd.make_plan(n, L, om)
    ref = timestep.rk4(op, fin, params, dt, steps)
    for b in range(3):
        bar = tol
        if dtype == "f32":
            lm = fd.apply(op, fin[b], params[b, 0], params[b, 1:4], params[b, 4], parts=True)[2]
            bar = tol * (1.0 + 4 * steps * dt * np.linalg.norm(lm) / np.linalg.norm(ref[b]))
        check(got[b], ref[b], bar, tag=b)


def test_rk4_graph_replay_equals_eager_and_zero_steps():
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 4, seed=1500)
    f = h + np.stack([wl.maxwellian(n, L, q[0], q[1:4], q[4]) for q in params])
    a = gpu_rk4(n, L, om, "f64", f, params, 0.1, 5, graph=0)
    b = gpu_rk4(n, L, om, "f64", f, params, 0.1, 5, graph=1)
    assert np.array_equal(a, b)
    c = gpu_rk4(n, L, om, "f64", f, params, 0.1, 0, graph=1)
    assert np.array_equal(c, f)
