"""Out-of-memory paths through the C ABI, with allocation failures injected
by lincoll_debug_fail_alloc: a failed call returns LINCOLL_ENOMEM, later
calls either allocate again and give the right result or report
LINCOLL_ENOTREADY, and nothing is launched on a freed buffer."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
from test_gpu_parity import mixed_inputs  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _no_injection_left():
    yield
    lc.library().lincoll_debug_fail_alloc(0)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def status_of(fn, *a):
    try:
        fn(*a)
    except lc.LincollError as e:
        return e.status
    return lc.OK


def reference(n, L, om, dtype, path, h, params):
    plan = lc.Plan(n, L, om, dtype, path=path)
    plan.set_maxwellians(dev(params))
    out = plan.apply(dev(h, torch.float64 if dtype == "f64" else torch.float32))
    torch.cuda.synchronize()
    r = out.double().cpu().numpy()
    plan.close()
    return r


@pytest.mark.parametrize("k", [1, 4, 10])
def test_failed_maxwellian_growth_leaves_plan_not_ready(k):
    """The k-th allocation of the grown per-cell cache fails (first, middle,
    last buffer): the old cache is gone, so applies report ENOTREADY until
    set_maxwellians succeeds; then the results are right."""
    n, L, om = 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 5, seed=2500 + k)
    plan = lc.Plan(n, L, om, "f64")
    plan.set_maxwellians(dev(params[:2]))
    plan.apply(dev(h[:2]))
    torch.cuda.synchronize()
    lc.library().lincoll_debug_fail_alloc(k)
    assert status_of(plan.set_maxwellians, dev(params)) == lc.ENOMEM
    lc.library().lincoll_debug_fail_alloc(0)
    assert status_of(plan.apply, dev(h[:2])) == lc.ENOTREADY
    assert status_of(plan.apply, dev(h)) == lc.ENOTREADY
    assert plan.info("maxw_batch") == 0
    plan.set_maxwellians(dev(params))
    got = plan.apply(dev(h)).cpu().numpy()
    assert np.array_equal(got, reference(n, L, om, "f64", "auto", h, params))


@pytest.mark.parametrize("dtype,path,k", [("f64", "staged", 1), ("f64", "staged", 3), ("f32", "fused", 1),
                                          ("f32", "staged", 5)])
def test_failed_work_allocation_is_recovered(dtype, path, k):
    """An apply whose work buffers fail to allocate returns ENOMEM; the next
    apply allocates them again and matches a fresh plan bit for bit."""
    n, L, om = 32 if path == "fused" else 16, 8.0, 0.74
    h, params = mixed_inputs(n, L, 3, seed=2600 + k)
    td = torch.float64 if dtype == "f64" else torch.float32
    plan = lc.Plan(n, L, om, dtype, path=path)
    plan.set_maxwellians(dev(params))
    lc.library().lincoll_debug_fail_alloc(k)
    assert status_of(plan.apply, dev(h, td)) == lc.ENOMEM
    lc.library().lincoll_debug_fail_alloc(0)
    got = plan.apply(dev(h, td)).double().cpu().numpy()
    assert np.array_equal(got, reference(n, L, om, dtype, path, h, params))


def test_failed_quadcoll_and_rk4_buffers_are_recovered():
    n, L, om = 8, 4.0, 1.0
    h, params = mixed_inputs(n, L, 2, seed=2700)
    plan = lc.Plan(n, L, om, "f64")
    f = dev(h)
    lc.library().lincoll_debug_fail_alloc(3)
    assert status_of(plan.quadcoll, f) == lc.ENOMEM
    lc.library().lincoll_debug_fail_alloc(0)
    q1 = plan.quadcoll(f).cpu().numpy()
    q2 = lc.Plan(n, L, om, "f64").quadcoll(f).cpu().numpy()
    assert np.array_equal(q1, q2)
    plan.set_maxwellians(dev(params))
    g = dev(h)
    plan.apply(g)          # the apply work buffers exist; the next allocations are RK4's stage buffers
    torch.cuda.synchronize()
    lc.library().lincoll_debug_fail_alloc(2)
    assert status_of(plan.rk4, g, 0.1, 1) == lc.ENOMEM
    lc.library().lincoll_debug_fail_alloc(0)
    plan.rk4(g, 0.1, 2)
    ref = lc.Plan(n, L, om, "f64")
    ref.set_maxwellians(dev(params))
    g2 = dev(h)
    ref.rk4(g2, 0.1, 2)
    torch.cuda.synchronize()
    assert torch.equal(g, g2)
