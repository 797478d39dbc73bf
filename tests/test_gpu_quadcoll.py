"""quadcoll_apply (binary operator Q(f, f), eq. (14), hemisphere product rule)
through the C ABI against the oracle's binary method (O2), FP64, 1e-12.

Also the polarisation identity Q(M+h) - Q(M) - Q(h) = Q(M,h) + Q(h,M), i.e.
the linearized binary operator of Sec. 4.1, against O2's direct evaluation of
that linearization (bilinearity of the GPU evaluation)."""
import numpy as np
import pytest

from oracle import binary, fast_direct as fd, quadrature
from paper_2503_09580_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")
from test_gpu_parity import mixed_inputs  # noqa: E402
from parity_util import check  # noqa: E402

DEV = torch.device("cuda:0")


def gpu_q(n, L, om, f, polar=8, azim=16):
    plan = lc.Plan(n, L, om, "f64")
    plan.set_option("sphere_polar", polar)
    plan.set_option("sphere_azimuth", azim)
    out = plan.quadcoll(torch.from_numpy(np.ascontiguousarray(f)).to(DEV, torch.float64))
    torch.cuda.synchronize()
    return out.cpu().numpy()


# The kernel shares the first-axis transform between azimuths m and
# n_azim - m: odd counts (one unpaired azimuth), one and two azimuths (no
# pairs) and n = 32 (where the c/d exchange is a wave-half swap) are covered.
@pytest.mark.parametrize("n,L,om,polar,azim", [
    (8, 4.0, 1.0, 8, 16), (16, 8.0, 0.74, 8, 16), (16, 8.0, 0.5, 6, 10),
    (8, 4.0, 1.0, 6, 7), (16, 8.0, 0.74, 4, 1), (16, 8.0, 0.74, 4, 2), (16, 8.0, 0.74, 4, 9),
    (32, 8.0, 0.74, 4, 5), (32, 8.0, 0.74, 4, 6)])
def test_quadcoll_matches_binary_oracle(n, L, om, polar, azim):
    h, params = mixed_inputs(n, L, 3, seed=1600 + n + polar)
    f = h + np.stack([wl.maxwellian(n, L, q[0], q[1:4], q[4]) for q in params])
    got = gpu_q(n, L, om, f, polar, azim)
    plan = fd.make_plan(n, L, om)
    sphere = quadrature.hemisphere_product_rule(polar, azim)
    for b in range(3):
        ref = binary.q_binary(plan, sphere, f[b], f[b], method="fast")
        check(got[b], ref, 1e-12, tag=b)


def test_hemisphere_rule_changes_between_calls():
    """One plan, successive calls with different hemisphere rules: the
    azimuth phase tables grow (reallocation) and shrink (reuse) with the
    rule, and every call matches the oracle at 1e-12."""
    n, L, om = 8, 4.0, 1.0
    h, params = mixed_inputs(n, L, 2, seed=1650)
    f = h + np.stack([wl.maxwellian(n, L, q[0], q[1:4], q[4]) for q in params])
    plan = lc.Plan(n, L, om, "f64")
    fd_plan = fd.make_plan(n, L, om)
    fdev = torch.from_numpy(np.ascontiguousarray(f)).to(DEV, torch.float64)
    for polar, azim in [(4, 6), (8, 16), (4, 5), (10, 24), (2, 1)]:
        plan.set_option("sphere_polar", polar)
        plan.set_option("sphere_azimuth", azim)
        got = plan.quadcoll(fdev).cpu().numpy()
        sphere = quadrature.hemisphere_product_rule(polar, azim)
        for b in range(2):
            ref = binary.q_binary(fd_plan, sphere, f[b], f[b], method="fast")
            check(got[b], ref, 1e-12, tag=(polar, azim, b))


def test_polarisation_gives_the_linearized_binary_operator():
    n, L, om = 16, 8.0, 0.74
    M = wl.maxwellian(n, L, 1.0, (0, 0, 0), 1.0)
    h, _ = mixed_inputs(n, L, 1, seed=1700, per_cell=False)
    q = gpu_q(n, L, om, np.stack([M + h[0], M, h[0]]))
    lin_gpu = q[0] - q[1] - q[2]
    plan = fd.make_plan(n, L, om)
    ref = binary.linearized_binary(plan, quadrature.hemisphere_product_rule(8, 16), h[0], M)
    check(lin_gpu, ref, 1e-10)


def test_quadcoll_errors():
    import ctypes
    lib = lc.library()
    plan = lc.Plan(16, 8.0, 0.74, "f64")
    x = torch.zeros((2, 16, 16, 16), dtype=torch.float64, device=DEV)
    p = ctypes.c_void_p(x.data_ptr())
    assert lib.quadcoll_apply(plan._h, p, p, 2) == lc.EINVAL               # aliased
    assert lib.lincoll_set_option(plan._h, lc.OPTIONS["sphere_polar"], 7) == lc.EINVAL
    big = lc.Plan(64, 10.0, 0.74, "f32")
    y = torch.zeros((1, 64, 64, 64), dtype=torch.float64, device=DEV)
    z = torch.zeros_like(y)
    assert lib.quadcoll_apply(big._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(z.data_ptr()), 1) == lc.ENOTIMPL


@pytest.mark.parametrize("n,L,polar,azim,fix", [
    (8, 4.0, 4, 3, 1), (8, 4.0, 4, 3, 2), (16, 4.5, 4, 5, 1), (16, 4.5, 4, 5, 2), (16, 8.0, 8, 16, 2),
    (32, 8.0, 4, 6, 1), (32, 8.0, 4, 6, 2)])
def test_quadcoll_mass_fixes_match_oracle(n, L, polar, azim, fix):
    """The mass fixes of Sec. 2.3 (LINCOLL_OPT_QUAD_FIX): 1 = Q^_0 set to 0
    (eq. (15)), 2 = the loss sinc replaced by its hemisphere estimate
    (eq. (16)), against O2 with the same fix at 1e-12; fix 1 conserves mass
    to round-off.  The plan switches fixes and rules between calls."""
    h, params = mixed_inputs(n, L, 2, seed=1800 + n + fix)
    f = h + np.stack([wl.maxwellian(n, L, q[0], q[1:4], q[4]) for q in params])
    plan = lc.Plan(n, L, 0.74, "f64")
    plan.set_option("sphere_polar", polar)
    plan.set_option("sphere_azimuth", azim)
    fdev = torch.from_numpy(np.ascontiguousarray(f)).to(DEV, torch.float64)
    plain = plan.quadcoll(fdev).cpu().numpy()
    plan.set_option("quad_fix", fix)
    assert plan.info("quad_fix") == fix
    got = plan.quadcoll(fdev).cpu().numpy()
    fd_plan = fd.make_plan(n, L, 0.74)
    sphere = quadrature.hemisphere_product_rule(polar, azim)
    for b in range(2):
        ref = binary.q_binary(fd_plan, sphere, f[b], f[b], method="fast", fix=fix)
        check(got[b], ref, 1e-12, tag=(fix, b))
        if fix == 1:
            assert abs(got[b].sum()) < 1e-13 * np.abs(got[b]).sum()
    plan.set_option("quad_fix", 0)
    assert np.array_equal(plan.quadcoll(fdev).cpu().numpy(), plain)
