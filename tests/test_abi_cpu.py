"""The C-ABI library without a GPU: it loads, exports every symbol the
header declares, rejects bad arguments on the host before touching a
device, and its host-side plan tables match the oracle's independent
computation."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fast_direct as fd
from oracle import grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lincoll.h")

lc = pytest.importorskip("paper_2503_09580_amd.lincoll")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lincoll|quadcoll)_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    syms = declared_symbols()
    assert len(syms) >= 12
    lib = lc.library()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(lc.SYMBOLS)


def test_strerror():
    lib = lc.library()
    assert lib.lincoll_strerror(0) == b"success"
    assert lib.lincoll_strerror(-1) == b"invalid argument"
    assert lib.lincoll_strerror(-5) == b"not implemented"
    assert lib.lincoll_strerror(-7) == b"non-finite values in the output"
    assert lib.lincoll_strerror(-99) == b"unknown status"


@pytest.mark.parametrize("kw", [dict(n=12), dict(n=0), dict(n=128), dict(L=0.0), dict(L=-1.0),
                                dict(omega=0.4), dict(omega=1.2), dict(dtype=7), dict(eps=-1.0),
                                dict(quad_rule=3), dict(max_batch=-2), dict(path=9), dict(J=-3)])
def test_plan_rejects_bad_parameters_on_host(kw):
    base = dict(n=16, L=8.0, omega=0.74, dtype="f64")
    n, L, om = kw.pop("n", base["n"]), kw.pop("L", base["L"]), kw.pop("omega", base["omega"])
    dt = kw.pop("dtype", None)
    p = lc.make_params(n, L, om, "f64", **kw)
    if dt is not None:
        p.dtype = dt
    h = ctypes.c_void_p()
    st = lc.library().lincoll_plan_ex(ctypes.byref(p), ctypes.byref(h))
    assert st == lc.EINVAL
    assert not h.value


def test_null_handles_rejected():
    lib = lc.library()
    nullp = ctypes.c_void_p()
    assert lib.lincoll_plan(16, 8.0, 0.74, 0, None) == lc.EINVAL
    assert lib.lincoll_apply(nullp, nullp, nullp, 1) == lc.EINVAL
    assert lib.lincoll_set_maxwellians(nullp, nullp, 1) == lc.EINVAL
    assert lib.lincoll_project(nullp, nullp, nullp, 1) == lc.EINVAL
    assert lib.quadcoll_apply(nullp, nullp, nullp, 1) == lc.EINVAL
    v = ctypes.c_double()
    assert lib.lincoll_get_info(nullp, 0, ctypes.byref(v)) == lc.EINVAL
    assert lib.lincoll_get_info(nullp, lc.INFO["hip_error"], ctypes.byref(v)) == lc.OK   # thread's last HIP error
    assert lib.lincoll_set_option(nullp, 0, 1) == lc.EINVAL
    assert lib.lincoll_autotune(nullp, nullp, nullp, 1, 3) == lc.EINVAL
    sp = lc.steady_params(4)
    rep = lc.SteadyReport()
    assert lib.lincoll_steady_residual(nullp, ctypes.byref(sp), nullp, nullp, None) == lc.EINVAL
    assert lib.lincoll_steady_newton_apply(nullp, ctypes.byref(sp), nullp, nullp, nullp) == lc.EINVAL
    assert lib.lincoll_steady_solve(nullp, ctypes.byref(sp), nullp, ctypes.byref(rep)) == lc.EINVAL
    assert lib.lincoll_steady_precondition(nullp, ctypes.byref(sp), nullp, nullp, nullp) == lc.EINVAL
    assert lib.lincoll_learned_features(nullp, ctypes.byref(sp), nullp, nullp, nullp, None) == lc.EINVAL
    assert lib.lincoll_learned_correction(nullp, ctypes.byref(sp), nullp, nullp, 1.0, nullp) == lc.EINVAL
    # the network: null handles and arguments are rejected before any device call
    assert lib.lincoll_mlp_create(1, None) == lc.EINVAL
    assert lib.lincoll_mlp_set_stream(nullp, nullp) == lc.EINVAL
    w = (ctypes.c_float * lc.MLP_WEIGHTS)()
    assert lib.lincoll_mlp_weights(nullp, w, lc.MLP_WEIGHTS, 0) == lc.EINVAL
    assert lib.lincoll_mlp_forward(nullp, nullp, nullp, 1) == lc.EINVAL
    assert lib.lincoll_mlp_loss_grad(nullp, nullp, nullp, 1, nullp, None) == lc.EINVAL
    assert lib.lincoll_mlp_train(nullp, nullp, nullp, 1, 1, 1e-3, None) == lc.EINVAL
    lib.lincoll_mlp_destroy(nullp)
    lib.lincoll_destroy(nullp)


@pytest.mark.parametrize("n,L,omega,rule", [(8, 4.0, 1.0, 0), (16, 8.0, 0.74, 0), (32, 8.0, 0.5, 0),
                                            (16, 8.0, 0.74, 1), (64, 10.0, 0.74, 0)])
def test_host_tables_match_oracle(n, L, omega, rule):
    """Plan precomputation (C++, own Golub-Welsch) against the oracle
    (numpy eigensolver, dense DFTs): at most 1e-13 relative."""
    p = fd.make_plan(n, L, omega, rule=rule)
    N = n // 2
    g = lc.plan_tables(n, L, omega, "g", quad_rule=rule)
    W = lc.plan_tables(n, L, omega, "W", quad_rule=rule)
    Phi = lc.plan_tables(n, L, omega, "Phi", quad_rule=rule).reshape(p.J, -1)
    Om = lc.plan_tables(n, L, omega, "Omega", quad_rule=rule)
    phi = lc.plan_tables(n, L, omega, "phi", quad_rule=rule).reshape(p.J, N + 1, N + 1, N + 1)
    np.testing.assert_allclose(g, p.g, rtol=0, atol=1e-13 * p.R)
    np.testing.assert_allclose(W, p.W, rtol=0, atol=1e-13 * p.W.max())
    k2 = np.rint(grid.kabs2(n)).astype(int)
    np.testing.assert_allclose(Phi[:, k2], p.Phi, rtol=0, atol=1e-13 * np.abs(p.Phi).max())
    np.testing.assert_allclose(Om[k2], p.Omega, rtol=0, atol=1e-13 * np.abs(p.Omega).max())
    idx = np.r_[N:n, 0]          # octant |d| = 0..N  ->  storage index N+d, with |d| = N at 0
    po = p.phi[:, idx][:, :, idx][:, :, :, idx]
    np.testing.assert_allclose(phi, po, rtol=0, atol=1e-13 * np.abs(po).max())


def test_plan_tables_rejects_small_buffer():
    lib = lc.library()
    p = lc.make_params(8, 4.0, 1.0)
    out = (ctypes.c_double * 2)()
    assert lib.lincoll_plan_tables(ctypes.byref(p), 0, out, 2) == lc.EINVAL
    assert lib.lincoll_plan_tables(ctypes.byref(p), 99, None, 0) == lc.EINVAL


def test_mlp_constants_match_header():
    import re
    hdr = open(os.path.join(ROOT, "include", "lincoll.h")).read()
    vals = {k: int(v) for k, v in re.findall(r"#define LINCOLL_MLP_(IN|HIDDEN|OUT) (\d+)", hdr)}
    assert (vals["IN"], vals["HIDDEN"], vals["OUT"]) == (lc.MLP_IN, lc.MLP_HIDDEN, lc.MLP_OUT)
    assert lc.MLP_WEIGHTS == 26 * 128 + 128 + 128 * 5 + 5


def test_steady_defaults():
    sp = lc.steady_params(256)
    assert (sp.nx, sp.x_l, sp.x_r, sp.kn, sp.mass, sp.theta_l, sp.theta_r) == (256, -0.5, 0.5, 0.1, 1.0, 1.0, 1.5)
    assert (sp.tol, sp.inner_rtol, sp.inner_atol) == (1e-5, 1e-3, 1e-7)
    assert (sp.restart, sp.init) == (30, 1) and list(sp.u_l) == [0.0, 0.0, 0.0]
    sp = lc.steady_params(3, u_r=(0.0, 0.4, 0.0), kn=1.0)
    assert list(sp.u_r) == [0.0, 0.4, 0.0] and sp.kn == 1.0
