"""GPU parity of the super-step variants of Sec. 6 (rkl_step) against the
oracle (oracle/rkl_variants.py) on the 32 x 32 x 64 shell, and on three
viscosity components.  Tolerances as for rkl2_step: 1e-12 relative in u,
1e-9 relative in the increment u^{n+1} - u^n (cancellation of u ~ 1e6)."""
import numpy as np
import pytest

from helpers import gpu_spitzer, oracle_spitzer, relmax, small_shell
from oracle import operator as O
from oracle import rkl2 as R2
from oracle import rkl_variants as V
from workloads import make_workload

pytestmark = pytest.mark.gpu
SHELL_BC = (1, 0, 0, 0, 2, 2)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def shell32(gpu_lib):
    w = make_workload("shell32")
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], SHELL_BC, u_lo=w["T_inner"])
    ctx = gpu_spitzer(gpu_lib, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], SHELL_BC, u_lo=w["T_inner"])
    return w, op, ctx


CASES = [
    dict(scheme=2),
    dict(scheme=1),
    dict(scheme=1, extra=2),
    dict(scheme=2, extra=1, odd=True),
    dict(scheme=2, nsub=3),
    dict(scheme=2, euler_fraction=0.25),
    dict(scheme=1, extra=1, nsub=2, euler_fraction=0.25, euler_cfl=0.8),
]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_rkl_step_variants(shell32, case):
    w, op, ctx = shell32
    dte = O.gershgorin_dt_euler(op)
    dt = 50.0 * dte
    u = _cuda(w["T"])
    n = ctx.rkl_step(u, dt, **case)
    kw = dict(case)
    ref, n_ref = V.super_step(lambda v: O.apply_F(op, v), w["T"], dt, dte,
                              scheme=kw.pop("scheme"), extra=kw.pop("extra", 0),
                              odd=kw.pop("odd", False), nsub=kw.pop("nsub", 1),
                              euler_fraction=kw.pop("euler_fraction", 0.0),
                              euler_cfl=kw.pop("euler_cfl", 0.5))
    got = _host(u)
    assert n == n_ref
    assert relmax(got, ref) <= 1e-12
    assert relmax(got - w["T"], ref - w["T"]) <= 1e-9


def test_rkl_step_default_equals_rkl2_step(shell32):
    w, op, ctx = shell32
    dt = 50.0 * ctx.dt_euler()
    a, b = _cuda(w["T"]), _cuda(w["T"])
    s = ctx.rkl2_step(a, dt)
    n = ctx.rkl_step(b, dt)
    assert n == s and np.array_equal(_host(a), _host(b))


def test_rkl1_viscosity_components(gpu_lib):
    w = small_shell((10, 12, 20))
    v = np.random.default_rng(4).standard_normal((3,) + w["T"].shape)
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    ctx.set_dirichlet(0, value=0.0)
    ctx.set_isotropic(0.7)
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], O.isotropic_tensor(v[0].shape, 0.7),
                    (O.DIRICHLET, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.PERIODIC, O.PERIODIC))
    dte = O.gershgorin_dt_euler(op)
    dt = 80.0 * dte
    u = _cuda(v)
    ctx.rkl_step(u, dt, scheme=1, extra=1, nsub=2)
    got = _host(u)
    for m in range(3):
        ref, _ = V.super_step(lambda x: O.apply_F(op, x), v[m], dt, dte, scheme=1, extra=1, nsub=2)
        assert relmax(got[m], ref) <= 1e-12


def test_rkl_step_errors(shell32, gpu_lib):
    w, op, ctx = shell32
    u = _cuda(w["T"])
    dt = 10.0 * ctx.dt_euler()
    for kw in (dict(scheme=3), dict(nsub=0), dict(euler_fraction=1.0),
               dict(euler_fraction=0.2, euler_cfl=0.0), dict(extra=-1)):
        with pytest.raises(gpu_lib.StsError):
            ctx.rkl_step(u, dt, **kw)
    assert np.array_equal(_host(u), w["T"])  # rejected calls leave u untouched


def test_rkl_step_fp32_form(gpu_lib):
    """The FP32 form runs RKL2 sub-steps; other variants are rejected."""
    import torch
    w = make_workload("shell32")
    f32 = torch.float32
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    ctx.set_dirichlet(0, value=w["T_inner"])
    ctx.set_spitzer_f32(_cuda(w["T"]).to(f32), w["kappa0"], _cuda(w["br"]).to(f32),
                        _cuda(w["bt"]).to(f32), _cuda(w["bp"]).to(f32))
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], SHELL_BC, u_lo=w["T_inner"])
    dte = O.gershgorin_dt_euler(op)
    u = _cuda(w["T"])
    ctx.rkl_step(u, 50.0 * ctx.dt_euler(), nsub=2)
    ref, _ = V.super_step(lambda v: O.apply_F(op, v), w["T"], 50.0 * dte, dte, nsub=2)
    assert relmax(_host(u), ref, scale=np.max(np.abs(w["T"]))) <= 1e-6
    with pytest.raises(gpu_lib.StsError):
        ctx.rkl_step(u, 10.0 * dte, scheme=1)
