"""The 256 x 256 x 512 shell (33.5M cells) at its full size and dt = 500
dt_Euler: conduction and three-component viscosity, RKL2 (s = 45) and
Jacobi-PCG to 1e-8, and the FP32 form.  The oracle cannot run these steps on
the whole grid in test time, so:
  * RKL2: after s stages a cell depends only on the cells within s of it
    (19- and 7-point stencils), whose coefficients involve cells within
    s + 1; the oracle's step on the window of half-width s + 2 around a
    sampled cell is therefore exact at its centre, and is compared to
    1e-12 relative with the GPU's full-grid step (boundary and interior
    cells);
  * BE: the converged solution's residual b - A x is evaluated by the oracle
    at sampled cells (window rows are exact rows of A) and must satisfy the
    bound |r_c| <= ||r||_2 <= rtol ||b||_2 that convergence implies; the
    library's own true-residual norm must meet rtol too;
  * FP32 form: its RKL2 and BE results against the FP64 path (which the
    oracle pins above) to the stated 1e-6 relative in T and 1e-5 of max |v|.
"""
import numpy as np
import pytest

from helpers import relmax, window_op
from oracle import operator as O
from oracle import rkl2 as orkl2
from oracle.geometry import geometry
from workloads import make_workload

pytestmark = pytest.mark.gpu
SHELL_BC = (1, 0, 0, 0, 2, 2)
F = 500.0
RTOL = 1e-8
CELLS = [(0, 0, 0), (255, 255, 511), (0, 131, 260), (130, 0, 7), (97, 201, 389)]


def _cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dtype) if dtype is not None else t


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def big(gpu_lib):
    w = make_workload("shell256", with_velocity=True)
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    ctx.set_dirichlet(0, value=w["T_inner"])
    T = _cuda(w["T"])
    ctx.set_spitzer(T, w["kappa0"], _cuda(w["br"]), _cuda(w["bt"]), _cuda(w["bp"]))
    ctxv = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    ctxv.set_dirichlet(0, value=0.0)
    ctxv.set_isotropic(w["nu"])
    res = {}
    yield w, ctx, ctxv, T, res
    ctx.close()
    ctxv.close()


def _rkl2_window(w, cell, dt, s, kind, field):
    op, take, c = window_op(w, cell, s + 2, kind=kind, nu=w["nu"])
    u = orkl2.rkl2_step(lambda v: O.apply_F(op, v), take(field), dt, s)
    return u[c]


def test_rkl2_conduction_sampled(big):
    w, ctx, _, T, res = big
    dt = F * ctx.dt_euler()
    u = T.clone()
    s = ctx.rkl2_step(u, dt)
    assert s == orkl2.stage_count(F) == 45
    got = _host(u)
    res["rkl2_T"] = got
    res["dt"] = dt
    ref = np.array([_rkl2_window(w, c, dt, s, "spitzer", w["T"]) for c in CELLS])
    assert relmax(np.array([got[c] for c in CELLS]), ref, scale=np.max(np.abs(got))) <= 1e-12
    assert relmax(np.array([got[c] - w["T"][c] for c in CELLS]), ref - w["T"][tuple(
        np.array(CELLS).T)]) <= 1e-9


def test_rkl2_viscosity_sampled(big):
    w, _, ctxv, _, res = big
    v0 = np.stack(w["v"])
    dt = F * ctxv.dt_euler()
    v = _cuda(v0)
    s = ctxv.rkl2_step(v, dt)
    assert s == 45
    got = _host(v)
    res["rkl2_v"] = got
    res["dtv"] = dt
    for m in range(3):
        cells = CELLS[m::2]
        ref = np.array([_rkl2_window(w, c, dt, s, "isotropic", v0[m]) for c in cells])
        assert relmax(np.array([got[m][c] for c in cells]), ref,
                      scale=np.max(np.abs(v0[m]))) <= 1e-12, m


def _b_norm(w, u_n, dt, kind):
    """||b||_2 with b = V u^n + dt g; g is non-zero only on the Dirichlet
    layer i = 0, whose rows the oracle assembles on a two-plane slab."""
    V = geometry("spherical", w["rf"], w["thf"], w["phf"])["V"]
    b = V * u_n
    slab = dict(w, rf=w["rf"][:3])
    for key in ("T", "br", "bt", "bp"):
        slab[key] = w[key][:2]
    if kind == "spitzer":
        D = O.spitzer_tensor(slab["T"], w["kappa0"], slab["br"], slab["bt"], slab["bp"])
        u_lo = w["T_inner"]
    else:
        D = O.isotropic_tensor(slab["T"].shape, w["nu"])
        u_lo = 0.0
    op = O.assemble("spherical", slab["rf"], w["thf"], w["phf"], D,
                    (O.DIRICHLET, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.PERIODIC, O.PERIODIC),
                    u_lo=u_lo)
    b[0] += dt * op.g[0]
    return float(np.linalg.norm(b))


def _residual_at(w, cells, u_n, x, dt, kind):
    out = []
    for c in cells:
        op, take, cc = window_op(w, c, 2, kind=kind, nu=w["nu"])
        A19, b = O.be_system(op, take(u_n), dt)
        out.append((b - O.apply19(A19, take(x)))[cc])
    return np.array(out)


def test_be_jacobi_conduction(big, gpu_lib):
    w, ctx, _, T, res = big
    dt = F * ctx.dt_euler()
    x = T.clone()
    it, rel, st = ctx.be_pcg_solve(T, x, dt, pc=gpu_lib.PC_JACOBI, rtol=RTOL)
    assert st == 0 and rel <= RTOL
    assert ctx.be_residual(T, x, dt) <= 1.01 * RTOL
    xh = _host(x)
    res["be_T"] = xh
    bn = _b_norm(w, w["T"], dt, "spitzer")
    r = _residual_at(w, CELLS, w["T"], xh, dt, "spitzer")
    assert np.max(np.abs(r)) <= 1.01 * RTOL * bn
    assert relmax(xh, w["T"]) > 1e-3  # the step moved the solution


def test_be_jacobi_viscosity(big, gpu_lib):
    w, _, ctxv, _, _ = big
    dt = F * ctxv.dt_euler()
    for m in range(3):
        v0 = _cuda(w["v"][m])
        x = v0.clone()
        it, rel, st = ctxv.be_pcg_solve(v0, x, dt, pc=gpu_lib.PC_JACOBI, rtol=RTOL)
        assert st == 0 and rel <= RTOL, m
        assert ctxv.be_residual(v0, x, dt) <= 1.01 * RTOL
        xh = _host(x)
        bn = _b_norm(w, w["v"][m], dt, "isotropic")
        r = _residual_at(w, CELLS[:3], w["v"][m], xh, dt, "isotropic")
        assert np.max(np.abs(r)) <= 1.01 * RTOL * bn, m


def test_fp32_form_errors(big, gpu_lib, capsys):
    import torch
    w, ctx, _, T, res = big
    assert "rkl2_T" in res and "be_T" in res and "rkl2_v" in res
    f32 = torch.float32
    c32 = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    c32.set_dirichlet(0, value=w["T_inner"])
    c32.set_spitzer_f32(_cuda(w["T"], f32), w["kappa0"], _cuda(w["br"], f32),
                        _cuda(w["bt"], f32), _cuda(w["bp"], f32))
    # the same dt as the FP64 path (the FP32 coefficients' dt_Euler differs in
    # its last digits)
    dt = res["dt"]
    u = T.clone()
    assert c32.rkl2_step(u, dt, 45) == 45
    e_rk = relmax(_host(u), res["rkl2_T"])
    # BE: FP64 reference solved tighter than the form's tolerance
    xr = T.clone()
    it, rel, st = ctx.be_pcg_solve(T, xr, dt, pc=gpu_lib.PC_JACOBI, rtol=1e-12)
    assert st == 0
    x = T.clone()
    it32, rel32, st32 = c32.be_pcg_solve(T, x, dt, pc=gpu_lib.PC_JACOBI, rtol=RTOL)
    assert st32 == 0 and rel32 <= RTOL
    e_be = relmax(_host(x), _host(xr))
    c32.close()
    cv = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    cv.set_dirichlet(0, value=0.0)
    cv.set_isotropic_f32(w["nu"])
    v = _cuda(np.stack(w["v"]))
    assert cv.rkl2_step(v, res["dtv"], 45) == 45
    vh = _host(v)
    e_v = max(relmax(vh[m], res["rkl2_v"][m], scale=np.max(np.abs(w["v"][m])))
              for m in range(3))
    cv.close()
    with capsys.disabled():
        print(f"\n[fp32 form, 256x256x512] RKL2 T max rel err {e_rk:.2e}; BE T max rel err "
              f"{e_be:.2e} ({it32} inner its); RKL2 v err / max|v| {e_v:.2e}")
    assert e_rk <= 1e-6 and e_be <= 1e-6 and e_v <= 1e-5
