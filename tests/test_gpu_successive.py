"""Successive steps under the lagged-diffusivity protocol (Sec. 2): kappa is
re-frozen from the evolving temperature at the start of every step, the time
step stays at f times the first step's explicit limit, and the RKL2 stage
count follows each step's own dt_Euler (Eq. rkl2_s).  RKL2, Jacobi-PCG and
block-ILU0-PCG are each marched three steps on the 32 x 32 x 64 shell, and
the GPU state is compared with the oracle's after every step, to the same
bars as a single step: 1e-12 relative in u, equal stage counts, PCG
iteration counts within one."""
import numpy as np
import pytest

from helpers import oracle_spitzer, relmax
from oracle import operator as O
from oracle import pcg as opcg
from oracle import rkl2 as orkl2
from workloads import make_workload

pytestmark = pytest.mark.gpu

SHELL_BC = (1, 0, 0, 0, 2, 2)
NSTEPS = 3


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def march(gpu_lib):
    w = make_workload("shell32")
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    ctx.set_dirichlet(0, value=w["T_inner"])
    b = tuple(_cuda(w[k]) for k in ("br", "bt", "bp"))
    yield w, ctx, b
    ctx.close()


def _oracle_op(w, u):
    return oracle_spitzer(w["rf"], w["thf"], w["phf"], u, w["br"], w["bt"], w["bp"],
                          w["kappa0"], SHELL_BC, u_lo=w["T_inner"])


def test_rkl2_successive_steps(march):
    w, ctx, b = march
    u_ref = w["T"].copy()
    dt = w["workload"].dt_factor * O.gershgorin_dt_euler(_oracle_op(w, u_ref))
    u = _cuda(w["T"])
    stages = []
    for n in range(NSTEPS):
        op = _oracle_op(w, u_ref)
        dte = O.gershgorin_dt_euler(op)
        s_ref = orkl2.stage_count(dt / dte)
        ctx.set_spitzer(u, w["kappa0"], *b)
        assert ctx.dt_euler() == pytest.approx(dte, rel=1e-12), n
        s = ctx.rkl2_step(u, dt)
        assert s == s_ref, n
        u_ref = orkl2.rkl2_step(lambda v: O.apply_F(op, v), u_ref, dt, s_ref)
        got = _host(u)
        assert relmax(got, u_ref) <= 1e-12, n
        stages.append(s)
    # the state has moved: later steps see a different diffusivity
    assert relmax(u_ref, w["T"]) > 1e-4


@pytest.mark.parametrize("pc,name", [(0, "jacobi"), (1, "ilu0")])
def test_be_pcg_successive_steps(march, gpu_lib, pc, name):
    w, ctx, b = march
    rtol = w["workload"].rtol
    u_ref = w["T"].copy()
    dt = w["workload"].dt_factor * O.gershgorin_dt_euler(_oracle_op(w, u_ref))
    u = _cuda(w["T"])
    for n in range(NSTEPS):
        op = _oracle_op(w, u_ref)
        ref = opcg.be_pcg(op, u_ref, dt, name, rtol=rtol, block=(8, 8, 8))
        assert ref.converged
        ctx.set_spitzer(u, w["kappa0"], *b)
        x = u.clone()
        it, rel, st = ctx.be_pcg_solve(u, x, dt, pc=pc, block=(8, 8, 8), rtol=rtol)
        assert st == 0 and rel <= rtol and abs(it - ref.iters) <= 1, (n, it, ref.iters)
        assert relmax(_host(x), ref.x) <= 1e-12, n
        # the new state's true residual against this step's system
        assert ctx.be_residual(u, x, dt) <= 2 * rtol
        u, u_ref = x, ref.x
    assert relmax(u_ref, w["T"]) > 1e-4
