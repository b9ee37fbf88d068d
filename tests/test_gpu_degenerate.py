"""Degenerate cases of the method on the 32 x 32 x 64 shell:
  * a zero problem (u^n = 0, zero Dirichlet value: b = 0) is solved at the
    initial check, with no iteration and x left at 0;
  * a constant state under zero-flux boundaries is steady: F(c) = 0 exactly
    (every face and edge difference vanishes), BE returns x = c after no
    iteration, RKL2 keeps c up to the rounding of its recurrence;
  * a vanishing step, dt = 1e-8 dt_E: RKL2 takes the minimum s = 2 and BE
    converges at once, both equal to the oracle's to 1e-12."""
import numpy as np
import pytest

from helpers import oracle_spitzer, relmax
from oracle import operator as O
from oracle import pcg as opcg
from oracle import rkl2 as orkl2
from workloads import make_workload

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _ctx(sts, w, bc, u_lo):
    c = sts.Context(sts.SPHERICAL, w["rf"], w["thf"], w["phf"], bc)
    if bc[0] == sts.BC_DIRICHLET:
        c.set_dirichlet(0, value=u_lo)
    c.set_spitzer(_cuda(w["T"]), w["kappa0"], _cuda(w["br"]), _cuda(w["bt"]), _cuda(w["bp"]))
    return c


@pytest.fixture(scope="module")
def w():
    return make_workload("shell32")


def test_zero_problem_needs_no_iteration(gpu_lib, w):
    c = _ctx(gpu_lib, w, (1, 0, 0, 0, 2, 2), 0.0)
    dt = 50.0 * c.dt_euler()
    zero = _cuda(np.zeros_like(w["T"]))
    x = zero.clone()
    it, rel, st = c.be_pcg_solve(zero, x, dt, rtol=1e-12)
    assert st == 0 and it == 0 and rel == 0.0
    assert not np.any(_host(x))
    c.close()


def test_constant_state_is_steady(gpu_lib, w):
    c = _ctx(gpu_lib, w, (0, 0, 0, 0, 2, 2), 0.0)
    dt = 50.0 * c.dt_euler()
    const = np.full_like(w["T"], 1.25e6)
    F = _host(c.apply_F(_cuda(const)))
    assert not np.any(F)
    x = _cuda(const)
    it, rel, st = c.be_pcg_solve(_cuda(const), x, dt, rtol=1e-12)
    assert st == 0 and it == 0
    assert np.array_equal(_host(x), const)
    u = _cuda(const)
    s = c.rkl2_step(u, dt)
    assert s == orkl2.stage_count(50.0)
    assert relmax(_host(u), const) <= 1e-15 * s
    c.close()


def test_vanishing_step(gpu_lib, w):
    c = _ctx(gpu_lib, w, (1, 0, 0, 0, 2, 2), w["T_inner"])
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], (1, 0, 0, 0, 2, 2), u_lo=w["T_inner"])
    dt = 1e-8 * O.gershgorin_dt_euler(op)
    u = _cuda(w["T"])
    s = c.rkl2_step(u, dt)
    assert s == 2 == orkl2.stage_count(1e-8)
    ref = orkl2.rkl2_step(lambda v: O.apply_F(op, v), w["T"], dt, 2)
    assert relmax(_host(u), ref) <= 1e-12
    x = _cuda(w["T"])
    it, rel, st = c.be_pcg_solve(_cuda(w["T"]), x, dt, rtol=1e-10)
    res = opcg.be_pcg(op, w["T"], dt, "jacobi", rtol=1e-10)
    assert st == 0 and it <= 2 and abs(it - res.iters) <= 1
    assert relmax(_host(x), res.x) <= 1e-12
    c.close()
