"""Where a PCG solve stops (Sec. 2.2, Fig. pcg), on the 32 x 32 x 64 shell.

The stopping test of an iteration is taken either by the next iteration's
first sweep or, after the last allowed iteration, by a kernel of its own; these
tests pin that bookkeeping:
  * maxit = 0 returns the initial guess untouched with STS_NOT_CONVERGED;
  * a solve allowed exactly the iteration count at which it converges reports
    convergence with that count and the same x, bit for bit, as an unlimited
    solve; one iteration fewer reports STS_NOT_CONVERGED after that many
    (Jacobi, block ILU0 and the factored preconditioner);
  * the same for the FP32 form (total inner iterations)."""
import numpy as np
import pytest

from helpers import oracle_spitzer
from oracle import operator as O
from workloads import make_workload

pytestmark = pytest.mark.gpu
SHELL_BC = (1, 0, 0, 0, 2, 2)


def _cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dtype) if dtype is not None else t


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def w():
    return make_workload("shell32")


def _ctx(sts, w, f32=False):
    import torch
    c = sts.Context(sts.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    c.set_dirichlet(0, value=w["T_inner"])
    if f32:
        f = torch.float32
        c.set_spitzer_f32(_cuda(w["T"], f), w["kappa0"], _cuda(w["br"], f), _cuda(w["bt"], f),
                          _cuda(w["bp"], f))
    else:
        c.set_spitzer(_cuda(w["T"]), w["kappa0"], _cuda(w["br"]), _cuda(w["bt"]), _cuda(w["bp"]))
    return c


def _dt(w):
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], SHELL_BC, u_lo=w["T_inner"])
    return 50.0 * O.gershgorin_dt_euler(op)


def _solve(c, w, dt, pc, maxit):
    x = _cuda(w["T"])
    it, rel, st = c.be_pcg_solve(_cuda(w["T"]), x, dt, pc=pc, rtol=1e-9, maxit=maxit,
                                 allow_not_converged=True)
    return it, rel, st, _host(x)


@pytest.mark.parametrize("pc", [0, 1, 2])
def test_fp64_stop_at_maxit(gpu_lib, w, pc):
    """Jacobi, block ILU0 and the factored M^-1 = G G^T (a seeded factor)."""
    c = _ctx(gpu_lib, w)
    dt = _dt(w)
    if pc == gpu_lib.PC_FACTOR:
        rng = np.random.default_rng(12)
        g = np.zeros((4,) + w["T"].shape, np.float32)
        g[0] = 1e-3 * (1.0 + 0.1 * rng.random(w["T"].shape))
        g[1:] = 1e-4 * rng.standard_normal((3,) + w["T"].shape)
        c.set_pc_factor(_cuda(g))
    n, rel, st, x = _solve(c, w, dt, pc, 10000)
    assert st == 0 and n > 2 and rel <= 1e-9
    it0, _, st0, x0 = _solve(c, w, dt, pc, 0)
    assert st0 == gpu_lib.STS_NOT_CONVERGED and it0 == 0 and np.array_equal(x0, w["T"])
    itn, reln, stn, xn = _solve(c, w, dt, pc, n)
    assert stn == 0 and itn == n and reln == rel and np.array_equal(xn, x)
    itm, relm, stm, _ = _solve(c, w, dt, pc, n - 1)
    assert stm == gpu_lib.STS_NOT_CONVERGED and itm == n - 1 and relm > 1e-9
    c.close()


def test_fp32_form_stop_at_maxit(gpu_lib, w):
    c = _ctx(gpu_lib, w, f32=True)
    dt = _dt(w)
    n, rel, st, x = _solve(c, w, dt, 0, 10000)
    assert st == 0 and n > 2 and rel <= 1e-9
    it0, _, st0, x0 = _solve(c, w, dt, 0, 0)
    assert st0 == gpu_lib.STS_NOT_CONVERGED and it0 == 0 and np.array_equal(x0, w["T"])
    itn, reln, stn, xn = _solve(c, w, dt, 0, n)
    assert stn == 0 and itn == n and reln == rel and np.array_equal(xn, x)
    c.close()
