"""Artificial viscosity (Eq. mhd:v with rho = 1, uniform nu) at 128 x 128 x
256, the size at which the 7-point march runs 8-plane chunks per workgroup:
one RKL2 super-step of all three velocity components in one call, and one
backward-Euler Jacobi-PCG solve of a component, against the oracle on the
whole grid, element by element (1e-12 relative; PCG iteration counts within
one).  dt = 100 x the operator's explicit limit (s = 20)."""
import numpy as np
import pytest

from helpers import relmax
from oracle import operator as O
from oracle import pcg as opcg
from oracle import rkl2 as orkl2
from workloads import shell_faces, velocity

pytestmark = pytest.mark.gpu

SHAPE = (128, 128, 256)
BC = (1, 0, 0, 0, 2, 2)
NU = 1.0
RATIO = 100.0


@pytest.fixture(scope="module")
def visc(gpu_lib):
    rf, thf, phf = shell_faces(*SHAPE)
    v = np.stack(velocity(rf, thf, phf))
    op = O.assemble("spherical", rf, thf, phf, O.isotropic_tensor(SHAPE, NU),
                    (O.DIRICHLET, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.PERIODIC, O.PERIODIC))
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, rf, thf, phf, BC)
    ctx.set_dirichlet(0, value=0.0)
    ctx.set_isotropic(NU)
    yield v, op, ctx
    ctx.close()


def test_viscosity_rkl2_three_components_full_grid(visc):
    import torch
    v, op, ctx = visc
    dte = O.gershgorin_dt_euler(op)
    assert ctx.dt_euler() == pytest.approx(dte, rel=1e-12)
    dt = RATIO * dte
    u = torch.from_numpy(v.copy()).cuda()
    s = ctx.rkl2_step(u, dt)
    assert s == orkl2.stage_count(RATIO)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for m in range(3):
        ref = orkl2.rkl2_step(lambda x: O.apply_F(op, x), v[m], dt, s)
        assert relmax(got[m], ref) <= 1e-12, m
        assert relmax(got[m] - v[m], ref - v[m]) <= 1e-9, m


def test_viscosity_jacobi_pcg_full_grid(visc):
    import torch
    v, op, ctx = visc
    dt = RATIO * O.gershgorin_dt_euler(op)
    m = 1
    x = torch.from_numpy(v[m].copy()).cuda()
    it, rel, st = ctx.be_pcg_solve(torch.from_numpy(v[m].copy()).cuda(), x, dt, rtol=1e-8)
    ref = opcg.be_pcg(op, v[m], dt, "jacobi", rtol=1e-8)
    assert st == 0 and ref.converged and rel <= 1e-8
    assert abs(it - ref.iters) <= 1, (it, ref.iters)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    assert relmax(xh, ref.x) <= 2e-12
    _, b = O.be_system(op, v[m], dt)
    vmin = float(np.min(op.V))
    assert np.linalg.norm(xh - ref.x) <= 2 * 1e-8 * np.linalg.norm(b) / vmin
