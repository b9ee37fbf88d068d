"""The largest grid a context accepts: 1023 x 1024 x 1024 = 1 072 693 248
cells, just under the 2^30 - 1 cell limit (the library rejects 1024^3; see
test_abi.py).  32-bit cell indices come closest to overflow here.  Inputs are
products of small host factors expanded on the device (about 110 GB of
device memory in all): b is the tilted dipole, which depends on (theta, phi)
only, and T(r, theta, phi) = A(r) B(theta, phi) with a smooth angular
pattern.  F and a three-stage RKL2 step are compared with the oracle at
sampled boundary and interior cells, each on the window of the grid that
determines it (rows of F need cells within 2; a 3-stage step within 5)."""
import math

import numpy as np
import pytest

from helpers import relmax, window_op
from workloads import dipole_bhat, shell_faces

pytestmark = pytest.mark.gpu
SHAPE = (1023, 1024, 1024)
SHELL_BC = (1, 0, 0, 0, 2, 2)
CELLS = [(0, 0, 0), (1022, 1023, 1023), (0, 512, 1023), (1022, 0, 511), (511, 700, 3),
         (777, 1023, 640)]


class _Outer:
    """T[i, j, k] = A[i] * B[j, k] without forming T: slicing then fancy
    indexing along phi (what the oracle window does) yields the product."""

    def __init__(self, A, B):
        self.A, self.B = A, B

    def __getitem__(self, sl):
        outer = self

        class _Rows:
            def __getitem__(self, idx):
                return outer.A[sl[0]][:, None, None] * outer.B[sl[1]][:, idx[2]][None]
        return _Rows()


class _Angular:
    """b[i, j, k] = b2[j, k] for every i, sliced the same way."""

    def __init__(self, b2):
        self.b2 = b2

    def __getitem__(self, sl):
        outer = self
        n0 = len(range(*sl[0].indices(SHAPE[0])))

        class _Rows:
            def __getitem__(self, idx):
                return np.broadcast_to(outer.b2[sl[1]][:, idx[2]][None],
                                       (n0,) + outer.b2[sl[1]][:, idx[2]].shape).copy()
        return _Rows()


@pytest.fixture(scope="module")
def big(gpu_lib):
    import torch
    rf, thf, phf = shell_faces(*SHAPE)
    rc = 0.5 * (rf[1:] + rf[:-1])
    tc = 0.5 * (thf[1:] + thf[:-1])
    pc = 0.5 * (phf[1:] + phf[:-1])
    A = 1e6 * (1.0 + 0.5 / rc ** 2)
    B = 1.0 + 0.1 * np.sin(2.0 * tc)[:, None] * np.cos(3.0 * pc)[None, :]
    # one r-row of the dipole field: it does not depend on r
    b2 = [c[0] for c in dipole_bhat(rf[:2], thf, phf)]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T = (dev(A)[:, None, None] * dev(B)[None]).contiguous()
    bg = [dev(c)[None].expand(SHAPE[0], -1, -1).contiguous() for c in b2]
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, rf, thf, phf, SHELL_BC)
    ctx.set_dirichlet(0, value=1.5e6)
    ctx.set_spitzer(T, 1e-15, *bg)
    w = dict(rf=rf, thf=thf, phf=phf, T=_Outer(A, B), br=_Angular(b2[0]), bt=_Angular(b2[1]),
             bp=_Angular(b2[2]), kappa0=1e-15, T_inner=1.5e6)
    yield w, ctx, T
    ctx.close()
    del T, bg
    torch.cuda.empty_cache()


def test_max_grid_F_at_sampled_cells(big):
    from oracle import operator as O
    w, ctx, T = big
    F = ctx.apply_F(T)
    scale = float(F.abs().max())
    got = np.array([float(F[c]) for c in CELLS])
    del F
    ref = []
    for c in CELLS:
        op, take, cc = window_op(w, c, 2)
        ref.append(O.apply_F(op, take(w["T"]))[cc])
    assert math.isfinite(scale) and scale > 0
    assert relmax(got, np.array(ref), scale=scale) <= 1e-12


def test_max_grid_rkl2_at_sampled_cells(big):
    from oracle import operator as O
    from oracle import rkl2 as orkl2
    w, ctx, T = big
    dt = 2.0 * ctx.dt_euler()  # within the 3-stage stability limit of 2.5 dt_E
    u = T.clone()
    assert ctx.rkl2_step(u, dt, 3) == 3
    got = np.array([float(u[c]) for c in CELLS])
    scale = float(u.abs().max())
    del u
    ref = []
    for c in CELLS:
        op, take, cc = window_op(w, c, 5)
        ref.append(orkl2.rkl2_step(lambda v: O.apply_F(op, v), take(w["T"]), dt, 3)[cc])
    assert relmax(got, np.array(ref), scale=scale) <= 1e-12


def test_max_grid_be_jacobi_residual(big, gpu_lib):
    """A converged Jacobi-PCG solve at the largest grid: the oracle's residual
    rows at the sampled cells obey |r_c| <= ||r||_2 <= rtol ||b||_2, with
    ||b||_2 from the separable factors (cell volume = radial x polar x
    azimuthal factor, T = A B) plus the Dirichlet layer i = 0 taken from a
    two-plane oracle slab."""
    from oracle import operator as O
    w, ctx, T = big
    dt = 2.0 * ctx.dt_euler()
    rtol = 1e-10
    x = T.clone()
    it, rel, st = ctx.be_pcg_solve(T, x, dt, pc=gpu_lib.PC_JACOBI, rtol=rtol)
    assert st == 0 and rel <= rtol
    assert ctx.be_residual(T, x, dt) <= 1.01 * rtol
    rf, thf, phf = w["rf"], w["thf"], w["phf"]
    # ||b||^2: rows i >= 1 are V T; row 0 also carries dt g
    vr = (rf[1:] ** 3 - rf[:-1] ** 3) / 3.0
    vt = np.cos(thf[:-1]) - np.cos(thf[1:])
    vp = phf[1:] - phf[:-1]
    A, B = w["T"].A, w["T"].B
    sb = float(np.sum((vt[:, None] * vp[None, :] * B) ** 2))
    slab_T = A[:2, None, None] * B[None]
    b2 = [np.broadcast_to(w[k].b2, (2,) + B.shape) for k in ("br", "bt", "bp")]
    op = O.assemble("spherical", rf[:3], thf, phf, O.spitzer_tensor(slab_T, 1e-15, *b2),
                    (O.DIRICHLET, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.PERIODIC, O.PERIODIC),
                    u_lo=1.5e6)
    b0 = op.V[0] * slab_T[0] + dt * op.g[0]
    bnorm = math.sqrt(float(np.sum((vr[1:] * A[1:]) ** 2)) * sb + float(np.sum(b0 ** 2)))
    r = []
    for c in CELLS:
        opw, take, cc = window_op(w, c, 2)
        # x on the window: gather the window's cells from the device
        i0, i1 = max(0, c[0] - 2), min(SHAPE[0], c[0] + 3)
        j0, j1 = max(0, c[1] - 2), min(SHAPE[1], c[1] + 3)
        ks = [(c[2] + d) % SHAPE[2] for d in range(-2, 3)]
        xw = x[i0:i1, j0:j1][:, :, ks].cpu().numpy()
        A19, b = O.be_system(opw, take(w["T"]), dt)
        r.append((b - O.apply19(A19, xw))[cc])
    assert np.max(np.abs(r)) <= 1.01 * rtol * bnorm, (max(abs(v) for v in r), bnorm)
