"""GPU parity of the un-lagged conduction operator and its RKL2 step
(apply_F_nonlinear, rkl2_step_nonlinear) against the oracle
(oracle/nonlinear.py).  Tolerances as for the lagged path: 1e-12 relative in
F and u, 1e-9 relative in the increment u^{n+1} - u^n (T ~ 1e6 cancels).

At 128 x 128 x 256 (the benchmark's launch configuration) the oracle cannot
run whole super-steps in seconds, so there the check is (a) F at sampled
cells, each computed by the oracle on a small window, (b) whole steps of
s = 8 stages at sampled cells, each computed by the oracle on a window of
half-width s + 2 (a stage reaches one cell further, its coefficients one
more), and (c) conservation of sum V u under zero-flux boundaries over a
full step of s = 28 stages."""
import numpy as np
import pytest

from helpers import ORACLE_BC, relmax, small_shell
from oracle import geometry as geo
from oracle import nonlinear as NL
from oracle import operator as O
from workloads import box_faces, make_workload, random_unit_vectors

pytestmark = pytest.mark.gpu
SHELL_BC = (1, 0, 0, 0, 2, 2)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _ctx(sts, f, bc, u_lo=0.0, u_hi=0.0, coord=None):
    ctx = sts.Context(sts.SPHERICAL if coord is None else coord, *f, bc)
    if bc[0] == sts.BC_DIRICHLET:
        ctx.set_dirichlet(0, value=u_lo)
    if bc[1] == sts.BC_DIRICHLET:
        ctx.set_dirichlet(1, value=u_hi)
    return ctx


def _obc(bc):
    return tuple(ORACLE_BC[b] for b in bc)


@pytest.fixture(scope="module")
def shell32(gpu_lib):
    w = make_workload("shell32")
    f = (w["rf"], w["thf"], w["phf"])
    ctx = _ctx(gpu_lib, f, SHELL_BC, u_lo=w["T_inner"])
    b = [_cuda(w[x]) for x in ("br", "bt", "bp")]
    return w, f, ctx, b


def test_F_shell32(shell32):
    w, f, ctx, b = shell32
    for u in (w["T"], w["T"] * (1.0 + 0.3 * np.random.default_rng(3).standard_normal(w["T"].shape))):
        got = _host(ctx.apply_F_nonlinear(_cuda(u), w["kappa0"], *b))
        ref = NL.F_nonlinear("spherical", *f, u, w["kappa0"], w["br"], w["bt"], w["bp"],
                             _obc(SHELL_BC), u_lo=w["T_inner"])
        assert relmax(got, ref) <= 1e-12


def test_F_negative_states_clip(shell32):
    w, f, ctx, b = shell32
    u = w["T"].copy()
    u[3:6, 10:20, 5:40] *= -0.5
    got = _host(ctx.apply_F_nonlinear(_cuda(u), w["kappa0"], *b))
    ref = NL.F_nonlinear("spherical", *f, u, w["kappa0"], w["br"], w["bt"], w["bp"],
                         _obc(SHELL_BC), u_lo=w["T_inner"])
    assert np.all(np.isfinite(got)) and relmax(got, ref) <= 1e-12


@pytest.mark.parametrize("shape", [(1, 4, 65), (5, 7, 9), (3, 13, 70), (6, 5, 130), (9, 9, 64)])
@pytest.mark.parametrize("bc", [(1, 0, 0, 0, 2, 2), (1, 1, 0, 0, 2, 2), (0, 0, 0, 0, 0, 0)])
def test_F_ragged_and_boundaries(gpu_lib, shape, bc):
    """Tiles with ragged theta / phi tails, tiles wider than the phi axis,
    one radial cell, Dirichlet on one or both radial sides, no periodic axis."""
    w = small_shell(shape, seed=6)
    f = (w["rf"], w["thf"], w["phf"])
    rng = np.random.default_rng(sum(shape))
    b = random_unit_vectors(shape, sum(shape))
    u = w["T"] * (1.0 + 0.2 * rng.random(shape))
    ctx = _ctx(gpu_lib, f, bc, u_lo=1.2e6, u_hi=0.7e6)
    got = _host(ctx.apply_F_nonlinear(_cuda(u), w["kappa0"], *[_cuda(x) for x in b]))
    ref = NL.F_nonlinear("spherical", *f, u, w["kappa0"], *b, _obc(bc), u_lo=1.2e6, u_hi=0.7e6)
    assert relmax(got, ref) <= 1e-12


def test_F_cartesian_periodic_box(gpu_lib):
    """Every axis periodic: the r-march wraps across chunks."""
    n, h = (8, 10, 12), (0.7, 1.1, 0.9)
    f = box_faces(*n, h=h)
    rng = np.random.default_rng(1)
    u = 1.0 + 0.2 * rng.random(n)
    b = random_unit_vectors(n, 11)
    bc = (2, 2, 2, 2, 2, 2)
    ctx = _ctx(gpu_lib, f, bc, coord=gpu_lib.CARTESIAN)
    got = _host(ctx.apply_F_nonlinear(_cuda(u), 0.8, *[_cuda(x) for x in b]))
    ref = NL.F_nonlinear("cartesian", *f, u, 0.8, *b, _obc(bc))
    assert relmax(got, ref) <= 1e-12


@pytest.mark.parametrize("ratio,s", [(50.0, 0), (20.0, 11), (3.0, 2)])
def test_step_shell32(shell32, ratio, s):
    w, f, ctx, b = shell32
    op0 = NL.operator_at("spherical", *f, w["T"], w["kappa0"], w["br"], w["bt"], w["bp"],
                         _obc(SHELL_BC), u_lo=w["T_inner"])
    dt = ratio * O.gershgorin_dt_euler(op0)
    u = _cuda(w["T"])
    used = ctx.rkl2_step_nonlinear(u, dt, w["kappa0"], *b, s=s)
    ref, s_ref = NL.rkl2_step_nonlinear("spherical", *f, w["T"], w["kappa0"], w["br"], w["bt"],
                                        w["bp"], dt, s if s else None, _obc(SHELL_BC),
                                        u_lo=w["T_inner"])
    got = _host(u)
    assert used == s_ref
    assert relmax(got, ref) <= 1e-12
    assert relmax(got - w["T"], ref - w["T"]) <= 1e-9
    # the context now holds the lagged operator at u^n
    assert ctx.dt_euler() == pytest.approx(O.gershgorin_dt_euler(op0), rel=1e-12)


def test_step_differs_from_lagged_step(shell32, gpu_lib):
    """Same dt and s: the lagged step (rkl2_step after set_spitzer at u^n)
    and the un-lagged one differ by the lagging error, not by rounding."""
    w, f, ctx, b = shell32
    ctx.set_spitzer(_cuda(w["T"]), w["kappa0"], *b)
    dt = 50.0 * ctx.dt_euler()
    u1, u2 = _cuda(w["T"]), _cuda(w["T"])
    s = ctx.rkl2_step_nonlinear(u1, dt, w["kappa0"], *b)
    ctx.set_spitzer(u2.clone(), w["kappa0"], *b)
    assert ctx.rkl2_step(u2, dt, s) == s
    d = relmax(_host(u1) - w["T"], _host(u2) - w["T"])
    assert d > 1e-4


def test_step_errors(shell32, gpu_lib):
    w, f, ctx, b = shell32
    T = w["T"].copy()
    T[4, 5, 6] = -1.0
    u = _cuda(T)
    with pytest.raises(gpu_lib.StsError):
        ctx.rkl2_step_nonlinear(u, 1.0, w["kappa0"], *b)
    assert np.array_equal(_host(u), T)  # rejected before any stage
    u = _cuda(w["T"])
    for args in ((1.0, w["kappa0"], 1), (-1.0, w["kappa0"], 0), (1.0, 0.0, 0)):
        with pytest.raises(gpu_lib.StsError):
            ctx.rkl2_step_nonlinear(u, args[0], args[1], *b, s=args[2])
    assert np.array_equal(_host(u), w["T"])
    with pytest.raises(gpu_lib.StsError):
        ctx.apply_F_nonlinear(u, w["kappa0"], *b, out=u)


# ----------------------------------------------------------------------------- full size
def _window(w, c, half, fields):
    """Sub-grid of half-width `half` around cell c: faces, the given fields,
    the oracle boundary conditions and c's position in the window.  Cut faces
    are zero-flux (their effect does not reach c within the stages run);
    a window reaching r = 1 keeps the Dirichlet inner boundary."""
    rf, thf, phf = w["rf"], w["thf"], w["phf"]
    n0, n1, n2 = len(rf) - 1, len(thf) - 1, len(phf) - 1
    i, j, k = c
    i0, i1 = max(0, i - half), min(n0, i + half + 1)
    j0, j1 = max(0, j - half), min(n1, j + half + 1)
    if 2 * half + 1 >= n2:
        ks, pf, kc, per = list(range(n2)), phf, k, True
    else:
        ks = [(k + d) % n2 for d in range(-half, half + 1)]
        pf = [phf[ks[0]]]
        for kk in ks:
            pf.append(pf[-1] + (phf[kk + 1] - phf[kk]))
        pf, kc, per = np.array(pf), half, False
    take = lambda a: a[i0:i1, j0:j1][:, :, ks]  # noqa: E731
    ph = O.PERIODIC if per else O.ZEROFLUX
    bc = (O.DIRICHLET if i0 == 0 else O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, ph, ph)
    return (rf[i0:i1 + 1], thf[j0:j1 + 1], pf), [take(x) for x in fields], bc, \
        (i - i0, j - j0, kc)


@pytest.fixture(scope="module")
def shell128(gpu_lib):
    w = make_workload("shell128")
    f = (w["rf"], w["thf"], w["phf"])
    ctx = _ctx(gpu_lib, f, SHELL_BC, u_lo=w["T_inner"])
    b = [_cuda(w[x]) for x in ("br", "bt", "bp")]
    return w, f, ctx, b


def _cells(shape, n, seed):
    rng = np.random.default_rng(seed)
    m0, m1, m2 = shape
    cells = [(0, 0, 0), (m0 - 1, m1 - 1, m2 - 1), (0, m1 // 2, m2 - 1), (m0 // 2, 0, 63),
             (m0 - 1, 3, 64), (7, 4, 0), (8, 3, 191)]
    return cells + [tuple(int(rng.integers(0, m)) for m in shape) for _ in range(n)]


def test_shell128_sampled_F(shell128):
    w, f, ctx, b = shell128
    F = _host(ctx.apply_F_nonlinear(_cuda(w["T"]), w["kappa0"], *b))
    got, ref = [], []
    for c in _cells(w["T"].shape, 30, 0):
        wf, (T, br, bt, bp), bc, cw = _window(w, c, 2, (w["T"], w["br"], w["bt"], w["bp"]))
        ref.append(NL.F_nonlinear("spherical", *wf, T, w["kappa0"], br, bt, bp, bc,
                                  u_lo=w["T_inner"])[cw])
        got.append(F[c])
    assert relmax(np.array(got), np.array(ref), scale=np.max(np.abs(F))) <= 1e-12


def test_shell128_sampled_step(shell128):
    w, f, ctx, b = shell128
    s = 8
    ctx.set_spitzer(_cuda(w["T"]), w["kappa0"], *b)
    dt = 15.0 * ctx.dt_euler()
    u = _cuda(w["T"])
    assert ctx.rkl2_step_nonlinear(u, dt, w["kappa0"], *b, s=s) == s
    got = _host(u)
    res = []
    for c in _cells(w["T"].shape, 8, 1):
        wf, (T, br, bt, bp), bc, cw = _window(w, c, s + 2, (w["T"], w["br"], w["bt"], w["bp"]))
        ref, _ = NL.rkl2_step_nonlinear("spherical", *wf, T, w["kappa0"], br, bt, bp, dt, s, bc,
                                        u_lo=w["T_inner"])
        res.append((got[c], ref[cw], w["T"][c]))
    g, r, t0 = (np.array(x) for x in zip(*res))
    assert relmax(g, r, scale=np.max(np.abs(w["T"]))) <= 1e-12
    assert relmax(g - t0, r - t0, scale=np.max(np.abs(got - w["T"]))) <= 1e-9


def test_shell128_step_conserves_energy(gpu_lib):
    """Zero-flux boundaries everywhere: sum V u is conserved by every stage."""
    w = make_workload("shell128")
    f = (w["rf"], w["thf"], w["phf"])
    ctx = _ctx(gpu_lib, f, (0, 0, 0, 0, 2, 2))
    b = [_cuda(w[x]) for x in ("br", "bt", "bp")]
    u = _cuda(w["T"])
    ctx.set_spitzer(u.clone(), w["kappa0"], *b)
    s = ctx.rkl2_step_nonlinear(u, 200.0 * ctx.dt_euler(), w["kappa0"], *b)
    assert s >= 28
    V = geo.geometry("spherical", *f)["V"]
    du = _host(u) - w["T"]
    assert abs(np.sum(V * du)) <= 1e-12 * np.sum(V * np.abs(du))
    assert np.max(np.abs(du)) > 1e-3 * np.max(w["T"])
