"""GPU parity: the HIP library against the FP64 CPU oracle on the same seeded
inputs.  Tolerances (FP64 on both sides, different summation order):
  * F(u), dt_Euler: 1e-12 relative to max |F| (per-element rounding ~1e-16
    of the largest stencil terms);
  * RKL2 step: 1e-12 relative in u, 1e-9 relative in the increment u^{n+1} - u^n;
  * BE+PCG: equal iteration counts (+-1), 1e-12 relative in u^{n+1}; iterates
    x_k at equal k: 1e-12 relative.
"""
import math

import numpy as np
import pytest

from helpers import gpu_spitzer, oracle_spitzer, relmax, small_shell, window_F
from oracle import operator as O
from oracle import pcg as opcg
from oracle.geometry import geometry
from oracle import rkl2 as orkl2
from workloads import make_workload, box_faces

pytestmark = pytest.mark.gpu

SHELL_BC = (1, 0, 0, 0, 2, 2)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _pair(sts, w, bc=SHELL_BC):
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], bc, u_lo=w["T_inner"])
    ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], bc, u_lo=w["T_inner"])
    return op, ctx


@pytest.fixture(scope="module")
def shell32(gpu_lib):
    w = make_workload("shell32")
    op, ctx = _pair(gpu_lib, w)
    return w, op, ctx


# ----------------------------------------------------------------------------- operator
def test_dt_euler(shell32):
    w, op, ctx = shell32
    assert ctx.dt_euler() == pytest.approx(O.gershgorin_dt_euler(op), rel=1e-12)


@pytest.mark.parametrize("field", ["T", "random"])
def test_apply_F(shell32, field):
    w, op, ctx = shell32
    u = w["T"] if field == "T" else np.random.default_rng(5).standard_normal(w["T"].shape) * 1e6
    F = _host(ctx.apply_F(_cuda(u)))
    assert relmax(F, O.apply_F(op, u)) <= 1e-12


@pytest.mark.parametrize("shape", [(5, 7, 9), (3, 3, 3), (1, 4, 65), (6, 5, 130)])
def test_apply_F_ragged_and_tiny(gpu_lib, shape):
    w = small_shell(shape, seed=4)
    op, ctx = _pair(gpu_lib, w)
    u = np.random.default_rng(2).standard_normal(shape)
    assert relmax(_host(ctx.apply_F(_cuda(u))), O.apply_F(op, u)) <= 1e-12


@pytest.mark.parametrize("bc", [(0, 0, 0, 0, 2, 2), (1, 1, 0, 0, 2, 2), (0, 0, 0, 0, 0, 0)])
def test_apply_F_boundaries(gpu_lib, bc):
    w = small_shell((6, 8, 10), seed=3)
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], bc, u_lo=1.2e6, u_hi=0.7e6)
    ctx = gpu_spitzer(gpu_lib, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], bc, u_lo=1.2e6, u_hi=0.7e6)
    assert relmax(_host(ctx.apply_F(_cuda(w["T"]))), O.apply_F(op, w["T"])) <= 1e-12
    assert ctx.dt_euler() == pytest.approx(O.gershgorin_dt_euler(op), rel=1e-12)


def test_apply_F_cartesian_periodic_box(gpu_lib):
    n, h = (8, 10, 12), (0.7, 1.1, 0.9)
    f = box_faces(*n, h=h)
    rng = np.random.default_rng(1)
    T = 1.0 + 0.2 * rng.random(n)
    b = rng.standard_normal((3,) + n)
    b /= np.sqrt((b * b).sum(0))
    bc = (2, 2, 2, 2, 2, 2)
    op = oracle_spitzer(*f, T, b[0], b[1], b[2], 1.0, bc, coord="cartesian")
    ctx = gpu_spitzer(gpu_lib, *f, T, b[0], b[1], b[2], 1.0, bc, coord=gpu_lib.CARTESIAN)
    u = rng.standard_normal(n)
    assert relmax(_host(ctx.apply_F(_cuda(u))), O.apply_F(op, u)) <= 1e-12


def test_conservation_zero_flux_gpu(gpu_lib):
    w = make_workload("shell32")
    ctx = gpu_spitzer(gpu_lib, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], (0, 0, 0, 0, 2, 2))
    F = _host(ctx.apply_F(_cuda(w["T"])))
    V = O.assemble("spherical", w["rf"], w["thf"], w["phf"],
                   O.isotropic_tensor(w["T"].shape, 1.0)).V
    assert abs(np.sum(V * F)) <= 1e-13 * np.sum(np.abs(V * F))


# ----------------------------------------------------------------------------- RKL2
@pytest.mark.parametrize("s", [0, 2, 3, 7])
def test_rkl2_step(shell32, s):
    w, op, ctx = shell32
    dtE = O.gershgorin_dt_euler(op)
    dt = 50.0 * dtE
    u = _cuda(w["T"])
    used = ctx.rkl2_step(u, dt, s)
    s_ref = orkl2.stage_count(50.0) if s <= 0 else s
    assert used == s_ref
    ref = orkl2.rkl2_step(lambda v: O.apply_F(op, v), w["T"], dt, s_ref)
    got = _host(u)
    assert relmax(got, ref) <= 1e-12
    assert relmax(got - w["T"], ref - w["T"]) <= 1e-9


def test_rkl2_fourier_mode_closed_form(gpu_lib):
    """rkl2_step on one cosine mode of a periodic box returns R_s(dt lambda) * mode."""
    from scipy.special import eval_legendre
    n, h = (8, 10, 12), (1.0, 0.8, 1.2)
    bvec = np.array([0.4, 0.5, -0.7])
    bvec /= np.linalg.norm(bvec)
    f = box_faces(*n, h=h)
    ones = np.ones(n)
    ctx = gpu_spitzer(gpu_lib, *f, 2.0 ** 0.4 * ones, bvec[0] * ones, bvec[1] * ones,
                      bvec[2] * ones, 1.0, (2,) * 6, coord=gpu_lib.CARTESIAN)  # kappa = 2
    theta = [2 * math.pi * m / nn for m, nn in zip((3, 4, 5), n)]
    idx = np.meshgrid(*[np.arange(nn) for nn in n], indexing="ij")
    mode = np.cos(sum(t * i for t, i in zip(theta, idx)))
    lam = -sum(4 * 2.0 * bvec[a] ** 2 * math.sin(theta[a] / 2) ** 2 / h[a] ** 2 for a in range(3))
    lam -= sum(2 * 2.0 * bvec[a] * bvec[b] * math.sin(theta[a]) * math.sin(theta[b]) / (h[a] * h[b])
               for a in range(3) for b in range(a + 1, 3))
    dt = 37.0 * ctx.dt_euler()
    u = _cuda(mode)
    s = ctx.rkl2_step(u, dt)
    bs = (s * s + s - 2.0) / (2.0 * s * (s + 1.0))
    R = 1 - bs + bs * eval_legendre(s, 1 + 4.0 / (s * s + s - 2.0) * dt * lam)
    assert relmax(_host(u), R * mode, scale=1.0) <= 1e-12


def test_rkl2_viscosity_three_components(gpu_lib):
    """Isotropic 7-point operator on 3 velocity components in one call."""
    import torch
    w = small_shell((10, 12, 20))
    v = np.random.default_rng(3).standard_normal((3,) + w["T"].shape)
    bc = SHELL_BC
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], bc)
    ctx.set_dirichlet(0, value=0.0)
    ctx.set_isotropic(0.7)
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], O.isotropic_tensor(w["T"].shape, 0.7),
                    tuple({0: O.ZEROFLUX, 1: O.DIRICHLET, 2: O.PERIODIC}[b] for b in bc))
    assert ctx.dt_euler() == pytest.approx(O.gershgorin_dt_euler(op), rel=1e-12)
    dt = 120 * O.gershgorin_dt_euler(op)
    u = torch.from_numpy(v.copy()).cuda()
    F = _host(ctx.apply_F(u))
    for m in range(3):
        assert relmax(F[m], O.apply_F(op, v[m])) <= 1e-12
    s = ctx.rkl2_step(u, dt)
    got = _host(u)
    for m in range(3):
        ref = orkl2.rkl2_step(lambda x: O.apply_F(op, x), v[m], dt, s)
        assert relmax(got[m], ref) <= 1e-12


# ----------------------------------------------------------------------------- BE + PCG
def _pcg_pair(op, ctx, u_n, dt, pc, block, rtol, maxit=10000):
    x = _cuda(u_n.copy())
    it, rel, st = ctx.be_pcg_solve(_cuda(u_n), x, dt, pc=pc, block=block, rtol=rtol, maxit=maxit,
                                   allow_not_converged=True)
    ref = opcg.be_pcg(op, u_n, dt, {0: "jacobi", 1: "ilu0"}[pc], rtol=rtol, maxit=maxit,
                      block=block)
    return _host(x), it, rel, st, ref


@pytest.mark.parametrize("pc,block", [(0, (8, 8, 8)), (1, (8, 8, 8)), (1, (5, 6, 7)),
                                      (1, (2, 8, 3))])
def test_be_pcg_shell32(shell32, pc, block):
    w, op, ctx = shell32
    dt = 50.0 * O.gershgorin_dt_euler(op)
    x, it, rel, st, ref = _pcg_pair(op, ctx, w["T"], dt, pc, block, 1e-9)
    assert st == 0 and ref.converged
    assert abs(it - ref.iters) <= 1
    assert rel <= 1e-9
    assert relmax(x, ref.x) <= 1e-12
    assert relmax(x - w["T"], ref.x - w["T"]) <= 1e-8


@pytest.mark.parametrize("pc", [0, 1])
def test_pcg_iterates_match_oracle(shell32, pc):
    w, op, ctx = shell32
    dt = 50.0 * O.gershgorin_dt_euler(op)
    ks = (1, 3, 10)
    ref = opcg.be_pcg(op, w["T"], dt, {0: "jacobi", 1: "ilu0"}[pc], rtol=1e-30, maxit=max(ks),
                      keep=set(ks))
    for k, xk in zip(sorted(ks), ref.iterates):
        x = _cuda(w["T"])
        it, rel, st = ctx.be_pcg_solve(_cuda(w["T"]), x, dt, pc=pc, rtol=1e-30, maxit=k,
                                       allow_not_converged=True)
        assert st == 1 and it == k  # STS_NOT_CONVERGED after exactly k iterations
        assert relmax(_host(x) - w["T"], xk - w["T"]) <= 1e-10
        assert relmax(_host(x), xk) <= 1e-12


def test_ilu_unit_blocks_equal_jacobi(shell32):
    w, op, ctx = shell32
    dt = 50.0 * O.gershgorin_dt_euler(op)
    xj = _cuda(w["T"])
    xi = _cuda(w["T"])
    itj, _, _ = ctx.be_pcg_solve(_cuda(w["T"]), xj, dt, pc=0, rtol=1e-9)
    iti, _, _ = ctx.be_pcg_solve(_cuda(w["T"]), xi, dt, pc=1, block=(1, 1, 1), rtol=1e-9)
    assert itj == iti
    assert relmax(_host(xi), _host(xj)) <= 1e-13


def test_be_residual_and_guess(shell32):
    w, op, ctx = shell32
    dt = 50.0 * O.gershgorin_dt_euler(op)
    x = _cuda(w["T"])
    it, rel, st = ctx.be_pcg_solve(_cuda(w["T"]), x, dt, rtol=1e-10)
    true = ctx.be_residual(_cuda(w["T"]), x, dt)
    assert true <= 2e-10
    # starting from the solution converges in 0 iterations
    it2, rel2, st2 = ctx.be_pcg_solve(_cuda(w["T"]), x, dt, rtol=1e-9)
    assert it2 == 0 and st2 == 0


def test_pcg_maxit_and_errors(shell32, gpu_lib):
    w, op, ctx = shell32
    dt = 50.0 * O.gershgorin_dt_euler(op)
    x = _cuda(w["T"])
    it, rel, st = ctx.be_pcg_solve(_cuda(w["T"]), x, dt, rtol=1e-14, maxit=2,
                                   allow_not_converged=True)
    assert st == gpu_lib.STS_NOT_CONVERGED and it == 2
    with pytest.raises(gpu_lib.StsError):
        ctx.be_pcg_solve(_cuda(w["T"]), x, -1.0)
    with pytest.raises(gpu_lib.StsError):
        ctx.be_pcg_solve(_cuda(w["T"]), x, dt, pc=1, block=(9, 8, 8))
    with pytest.raises(gpu_lib.StsError):
        ctx.rkl2_step(x, float("nan"))
    bad = w["T"].copy()
    bad[3, 4, 5] = -1.0
    with pytest.raises(gpu_lib.StsError):
        ctx2 = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
        ctx2.set_spitzer(_cuda(bad), 1e-15, _cuda(w["br"]), _cuda(w["bt"]), _cuda(w["bp"]))


@pytest.mark.parametrize("shape,pc,block", [((5, 7, 9), 0, (8, 8, 8)), ((5, 7, 9), 1, (3, 4, 5)),
                                            ((9, 10, 70), 1, (8, 8, 8))])
def test_be_pcg_ragged(gpu_lib, shape, pc, block):
    w = small_shell(shape, seed=6)
    op, ctx = _pair(gpu_lib, w)
    dt = 120 * O.gershgorin_dt_euler(op)
    x, it, rel, st, ref = _pcg_pair(op, ctx, w["T"], dt, pc, block, 1e-10)
    assert st == 0 and abs(it - ref.iters) <= 1
    assert relmax(x, ref.x) <= 1e-12


def test_be_pcg_viscosity_component(gpu_lib):
    w = small_shell((8, 10, 16))
    v = np.random.default_rng(8).standard_normal(w["T"].shape)
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    ctx.set_dirichlet(0, value=0.0)
    ctx.set_isotropic(1.0)
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], O.isotropic_tensor(v.shape, 1.0),
                    (O.DIRICHLET, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.PERIODIC, O.PERIODIC))
    dt = 300 * O.gershgorin_dt_euler(op)
    for pc in (0, 1):
        x, it, rel, st, ref = _pcg_pair(op, ctx, v, dt, pc, (4, 4, 4), 1e-10)
        assert st == 0 and abs(it - ref.iters) <= 1
        assert relmax(x, ref.x) <= 1e-11


# ----------------------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def shell128(gpu_lib):
    w = make_workload("shell128")
    op, ctx = _pair(gpu_lib, w)
    return w, op, ctx


def test_shell128_dt_and_F(shell128):
    w, op, ctx = shell128
    assert ctx.dt_euler() == pytest.approx(O.gershgorin_dt_euler(op), rel=1e-12)
    F = _host(ctx.apply_F(_cuda(w["T"])))
    assert relmax(F, O.apply_F(op, w["T"])) <= 1e-12


def test_shell128_rkl2(shell128):
    w, op, ctx = shell128
    dt = 200.0 * O.gershgorin_dt_euler(op)
    u = _cuda(w["T"])
    s = ctx.rkl2_step(u, dt)
    assert s == 28
    ref = orkl2.rkl2_step(lambda v: O.apply_F(op, v), w["T"], dt, s)
    got = _host(u)
    assert relmax(got, ref) <= 1e-12
    assert relmax(got - w["T"], ref - w["T"]) <= 1e-9


def test_shell128_be_jacobi(shell128):
    w, op, ctx = shell128
    dt = 200.0 * O.gershgorin_dt_euler(op)
    x, it, rel, st, ref = _pcg_pair(op, ctx, w["T"], dt, 0, (8, 8, 8), 1e-8)
    assert st == 0 and abs(it - ref.iters) <= 1
    assert relmax(x, ref.x) <= 1e-12


def test_shell128_be_ilu0(shell128):
    w, op, ctx = shell128
    dt = 200.0 * O.gershgorin_dt_euler(op)
    x, it, rel, st, ref = _pcg_pair(op, ctx, w["T"], dt, 1, (8, 8, 8), 1e-8)
    assert st == 0 and abs(it - ref.iters) <= 1
    assert relmax(x, ref.x) <= 1e-12


def test_shell256_sampled_F_and_conservation(gpu_lib):
    """Largest grid (256 x 256 x 512): F at sampled cells against the oracle
    evaluated cell by cell on small windows, plus conservation of sum V F
    under zero-flux boundaries (a property at any size)."""
    w = make_workload("shell256", with_velocity=False)
    ctx = gpu_spitzer(gpu_lib, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], SHELL_BC, u_lo=w["T_inner"])
    F = _host(ctx.apply_F(_cuda(w["T"])))
    rng = np.random.default_rng(0)
    n = w["T"].shape
    cells = [(0, 0, 0), (255, 255, 511), (0, 128, 511), (128, 0, 17), (255, 3, 0)]
    cells += [tuple(int(rng.integers(0, m)) for m in n) for _ in range(40)]
    ref = window_F(w, cells)
    got = np.array([F[c] for c in cells])
    assert relmax(got, ref, scale=np.max(np.abs(F))) <= 1e-12
    ctx.close()
    ctx0 = gpu_spitzer(gpu_lib, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                       w["kappa0"], (0, 0, 0, 0, 2, 2))
    F0 = _host(ctx0.apply_F(_cuda(w["T"])))
    G = geometry("spherical", w["rf"], w["thf"], w["phf"])
    assert abs(np.sum(G["V"] * F0)) <= 1e-12 * np.sum(np.abs(G["V"] * F0))
