"""Pins for the un-lagged conduction operator and its RKL2 step
(oracle/nonlinear.py).

  * F_nl is homogeneous of degree 7/2 in (u, boundary values), because
    kappa ~ u^{5/2}; the lagged F is of degree 1.
  * On a travelling-wave solution of du/dt = div(kappa0 u^{5/2} b b.grad u)
    along an oblique constant b, F_nl(u) converges to the exact du/dt at
    second order in the mesh width (every face and edge term contributes).
  * RKL2 steps of F_nl converge to an independent adaptive ODE integration of
    du/dt = F_nl(u) at second order in dt; freezing kappa at the start of each
    step (the lagged operator) converges at first order only.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import geometry as geo
from oracle import nonlinear as NL
from oracle import operator as O
from oracle import rkl2 as R2
from workloads import dipole_bhat, shell_faces, temperature

ZF, DI = O.ZEROFLUX, O.DIRICHLET


def test_homogeneity_degree_seven_halves():
    rf, thf, phf = shell_faces(4, 5, 6)
    T = temperature(rf, thf, phf, 7) / 1e6
    br, bt, bp = dipole_bhat(rf, thf, phf)
    u_lo = 1.3
    lam = 1.7
    F1 = NL.F_nonlinear("spherical", rf, thf, phf, T, 0.2, br, bt, bp, u_lo=u_lo)
    F2 = NL.F_nonlinear("spherical", rf, thf, phf, lam * T, 0.2, br, bt, bp, u_lo=lam * u_lo)
    assert np.max(np.abs(F2 - lam ** 3.5 * F1)) <= 1e-12 * np.max(np.abs(F2))
    # the lagged operator (kappa frozen at T) is affine of degree 1
    op = NL.operator_at("spherical", rf, thf, phf, T, 0.2, br, bt, bp, u_lo=u_lo)
    opl = NL.operator_at("spherical", rf, thf, phf, T, 0.2, br, bt, bp, u_lo=lam * u_lo)
    assert np.allclose(O.apply_F(opl, lam * T), lam * O.apply_F(op, T), rtol=1e-12, atol=0)
    assert np.max(np.abs(F2 - lam * F1)) > 0.5 * np.max(np.abs(F2))


def test_negative_states_give_zero_diffusivity():
    """kappa(u) = kappa0 max(u, 0)^{5/2}: F_nl stays finite where u < 0 and
    equals the operator assembled with zero diffusivity in those cells."""
    rf, thf, phf = shell_faces(4, 5, 6)
    T = temperature(rf, thf, phf, 2) / 1e6
    T[1, 2, :3] = -0.4
    br, bt, bp = dipole_bhat(rf, thf, phf)
    F = NL.F_nonlinear("spherical", rf, thf, phf, T, 0.2, br, bt, bp, u_lo=1.0)
    kap = 0.2 * np.where(T > 0, T, 0.0) ** 2.5
    D = {(a, c): kap * x * y for a, x in enumerate((br, bt, bp))
         for c, y in enumerate((br, bt, bp)) if c >= a}
    ref = O.apply_F(O.assemble("spherical", rf, thf, phf, D, O.SHELL_BC, u_lo=1.0), T)
    assert np.all(np.isfinite(F)) and np.array_equal(F, ref)


B_OBLIQUE = np.array([1.0, 2.0, 2.0]) / 3.0
NE, KAPPA0, WAVE_C, XI0 = 2.5, 0.3, 1.0, 2.5


def _wave(x, t):
    """u = (n c xi / kappa0)^{1/n}, xi = xi0 + c t - b.x: an exact solution of
    du/dt = d/ds (kappa0 u^n du/ds), s = b.x, with n = 5/2 (the flux
    kappa0 u^n du/ds equals -c u)."""
    xi = XI0 + WAVE_C * t - sum(B_OBLIQUE[a] * x[a] for a in range(3))
    u = (NE * WAVE_C * xi / KAPPA0) ** (1.0 / NE)
    ut = (WAVE_C ** 2 / KAPPA0) * (NE * WAVE_C * xi / KAPPA0) ** (1.0 / NE - 1.0)
    return u, ut


def _wave_error(n):
    f = [np.linspace(0.0, 1.0, n + 1)] * 3
    x = np.meshgrid(*[geo.centres(ff) for ff in f], indexing="ij")
    u, ut = _wave(x, 0.0)
    b = [np.full(u.shape, B_OBLIQUE[a]) for a in range(3)]
    F = NL.F_nonlinear("cartesian", *f, u, KAPPA0, *b, bc=(ZF,) * 6)
    t = n // 4  # the same physical interior region at every n
    return np.max(np.abs(F - ut)[t:-t, t:-t, t:-t]) / np.max(np.abs(ut))


def test_travelling_wave_second_order_in_space():
    errs = [_wave_error(n) for n in (8, 16, 32)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-4 and min(rates) > 1.85, (errs, rates)


def _small_problem():
    f = (np.linspace(0.0, 1.0, 9), np.linspace(0.0, 0.8, 7), np.linspace(0.0, 0.6, 6))
    x = np.meshgrid(*[geo.centres(ff) for ff in f], indexing="ij")
    u0 = 1.0 + 0.15 * np.sin(2.0 * x[0] + 1.0) * np.cos(3.0 * x[1]) + 0.1 * x[2]
    b = [np.full(u0.shape, B_OBLIQUE[a]) for a in range(3)]
    bc = (DI, ZF, ZF, ZF, ZF, ZF)
    return f, u0, b, bc


def test_rkl2_nonlinear_second_order_in_time():
    f, u0, b, bc = _small_problem()
    kw = dict(bc=bc, u_lo=1.2)

    def F(v):
        return NL.F_nonlinear("cartesian", *f, v, 0.01, *b, **kw)

    dte = O.gershgorin_dt_euler(NL.operator_at("cartesian", *f, u0, 0.01, *b, **kw))
    T_end = 16.0 * dte
    ref = solve_ivp(lambda t, y: F(y.reshape(u0.shape)).ravel(), (0.0, T_end), u0.ravel(),
                    method="DOP853", rtol=1e-12, atol=1e-14).y[:, -1].reshape(u0.shape)

    def run(nstep, lagged):
        u = u0.copy()
        for _ in range(nstep):
            if lagged:
                op = NL.operator_at("cartesian", *f, u, 0.01, *b, **kw)
                u = R2.rkl2_step(lambda v: O.apply_F(op, v), u, T_end / nstep, 12)
            else:
                u, s = NL.rkl2_step_nonlinear("cartesian", *f, u, 0.01, *b, T_end / nstep, 12,
                                              **kw)
                assert s == 12
        return np.max(np.abs(u - ref))

    e_nl = [run(m, False) for m in (4, 8, 16)]
    e_lag = [run(m, True) for m in (4, 8, 16)]
    r_nl = [e_nl[i] / e_nl[i + 1] for i in range(2)]
    r_lag = [e_lag[i] / e_lag[i + 1] for i in range(2)]
    assert all(3.2 < r < 5.0 for r in r_nl), (e_nl, r_nl)
    assert all(1.5 < r < 2.6 for r in r_lag), (e_lag, r_lag)
    assert e_nl[-1] < 0.2 * e_lag[-1]


def test_default_stage_count_from_step_start_operator():
    rf, thf, phf = shell_faces(4, 5, 6)
    T = temperature(rf, thf, phf, 1) / 1e6
    br, bt, bp = dipole_bhat(rf, thf, phf)
    op = NL.operator_at("spherical", rf, thf, phf, T, 0.2, br, bt, bp, u_lo=1.0)
    dte = O.gershgorin_dt_euler(op)
    _, s = NL.rkl2_step_nonlinear("spherical", rf, thf, phf, T, 0.2, br, bt, bp, 37.0 * dte,
                                  u_lo=1.0)
    assert s == R2.stage_count(37.0)
