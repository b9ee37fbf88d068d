"""Variants of the super-step discussed in Sec. 6 with Fig. "ampfac"
(oracle, test-only).

The paper tests three ways to make the super-step damp high modes and
remarks on a fourth:
  * sub-cycling RKL2: the step dt is taken as m RKL2 steps of dt/m (about
    ten sub-cycles reproduced the BE solution);
  * explicit Euler sub-steps for about a quarter of the step, then RKL2 for
    the remainder;
  * s rounded up to odd (the recommendation of the RKL2 authors quoted after
    Eq. rkl2_s);
  * RKL1 with more than the minimal number of stages, whose amplification
    factor then stays below 1 in magnitude at the highest mode.

RKL1 is the first-order Runge-Kutta-Legendre scheme of the paper's RKL
references (Meyer, Balsara & Aslam 2014), restated here:
    Y_0 = u^n,  Y_1 = Y_0 + w1 dt F(Y_0),  w1 = 2 / (s^2 + s)
    Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + mu~_j dt F(Y_{j-1}),   j = 2..s
    mu_j = (2j-1)/j,  nu_j = -(j-1)/j,  mu~_j = w1 (2j-1)/j,   u^{n+1} = Y_s.
On du/dt = lambda u it gives P_s(1 + w1 dt lambda) with P_s the Legendre
polynomial, stable for dt |lambda| <= s^2 + s.

Readings: the paper gives no step size for the Euler sub-steps; they are
taken as at most euler_cfl * dt_E (default 1/2: steps at the Euler limit
itself leave the highest mode undamped, |1 - 2| = 1).  The RKL2 remainder
uses the minimal stable s for its own length.

Pinned by tests/test_oracle_rkl_variants.py (Legendre closed form of RKL1,
first-order consistency, stability bounds, the paper's RKL1 remark,
composition of sub-cycles, Euler damping against BE).
"""
from __future__ import annotations

import math

import numpy as np

from . import rkl2 as R2


def rkl1_stage_count(dt_ratio: float, extra: int = 0) -> int:
    """Least s >= 1 with s^2 + s >= 2 dt/dt_E (|dt lambda| <= 2 dt/dt_E), plus extra."""
    if not (dt_ratio > 0 and math.isfinite(dt_ratio)):
        raise ValueError("dt / dt_Euler must be positive and finite")
    s = max(1, math.ceil((math.sqrt(1.0 + 8.0 * dt_ratio) - 1.0) / 2.0))
    while s > 1 and (s - 1) * s >= 2.0 * dt_ratio:
        s -= 1
    while s * s + s < 2.0 * dt_ratio:
        s += 1
    return s + int(extra)


def rkl1_coefficients(s: int) -> dict:
    if s < 1:
        raise ValueError("RKL1 needs s >= 1")
    w1 = 2.0 / (s * s + s)
    mu = np.zeros(s + 1)
    nu = np.zeros(s + 1)
    mut = np.zeros(s + 1)
    mut[1] = w1
    for j in range(2, s + 1):
        mu[j] = (2.0 * j - 1.0) / j
        nu[j] = -(j - 1.0) / j
        mut[j] = w1 * (2.0 * j - 1.0) / j
    return dict(mu=mu, nu=nu, mut=mut, w1=w1)


def rkl1_step(F, u_n, dt: float, s: int):
    c = rkl1_coefficients(s)
    y0 = np.asarray(u_n, dtype=np.float64)
    y_km1 = y0 + c["mut"][1] * dt * F(y0)
    y_km2 = y0
    for j in range(2, s + 1):
        y = c["mu"][j] * y_km1 + c["nu"][j] * y_km2 + c["mut"][j] * dt * F(y_km1)
        y_km2, y_km1 = y_km1, y
    return y_km1


def rkl1_amplification(z, s: int):
    z = np.asarray(z, dtype=np.float64)
    return rkl1_step(lambda u: z * u, np.ones_like(z), 1.0, s)


def euler_substeps(dt: float, dt_e: float, fraction: float, cfl: float = 0.5):
    """(n, h): n explicit Euler steps of h covering fraction * dt, h <= cfl * dt_E."""
    if fraction <= 0.0:
        return 0, 0.0
    span = fraction * dt
    n = max(1, math.ceil(span / (cfl * dt_e) - 1e-12))
    return n, span / n


def super_step(F, u_n, dt: float, dt_e: float, scheme: int = 2, extra: int = 0,
               odd: bool = False, nsub: int = 1, euler_fraction: float = 0.0,
               euler_cfl: float = 0.5):
    """The step with all variants combined, in this order: Euler sub-steps for
    euler_fraction * dt, then nsub sub-steps of the scheme (2: RKL2, 1: RKL1)
    over the rest, each with the minimal stable s for its length plus extra
    (rounded up to odd when odd).  Returns (u^{n+1}, number of F evaluations)."""
    u = np.asarray(u_n, dtype=np.float64)
    n_e, h = euler_substeps(dt, dt_e, euler_fraction, euler_cfl)
    napply = 0
    for _ in range(n_e):
        u = u + h * F(u)
        napply += 1
    rest = dt - n_e * h
    if rest <= 0.0:
        return u, napply
    ds = rest / nsub
    ratio = ds / dt_e
    for _ in range(nsub):
        if scheme == 2:
            s = R2.stage_count(ratio) + int(extra)
            if odd and s % 2 == 0:
                s += 1
            u = R2.rkl2_step(F, u, ds, s)
        elif scheme == 1:
            s = rkl1_stage_count(ratio, extra)
            if odd and s % 2 == 0:
                s += 1
            u = rkl1_step(F, u, ds, s)
        else:
            raise ValueError("scheme must be 1 or 2")
        napply += s
    return u, napply
