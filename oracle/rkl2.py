"""RKL2 super-time-stepping (oracle, test-only).

Follows Sec. 3: the stage recurrence of Fig. "rkl2", the coefficient block
that follows it, and the stage count of Eq. (rkl2_s).

Readings of garbled passages:
  * Fig. "rkl2" writes "M_u" in the first stage; it is M_0 = M u^n.
  * Its loop body mixes indices j and k for mu, nu; all are the stage index k.
  * Its last term "(b_k - 1) mu~_k dt M_0" is the gamma~ term of the RKL2
    scheme of the paper's reference [RKL2_2014] with index k-1:
    gamma~_k = -(1 - b_{k-1}) mu~_k.  The literal index gives an unstable
    scheme (|R| > 1 inside the interval); the closed-form test pins this.
  * Eq. (rkl2_s) prints s = 1/2 ceil(sqrt(9 + 16 dt/dt_E) - 1), which yields
    half-integers; the minimal stable stage count is
    s = ceil((sqrt(9 + 16 dt/dt_E) - 1) / 2), i.e. the least s with
    s^2 + s - 2 >= 4 dt/dt_E.
  * s is not forced odd (the paper finds that unnecessary); ``odd=True``
    rounds up to the next odd s as an option.
"""
from __future__ import annotations

import math

import numpy as np


def stage_count(dt_ratio: float, odd: bool = False) -> int:
    """Minimal stable s for dt = dt_ratio * dt_Euler (Eq. rkl2_s)."""
    if not (dt_ratio > 0 and math.isfinite(dt_ratio)):
        raise ValueError("dt / dt_Euler must be positive and finite")
    s = math.ceil((math.sqrt(9.0 + 16.0 * dt_ratio) - 1.0) / 2.0)
    s = max(s, 2)
    # guard against rounding at exact boundaries: smallest s with s^2+s-2 >= 4r
    while (s - 1) >= 2 and (s - 1) ** 2 + (s - 1) - 2 >= 4.0 * dt_ratio:
        s -= 1
    while s * s + s - 2 < 4.0 * dt_ratio:
        s += 1
    if odd and s % 2 == 0:
        s += 1
    return s


def coefficients(s: int) -> dict:
    """Per-stage coefficients for k = 1..s (index 0 unused), from the block
    after Fig. "rkl2":
      b_0 = b_1 = b_2 = 1/3,  b_k = (k^2 + k - 2) / (2 k (k+1))
      mu~_1 = 4 / (3 (s^2 + s - 2))
      mu_k = (2k-1)/k * b_k / b_{k-1},  nu_k = -(k-1)/k * b_k / b_{k-2}
      mu~_k = 4 (2k-1) / (k (s^2+s-2)) * b_k / b_{k-1}
      gamma~_k = -(1 - b_{k-1}) mu~_k   (reading, module doc)."""
    if s < 2:
        raise ValueError("RKL2 needs s >= 2")
    b = np.zeros(s + 1)
    for k in range(s + 1):
        b[k] = 1.0 / 3.0 if k <= 2 else (k * k + k - 2.0) / (2.0 * k * (k + 1.0))
    w1 = 4.0 / (s * s + s - 2.0)
    mu = np.zeros(s + 1)
    nu = np.zeros(s + 1)
    mut = np.zeros(s + 1)
    gt = np.zeros(s + 1)
    mut[1] = w1 / 3.0
    for k in range(2, s + 1):
        mu[k] = (2.0 * k - 1.0) / k * b[k] / b[k - 1]
        nu[k] = -(k - 1.0) / k * b[k] / b[k - 2]
        mut[k] = 4.0 * (2.0 * k - 1.0) / (k * (s * s + s - 2.0)) * b[k] / b[k - 1]
        gt[k] = -(1.0 - b[k - 1]) * mut[k]
    return dict(b=b, mu=mu, nu=nu, mut=mut, gt=gt, w1=w1)


def rkl2_step(F, u_n: np.ndarray, dt: float, s: int) -> np.ndarray:
    """One super-step of Fig. "rkl2":
        F0 = F(u^n);  u_1 = u^n + mu~_1 dt F0
        u_k = mu_k u_{k-1} + nu_k u_{k-2} + (1 - mu_k - nu_k) u^n
              + mu~_k dt F(u_{k-1}) + gamma~_k dt F0,   k = 2..s
        u^{n+1} = u_s.
    F is the (affine) operator; with a Dirichlet source, F(u) = M u + V^-1 g,
    which the recurrence handles unchanged (it only ever calls F)."""
    c = coefficients(s)
    u0 = np.asarray(u_n, dtype=np.float64)
    F0 = F(u0)
    u_km2 = u0
    u_km1 = u0 + c["mut"][1] * dt * F0
    for k in range(2, s + 1):
        u_k = (c["mu"][k] * u_km1 + c["nu"][k] * u_km2 + (1.0 - c["mu"][k] - c["nu"][k]) * u0
               + c["mut"][k] * dt * F(u_km1) + c["gt"][k] * dt * F0)
        u_km2, u_km1 = u_km1, u_k
    return u_km1


def amplification(z, s: int) -> np.ndarray:
    """The recurrence applied to the scalar test equation du/dt = lambda u
    with z = dt lambda: returns u_s / u^n (the amplification factor plotted in
    Fig. "ampfac")."""
    z = np.asarray(z, dtype=np.float64)
    return rkl2_step(lambda u: (z / 1.0) * u, np.ones_like(z), 1.0, s)


def euler_amplification(z):
    """Explicit Euler: 1 + z."""
    return 1.0 + np.asarray(z, dtype=np.float64)


def be_amplification(z):
    """Backward Euler: 1 / (1 - z)."""
    return 1.0 / (1.0 - np.asarray(z, dtype=np.float64))
