"""Conduction with the diffusivity taken from the current state, not lagged
(oracle, test-only).

PCG needs a linear operator, so for BE+PCG the temperature-dependent Spitzer
coefficient is frozen at the start of the step (Sec. 1, Sec. 2.4).  RKL2 only
ever evaluates F, so it can use the nonlinear operator itself (Sec. 2.4,
Sec. 3.1).  Here

    F_nl(u) = V^-1 ( S(kappa(u)) u + g(kappa(u)) ),

with S, g the 19-point energy-form operator of operator.py assembled from
D = kappa(u) b b^T (Eq. mhd:e1, blue box), and the RKL2 recurrence of
Fig. "rkl2" applied to F_nl unchanged: every stage evaluates F_nl at u_{k-1},
and F0 = F_nl(u^n).

Readings (the paper gives none of these):
  * kappa(u) = kappa0 max(u, 0)^{5/2}: a stage value may undershoot below
    zero; clipping keeps kappa real and >= 0, so the operator stays
    dissipative;
  * b is fixed over the step;
  * the stage count s (Eq. rkl2_s) uses dt_E of the operator at u^n, the
    lagged operator of the step's start;
  * no flux limiter: the paper names flux limiting without giving a form.

Pinned by tests/test_oracle_nonlinear.py: F_nl is homogeneous of degree 7/2
(the lagged F of degree 1); on a travelling-wave solution of the nonlinear
equation along an oblique b, F_nl(u) converges to du/dt at second order in
the mesh width; RKL2 steps of F_nl converge at second order in dt to an
independent ODE integration of du/dt = F_nl(u), where lagged coefficients
converge at first order.
"""
from __future__ import annotations

import numpy as np

from . import operator as O
from . import rkl2 as R2


def operator_at(coord, f0, f1, f2, u, kappa0, br, bt, bp, bc=O.SHELL_BC, u_lo=0.0, u_hi=0.0):
    """The operator with D = kappa(u) b b^T, kappa(u) = kappa0 max(u, 0)^{5/2}."""
    T = np.maximum(np.asarray(u, dtype=np.float64), 0.0)
    D = O.spitzer_tensor(T, kappa0, br, bt, bp)
    return O.assemble(coord, f0, f1, f2, D, bc, u_lo=u_lo, u_hi=u_hi)


def F_nonlinear(coord, f0, f1, f2, u, kappa0, br, bt, bp, bc=O.SHELL_BC, u_lo=0.0, u_hi=0.0):
    """F_nl(u) = V^-1 (S(kappa(u)) u + g(kappa(u)))."""
    op = operator_at(coord, f0, f1, f2, u, kappa0, br, bt, bp, bc, u_lo, u_hi)
    return O.apply_F(op, np.asarray(u, dtype=np.float64))


def rkl2_step_nonlinear(coord, f0, f1, f2, u_n, kappa0, br, bt, bp, dt, s=None,
                        bc=O.SHELL_BC, u_lo=0.0, u_hi=0.0):
    """One RKL2 super-step (Fig. "rkl2") of du/dt = F_nl(u).  s = None takes the
    minimal stable s (Eq. rkl2_s) for dt / dt_E, dt_E the Gershgorin limit of
    the operator at u^n.  Returns (u^{n+1}, s)."""
    if s is None:
        op_n = operator_at(coord, f0, f1, f2, u_n, kappa0, br, bt, bp, bc, u_lo, u_hi)
        s = R2.stage_count(dt / O.gershgorin_dt_euler(op_n))

    def F(v):
        return F_nonlinear(coord, f0, f1, f2, v, kappa0, br, bt, bp, bc, u_lo, u_hi)

    return R2.rkl2_step(F, u_n, dt, s), s
