"""Backward Euler solved by preconditioned conjugate gradients (oracle).

Backward Euler: Eqs. (BE), (BE_lin), (BE_linsolve) of Sec. 2.1, written in
the symmetric form A u^{n+1} = b, A = V - dt S, b = V u^n + dt g (see
operator.be_system for the sign reading).

PCG: Fig. "pcg" of Sec. 2.2 with
  x_0 = u^n (or a caller-supplied guess), r_0 = b - A x_0, z_0 = P^-1 r_0,
  p_0 = z_0, r_r = r_0 . z_0, then per iteration
  y = A p; alpha = r_r / (p . y); x += alpha p; r -= alpha y; z = P^-1 r;
  r_old = r_r; r_r = r . z; convergence check; beta = r_r / r_old;
  p = z + beta p.
Readings:
  * the figure's last line "p_{k+1} = beta_k p_k + z_k" is a typo for
    z_{k+1};
  * the convergence check (the paper leaves the criterion open, citing
    [PCGstopcrit]) is ||r_k||_2 <= rtol ||b||_2 on the recursively updated
    residual, independent of the preconditioner, so every preconditioner and
    initial guess is judged at the same residual tolerance.
Preconditioners (Sec. 2.3, Appendix A): PC1 point-Jacobi z_i = r_i / A_ii;
PC2 non-overlapping block ILU0 (module ilu0).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .operator import apply19


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool
    history: list  # ||r_k|| / ||b|| per iteration (k = 0..iters)
    iterates: list  # x_k for k in keep


def pcg(matvec, b, x0, precond, rtol: float, maxit: int, keep=()):
    """Fig. "pcg" with the stopping reading of the module doc.  `keep` is a
    set of iteration indices whose iterates x_k are returned (tests)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.sqrt(np.vdot(b, b)))
    r = b - matvec(x)
    z = precond(r)
    p = z.copy()
    rr = float(np.vdot(r, z))
    rel = float(np.sqrt(np.vdot(r, r))) / bnorm if bnorm > 0 else 0.0
    hist = [rel]
    kept = []
    if 0 in keep:
        kept.append(x.copy())
    if rel <= rtol:
        return PCGResult(x, 0, rel, True, hist, kept)
    for k in range(maxit):
        y = matvec(p)
        py = float(np.vdot(p, y))
        if not py > 0.0:
            raise FloatingPointError("PCG breakdown: p . A p <= 0")
        alpha = rr / py
        x = x + alpha * p
        r = r - alpha * y
        z = precond(r)
        r_old = rr
        rr = float(np.vdot(r, z))
        rel = float(np.sqrt(np.vdot(r, r))) / bnorm
        hist.append(rel)
        if (k + 1) in keep:
            kept.append(x.copy())
        if rel <= rtol:
            return PCGResult(x, k + 1, rel, True, hist, kept)
        beta = rr / r_old
        p = z + beta * p
    return PCGResult(x, maxit, rel, False, hist, kept)


def jacobi(A19):
    """PC1 (Appendix A): P_ii = A_ii; z_i = r_i / P_ii."""
    d = A19[0].copy()
    return lambda r: r / d


def be_pcg(op, u_n, dt, precond="jacobi", rtol=1e-8, maxit=10000, x0=None, block=(8, 8, 8),
           keep=()):
    """One backward-Euler step solved with PCG; returns PCGResult."""
    from . import operator as O
    from . import ilu0
    A19, b = O.be_system(op, u_n, dt)
    if precond == "jacobi":
        P = jacobi(A19)
    elif precond == "ilu0":
        fac = ilu0.factor(A19, block)
        P = lambda r: ilu0.apply(fac, r)  # noqa: E731
    elif precond == "none":
        P = lambda r: r.copy()  # noqa: E731
    else:
        raise ValueError(precond)
    return pcg(lambda v: apply19(A19, v), b, u_n if x0 is None else x0, P, rtol, maxit, keep)
