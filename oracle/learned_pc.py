"""Learned local SPD preconditioner factor G, M^-1 = G G^T (oracle, test-only).

The paper's PCG (Sec. 2.2, Fig. "pcg") applies z = P^-1 r with PC1 (point
Jacobi) or PC2 (block ILU0), Sec. 2.3 and Appendix A.  Beside them the
library offers a preconditioner whose inverse is given in factored form,
M^-1 = G G^T, with G predicted cell by cell by a small convolutional network
(not in the paper).  Definitions followed here:

  * Pattern.  Cells are ordered lexicographically, axis 0 (r) slowest and
    axis 2 (phi) fastest.  Row c of G holds the cell itself and its three
    -1 neighbours c - e_a (a = 0, 1, 2) that lie inside the grid without
    wrapping across the periodic phi seam.  Every such neighbour precedes c,
    so G is lower triangular.
  * Entries from the network outputs o = (o0, o1, o2, o3) of the cell and
    the diagonal of the backward-Euler matrix A:
        G[c, c]       = d_c exp(o0_c),      d_c = A_cc^(-1/2)
        G[c, c - e_a] = d_c o_(a+1),c
    The diagonal is positive, so G is nonsingular and M^-1 = G G^T is
    symmetric positive definite whatever the outputs; o = 0 gives
    G = D^(-1/2) and M^-1 = D^-1, point Jacobi (PC1).
  * Training objective for a probe vector z: L(z) = ||G^T A G z - z||^2 / N
    (N cells), a stochastic estimate of ||G^T A G - I||_F^2 / N, which is
    zero exactly when the preconditioned operator G^T A G is the identity.
    With w = G z, y = A w, r = G^T y - z, q = G r, s = A q:
        dL/dG[c, m] = 2 (y_c r_m + s_c z_m) / N   for (c, m) in the pattern.

Pinned by tests/test_oracle_learned_pc.py: dense G built entry by entry
(lower triangular, positive diagonal, G G^T symmetric positive definite by
dense eigenvalues), the stencil applications against dense products, o = 0
against point Jacobi, the gradient against central finite differences of L,
and PCG with this preconditioner against a dense solve.
"""
from __future__ import annotations

import numpy as np

AXES = (0, 1, 2)


def has_lower(shape):
    """Boolean masks m_a[c]: c - e_a exists inside the grid without wrap."""
    masks = []
    for a in AXES:
        m = np.ones(shape, dtype=bool)
        idx = [slice(None)] * 3
        idx[a] = 0
        m[tuple(idx)] = False
        masks.append(m)
    return masks


def _back(x, a):
    """x at c - e_a (zero where it does not exist)."""
    out = np.zeros_like(x)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    src[a] = slice(0, -1)
    dst[a] = slice(1, None)
    out[tuple(dst)] = x[tuple(src)]
    return out


def _fwd(x, a):
    """x at c + e_a (zero where it does not exist)."""
    out = np.zeros_like(x)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    src[a] = slice(1, None)
    dst[a] = slice(0, -1)
    out[tuple(dst)] = x[tuple(src)]
    return out


def factor_entries(o, diagA):
    """G's entries from the outputs o[4, n0, n1, n2] and diag(A):
    g[0] = G[c, c], g[1 + a] = G[c, c - e_a] (zero where absent)."""
    o = np.asarray(o, np.float64)
    d = 1.0 / np.sqrt(np.asarray(diagA, np.float64))
    g = np.empty_like(o)
    g[0] = d * np.exp(o[0])
    for a, m in zip(AXES, has_lower(d.shape)):
        g[1 + a] = np.where(m, d * o[1 + a], 0.0)
    return g


def apply_G(g, x):
    """(G x)_c = G[c, c] x_c + sum_a G[c, c - e_a] x_(c - e_a)."""
    y = g[0] * x
    for a in AXES:
        y = y + g[1 + a] * _back(x, a)
    return y


def apply_GT(g, x):
    """(G^T x)_c = G[c, c] x_c + sum_a G[c + e_a, c] x_(c + e_a)."""
    y = g[0] * x
    for a in AXES:
        y = y + _fwd(g[1 + a] * x, a)
    return y


def apply_Minv(g, r):
    """z = M^-1 r = G (G^T r)."""
    return apply_G(g, apply_GT(g, r))


def dense_G(g):
    """G as a dense matrix, entry by entry (tests, tiny grids)."""
    shape = g.shape[1:]
    n = int(np.prod(shape))
    G = np.zeros((n, n))
    lin = lambda i, j, k: (i * shape[1] + j) * shape[2] + k  # noqa: E731
    for i in range(shape[0]):
        for j in range(shape[1]):
            for k in range(shape[2]):
                c = lin(i, j, k)
                G[c, c] = g[0, i, j, k]
                if i > 0:
                    G[c, lin(i - 1, j, k)] = g[1, i, j, k]
                if j > 0:
                    G[c, lin(i, j - 1, k)] = g[2, i, j, k]
                if k > 0:
                    G[c, lin(i, j, k - 1)] = g[3, i, j, k]
    return G


def loss_and_grad(g, matvec, z):
    """L = ||G^T A G z - z||^2 / N and dL/dg (same layout as g; zero where
    an entry is absent), for A given by matvec."""
    n = z.size
    w = apply_G(g, z)
    y = matvec(w)
    r = apply_GT(g, y) - z
    s = matvec(apply_G(g, r))
    L = float(np.vdot(r, r)) / n
    dg = np.empty_like(g)
    dg[0] = 2.0 * (y * r + s * z) / n
    for a, m in zip(AXES, has_lower(z.shape)):
        dg[1 + a] = np.where(m, 2.0 * (y * _back(r, a) + s * _back(z, a)) / n, 0.0)
    return L, dg


def grad_outputs(dg, g, diagA):
    """dL/do from dL/dg: G[c, c] = d exp(o0) gives dg0 * G[c, c]; the
    off-diagonal entries are d o_(a+1), giving dg_(a+1) * d."""
    d = 1.0 / np.sqrt(np.asarray(diagA, np.float64))
    do = np.empty_like(dg)
    do[0] = dg[0] * g[0]
    for a, m in zip(AXES, has_lower(d.shape)):
        do[1 + a] = np.where(m, dg[1 + a] * d, 0.0)
    return do


def precond(g):
    """PCG preconditioner callable z = M^-1 r (for oracle.pcg.pcg)."""
    return lambda r: apply_Minv(g, r)


def be_pcg_factor(op, u_n, dt, g, rtol=1e-8, maxit=10000, x0=None, keep=()):
    """One backward-Euler step solved by PCG with M^-1 = G G^T."""
    from . import operator as O
    from .pcg import pcg
    A19, b = O.be_system(op, u_n, dt)
    return pcg(lambda v: O.apply19(A19, v), b, u_n if x0 is None else x0, precond(g), rtol,
               maxit, keep)


__all__ = ["factor_entries", "apply_G", "apply_GT", "apply_Minv", "dense_G", "loss_and_grad",
           "grad_outputs", "precond", "be_pcg_factor", "has_lower"]
