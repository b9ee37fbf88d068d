"""PC2: non-overlapping domain-decomposition ILU0 (oracle, test-only).

Sec. 2.3 and Appendix A.  The domain is cut into non-overlapping blocks (the
paper's per-MPI-rank subdomains; here blocks of b0 x b1 x b2 cells, the last
block along an axis may be smaller).  Inside each block the matrix A is
restricted to the block (couplings to other blocks are dropped) and given a
zero-fill incomplete LU factorisation A ~ L U: L unit lower triangular and U
upper triangular, both confined to the sparsity pattern P of A, determined by
the defining equations of zero fill

    (L U)_ij = A_ij   for every (i, j) in P.

Taking the rows in order, each equation has exactly one unknown:
    j <  i:  L_ij = (A_ij - sum_{m < j} L_im U_mj) / U_jj
    j >= i:  U_ij =  A_ij - sum_{m < i} L_im U_mj
(sums over the m with (i, m) and (m, j) in P, taken in ascending m).  The
preconditioner applies z = U^-1 (L^-1 r) per block, here by sparse triangular
solves of the block-diagonal L and U (a library primitive).

Readings:
  * P is the structural pattern of A: the 19-point stencil restricted to the
    block, including entries that happen to be numerically zero (e.g. next
    to a boundary).
  * rows are ordered lexicographically inside the block, axis 0 (r) slowest
    and axis 2 (phi) fastest, i.e. in memory order.  ILU0 depends on this.
  * the forward substitution of Appendix A subtracts the strictly lower
    entries only (its printed loop bound includes the diagonal; L has a unit
    diagonal, which the substitution does not subtract).
  * the periodic phi coupling is a boundary condition (MAS applies BCs
    matrix-free, Sec. 4.2), so it is never part of a block's matrix, even
    for a block that spans the whole phi range.
With 1x1x1 blocks every block matrix is its diagonal and PC2 equals PC1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

from .operator import OFFSETS


def _blocks(n, b):
    return [(s, min(s + b, n)) for s in range(0, n, b)]


def _shape_groups(shape, block):
    """Group block origins by block shape."""
    groups = {}
    for r0 in _blocks(shape[0], block[0]):
        for r1 in _blocks(shape[1], block[1]):
            for r2 in _blocks(shape[2], block[2]):
                bs = (r0[1] - r0[0], r1[1] - r1[0], r2[1] - r2[0])
                groups.setdefault(bs, []).append((r0[0], r1[0], r2[0]))
    return groups


def _pattern(bs):
    """For a block shape: per local row, dict col -> slot (structural pattern)."""
    b0, b1, b2 = bs
    n = b0 * b1 * b2
    rows = []
    for l in range(n):
        li, rem = divmod(l, b1 * b2)
        lj, lk = divmod(rem, b2)
        d = {}
        for s, (o0, o1, o2) in enumerate(OFFSETS):
            m0, m1, m2 = li + o0, lj + o1, lk + o2
            if 0 <= m0 < b0 and 0 <= m1 < b1 and 0 <= m2 < b2:
                d[(m0 * b1 + m1) * b2 + m2] = s
        rows.append(d)
    return rows


def _gather_block_values(F, origins, bs):
    """F[..., n0, n1, n2] -> [..., nblocks, nrows] (local lexicographic order)."""
    b0, b1, b2 = bs
    o = np.asarray(origins)
    l0, l1, l2 = np.meshgrid(np.arange(b0), np.arange(b1), np.arange(b2), indexing="ij")
    i0 = o[:, 0, None] + l0.ravel()[None, :]
    i1 = o[:, 1, None] + l1.ravel()[None, :]
    i2 = o[:, 2, None] + l2.ravel()[None, :]
    return F[..., i0, i1, i2], (i0, i1, i2)


def _factor_group(A, pat):
    """Zero-fill ILU of every block of one shape at once.  A[nb, nrows, 19]
    holds the block matrices in stencil slots; returns LU of the same layout
    (strictly lower slots: L, the rest: U; slot 0 is the diagonal)."""
    LU = np.zeros_like(A)
    for i, row in enumerate(pat):
        cols = sorted(row)
        for j in cols:
            s = row[j]
            acc = A[:, i, s].copy()
            for m in cols:
                if m >= min(i, j):
                    break
                t = pat[m].get(j)
                if t is not None:
                    acc -= LU[:, i, row[m]] * LU[:, m, t]
            LU[:, i, s] = acc / LU[:, j, 0] if j < i else acc
    return LU


def factor(A19: np.ndarray, block) -> dict:
    """Block ILU0 factors.  Returns, per block shape, LU[nblocks, nrows, 19]
    (values of L and U in stencil slots), the pattern, and the block-diagonal
    sparse L and U over all blocks of that shape."""
    shape = A19.shape[1:]
    groups = _shape_groups(shape, tuple(block))
    out = {"shape": shape, "groups": []}
    for bs, origins in groups.items():
        vals, idx = _gather_block_values(A19, origins, bs)  # [19, nb, nrows]
        A = np.ascontiguousarray(np.moveaxis(vals, 0, -1))  # [nb, nrows, 19]
        pat = _pattern(bs)
        LU = _factor_group(A, pat)
        if np.any(~(LU[:, :, 0] > 0)):
            raise FloatingPointError("ILU0 breakdown: non-positive pivot")
        L, U = _sparse_factors(LU, pat)
        out["groups"].append(dict(bs=bs, origins=origins, LU=LU, pattern=pat, idx=idx,
                                  L=L, U=U))
    return out


def _sparse_factors(LU, pat):
    """Block-diagonal CSR matrices of L (unit diagonal stored) and U; block b
    occupies rows and columns b*n .. b*n + n - 1."""
    nb, n = LU.shape[0], len(pat)
    base = (np.arange(nb) * n)[:, None]
    lr, lc, lv, ur, uc, uv = [], [], [], [], [], []
    for i, row in enumerate(pat):
        for j, s in row.items():
            if j < i:
                lr.append(base[:, 0] + i), lc.append(base[:, 0] + j), lv.append(LU[:, i, s])
            else:
                ur.append(base[:, 0] + i), uc.append(base[:, 0] + j), uv.append(LU[:, i, s])
        lr.append(base[:, 0] + i), lc.append(base[:, 0] + i), lv.append(np.ones(nb))
    N = nb * n
    L = sp.csr_matrix((np.concatenate(lv), (np.concatenate(lr), np.concatenate(lc))),
                      shape=(N, N))
    U = sp.csr_matrix((np.concatenate(uv), (np.concatenate(ur), np.concatenate(uc))),
                      shape=(N, N))
    return L, U


def apply(fac: dict, r: np.ndarray) -> np.ndarray:
    """z = U^-1 (L^-1 r) on every block (Appendix A: forward substitution with
    the unit lower triangle, then backward substitution with the upper one)."""
    z = np.zeros(fac["shape"])
    for grp in fac["groups"]:
        idx = grp["idx"]
        rb = r[idx[0], idx[1], idx[2]].ravel()  # block-major, local lexicographic
        y = spsolve_triangular(grp["L"], rb, lower=True, unit_diagonal=True)
        zb = spsolve_triangular(grp["U"], y, lower=False)
        z[idx[0], idx[1], idx[2]] = zb.reshape(idx[0].shape)
    return z


def lower_upper_dense(fac: dict, group: int = 0, block: int = 0):
    """Dense unit-lower L and upper U of one block (tests)."""
    grp = fac["groups"][group]
    LU, pat = grp["LU"][block], grp["pattern"]
    n = len(pat)
    L = np.eye(n)
    U = np.zeros((n, n))
    for i, d in enumerate(pat):
        for j, s in d.items():
            if j < i:
                L[i, j] = LU[i, s]
            else:
                U[i, j] = LU[i, s]
    return L, U


def block_dense_A(A19: np.ndarray, block, group_origin):
    """Dense restriction of A (19-slot form) to one block (tests)."""
    shape = A19.shape[1:]
    groups = _shape_groups(shape, tuple(block))
    for bs, origins in groups.items():
        if tuple(group_origin) in [tuple(o) for o in origins]:
            pat = _pattern(bs)
            n = len(pat)
            M = np.zeros((n, n))
            o0, o1, o2 = group_origin
            for l, d in enumerate(pat):
                li, rem = divmod(l, bs[1] * bs[2])
                lj, lk = divmod(rem, bs[2])
                for j, s in d.items():
                    M[l, j] = A19[s, o0 + li, o1 + lj, o2 + lk]
            return M, pat
    raise KeyError(group_origin)


__all__ = ["factor", "apply", "lower_upper_dense", "block_dense_A"]
