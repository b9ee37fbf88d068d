"""PC2: non-overlapping domain-decomposition ILU0 (oracle, test-only).

Sec. 2.3 and Appendix A.  The domain is cut into non-overlapping blocks (the
paper's per-MPI-rank subdomains; here blocks of b0 x b1 x b2 cells, the last
block along an axis may be smaller).  Inside each block the matrix A is
restricted to the block (couplings to other blocks are dropped) and factored
by the zero-fill IKJ incomplete LU of Appendix A:

    for i = 2..N:  for k < i with LU_ik != 0:
        LU_ik = LU_ik / LU_kk
        for j > k with LU_ij != 0:  LU_ij = LU_ij - LU_ik LU_kj

and applied by the forward / backward substitution of Appendix A.

Readings:
  * "LU_ij != 0" is the structural pattern of A: the 19-point stencil
    restricted to the block, including entries that happen to be numerically
    zero (e.g. next to a boundary); an update LU_ij -= LU_ik LU_kj is applied
    when (i, j) and (k, j) are both in that pattern.
  * rows are ordered lexicographically inside the block, axis 0 (r) slowest
    and axis 2 (phi) fastest, i.e. in memory order.  ILU0 depends on this.
  * the periodic phi coupling is a boundary condition (MAS applies BCs
    matrix-free, Sec. 4.2), so it is never part of a block's matrix, even
    for a block that spans the whole phi range.
With 1x1x1 blocks every block matrix is its diagonal and PC2 equals PC1.
"""
from __future__ import annotations

import numpy as np

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


def factor(A19: np.ndarray, block) -> dict:
    """Block ILU0 factors.  Returns, per block shape, LU[nblocks, nrows, 19]
    (values of the combined LU matrix in stencil slots) and the pattern."""
    shape = A19.shape[1:]
    groups = _shape_groups(shape, tuple(block))
    out = {"shape": shape, "groups": []}
    for bs, origins in groups.items():
        vals, idx = _gather_block_values(A19, origins, bs)  # [19, nb, nrows]
        LU = np.ascontiguousarray(np.moveaxis(vals, 0, -1))  # [nb, nrows, 19]
        pat = _pattern(bs)
        # zero entries outside the block pattern (cross-block couplings dropped)
        for l, d in enumerate(pat):
            keep = np.zeros(19, dtype=bool)
            keep[list(d.values())] = True
            LU[:, l, ~keep] = 0.0
        n = len(pat)
        for i in range(1, n):
            row = pat[i]
            cols = sorted(row)
            for k in cols:
                if k >= i:
                    break
                sik = row[k]
                LU[:, i, sik] = LU[:, i, sik] / LU[:, k, 0]
                rowk = pat[k]
                for j in cols:
                    if j <= k:
                        continue
                    if j in rowk:
                        LU[:, i, row[j]] -= LU[:, i, sik] * LU[:, k, rowk[j]]
        if np.any(~(LU[:, :, 0] > 0)):
            raise FloatingPointError("ILU0 breakdown: non-positive pivot")
        out["groups"].append(dict(bs=bs, origins=origins, LU=LU, pattern=pat, idx=idx))
    return out


def apply(fac: dict, r: np.ndarray) -> np.ndarray:
    """z = (LU)^-1 r per block by the forward / backward substitution of
    Appendix A (unit lower triangle, then the upper triangle with its
    diagonal)."""
    z = np.zeros(fac["shape"])
    for grp in fac["groups"]:
        LU, pat, idx = grp["LU"], grp["pattern"], grp["idx"]
        rb = r[idx[0], idx[1], idx[2]]  # [nb, nrows]
        n = len(pat)
        zs = np.zeros_like(rb)
        for i in range(n):
            acc = rb[:, i].copy()
            for j, s in pat[i].items():
                if j < i:
                    acc -= LU[:, i, s] * zs[:, j]
            zs[:, i] = acc
        zz = np.zeros_like(rb)
        for i in range(n - 1, -1, -1):
            acc = zs[:, i].copy()
            for j, s in pat[i].items():
                if j > i:
                    acc -= LU[:, i, s] * zz[:, j]
            zz[:, i] = acc / LU[:, i, 0]
        z[idx[0], idx[1], idx[2]] = zz
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
