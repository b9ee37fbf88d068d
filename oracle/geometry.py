"""Finite-volume geometry of a logically rectangular grid (oracle, test-only).

The paper discretises on a "logically rectangular non-uniform spherical grid"
(Sec. 4.2, Table tab:grid).  The oracle uses a cell-centred finite-volume
reading of it: exact cell volumes and face areas of spherical-coordinate cells,
centre-to-centre distances measured along the coordinate lines, and cell
centres at the arithmetic midpoints of the faces.  A uniform Cartesian box
(same formulas with unit metric) is provided for Fourier / polynomial tests.

Axis order everywhere is (0, 1, 2) = (r, theta, phi) or (x, y, z);
arrays are [n0][n1][n2] with axis 2 fastest.
"""
from __future__ import annotations

import numpy as np

SPHERICAL = "spherical"
CARTESIAN = "cartesian"


def centres(f: np.ndarray) -> np.ndarray:
    return 0.5 * (f[1:] + f[:-1])


def _centre_gaps(f: np.ndarray, periodic: bool) -> np.ndarray:
    """Distance from centre m to centre m+1 along an axis, for m = 0..n-1
    (the last entry wraps for a periodic axis, else it is unused and 0)."""
    c = centres(f)
    gap = np.zeros(len(c))
    gap[:-1] = c[1:] - c[:-1]
    if periodic:
        gap[-1] = c[0] + (f[-1] - f[0]) - c[-1]
    return gap


def geometry(coord: str, f0, f1, f2, periodic=(False, False, True)) -> dict:
    """Volumes V, +face areas A[a], centre distances across +faces dl[a], and
    the Dirichlet boundary-face area / centre-to-face distance on both axis-0
    sides.  Entries for faces that do not exist (last index of a non-periodic
    axis) are left as computed but are never used with a non-zero weight."""
    f0, f1, f2 = (np.asarray(f, dtype=np.float64) for f in (f0, f1, f2))
    n0, n1, n2 = len(f0) - 1, len(f1) - 1, len(f2) - 1
    d0 = np.diff(f0)
    d1 = np.diff(f1)
    d2 = np.diff(f2)
    c0, c1 = centres(f0), centres(f1)
    g0 = _centre_gaps(f0, periodic[0])
    g1 = _centre_gaps(f1, periodic[1])
    g2 = _centre_gaps(f2, periodic[2])
    shape = (n0, n1, n2)
    I = lambda a: a[:, None, None]  # noqa: E731
    J = lambda a: a[None, :, None]  # noqa: E731
    K = lambda a: a[None, None, :]  # noqa: E731
    out = {"shape": shape, "periodic": tuple(periodic), "coord": coord}
    if coord == SPHERICAL:
        # cell volume: integral of r^2 sin(theta) dr dtheta dphi
        vr = (f0[1:] ** 3 - f0[:-1] ** 3) / 3.0
        vt = np.cos(f1[:-1]) - np.cos(f1[1:])
        V = I(vr) * J(vt) * K(d2)
        # +r face of cell i sits at radius f0[i+1]
        A0 = I(f0[1:] ** 2) * J(vt) * K(d2)
        # +theta face of cell j sits at colatitude f1[j+1]
        hr2 = 0.5 * (f0[1:] ** 2 - f0[:-1] ** 2)
        A1 = I(hr2) * J(np.sin(f1[1:])) * K(d2)
        # +phi face: a meridional plane
        A2 = I(hr2) * J(d1) * K(np.ones(n2))
        # centre distances along coordinate lines
        L0 = I(g0) * J(np.ones(n1)) * K(np.ones(n2))
        L1 = I(c0) * J(g1) * K(np.ones(n2))
        L2 = I(c0) * J(np.sin(c1)) * K(g2)
        # Dirichlet faces on the two radial sides
        Ab_lo = (f0[0] ** 2) * vt[:, None] * d2[None, :]
        Ab_hi = (f0[-1] ** 2) * vt[:, None] * d2[None, :]
        db_lo = c0[0] - f0[0]
        db_hi = f0[-1] - c0[-1]
    elif coord == CARTESIAN:
        V = I(d0) * J(d1) * K(d2)
        A0 = I(np.ones(n0)) * J(d1) * K(d2)
        A1 = I(d0) * J(np.ones(n1)) * K(d2)
        A2 = I(d0) * J(d1) * K(np.ones(n2))
        L0 = I(g0) * J(np.ones(n1)) * K(np.ones(n2))
        L1 = I(np.ones(n0)) * J(g1) * K(np.ones(n2))
        L2 = I(np.ones(n0)) * J(np.ones(n1)) * K(g2)
        Ab_lo = d1[:, None] * d2[None, :]
        Ab_hi = Ab_lo.copy()
        db_lo = c0[0] - f0[0]
        db_hi = f0[-1] - c0[-1]
    else:
        raise ValueError(coord)
    bc = lambda a: np.broadcast_to(a, shape).copy()  # noqa: E731
    out.update(V=bc(V), A=[bc(A0), bc(A1), bc(A2)], dl=[bc(L0), bc(L1), bc(L2)],
               Ab=(Ab_lo, Ab_hi), db=(db_lo, db_hi))
    return out


def cartesian_position(coord: str, f0, f1, f2):
    """Cartesian coordinates (x, y, z) of cell centres (for analytic tests)."""
    c0, c1, c2 = (centres(np.asarray(f)) for f in (f0, f1, f2))
    a0, a1, a2 = np.meshgrid(c0, c1, c2, indexing="ij")
    if coord == CARTESIAN:
        return a0, a1, a2
    return (a0 * np.sin(a1) * np.cos(a2), a0 * np.sin(a1) * np.sin(a2), a0 * np.cos(a1))


def local_basis(coord: str, f0, f1, f2):
    """Unit vectors (e0, e1, e2) of the local basis at cell centres, as Cartesian
    triples, for converting a Cartesian vector to local components."""
    c0, c1, c2 = (centres(np.asarray(f)) for f in (f0, f1, f2))
    _, th, ph = np.meshgrid(c0, c1, c2, indexing="ij")
    if coord == CARTESIAN:
        one, zero = np.ones_like(th), np.zeros_like(th)
        return (one, zero, zero), (zero, one, zero), (zero, zero, one)
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    er = (st * cp, st * sp, ct)
    et = (ct * cp, ct * sp, -st)
    ep = (-sp, cp, np.zeros_like(th))
    return er, et, ep


__all__ = ["geometry", "centres", "cartesian_position", "local_basis", "SPHERICAL", "CARTESIAN"]
