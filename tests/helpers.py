"""Shared test plumbing: build the same seeded inputs for the oracle and for
the HIP library, and compare results."""
from __future__ import annotations

import numpy as np

from oracle import operator as O
from workloads import make_workload, shell_faces, temperature, dipole_bhat

ORACLE_BC = {0: O.ZEROFLUX, 1: O.DIRICHLET, 2: O.PERIODIC}


def oracle_spitzer(rf, thf, phf, T, br, bt, bp, kappa0, bc, u_lo=0.0, u_hi=0.0,
                   coord="spherical"):
    D = O.spitzer_tensor(T, kappa0, br, bt, bp)
    obc = tuple(ORACLE_BC[b] for b in bc)
    return O.assemble(coord, rf, thf, phf, D, obc, u_lo=u_lo, u_hi=u_hi)


def gpu_spitzer(sts, rf, thf, phf, T, br, bt, bp, kappa0, bc, u_lo=0.0, u_hi=0.0,
                coord=None):
    import torch
    coord = sts.SPHERICAL if coord is None else coord
    ctx = sts.Context(coord, rf, thf, phf, bc)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    if bc[0] == sts.BC_DIRICHLET:
        ctx.set_dirichlet(0, value=u_lo)
    if bc[1] == sts.BC_DIRICHLET:
        ctx.set_dirichlet(1, value=u_hi)
    ctx.set_spitzer(dev(T), kappa0, dev(br), dev(bt), dev(bp))
    return ctx


def small_shell(shape, seed=1):
    rf, thf, phf = shell_faces(*shape)
    T = temperature(rf, thf, phf, seed)
    br, bt, bp = dipole_bhat(rf, thf, phf)
    return dict(rf=rf, thf=thf, phf=phf, T=T, br=br, bt=bt, bp=bp, kappa0=1e-15,
                T_inner=1.5e6)


def relmax(a, b, scale=None):
    a = np.asarray(a)
    b = np.asarray(b)
    s = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def window_F(w, cells, half=2):
    """F(T) at the given cells, each computed by the oracle on a small window
    of the grid around the cell (exact: a row of F only involves cells within
    one cell, whose coefficients involve cells within two)."""
    rf, thf, phf = w["rf"], w["thf"], w["phf"]
    n0, n1, n2 = len(rf) - 1, len(thf) - 1, len(phf) - 1
    out = []
    for (i, j, k) in cells:
        i0, i1 = max(0, i - half), min(n0, i + half + 1)
        j0, j1 = max(0, j - half), min(n1, j + half + 1)
        ks = [(k + d) % n2 for d in range(-half, half + 1)]
        # unwrap phi faces of the window
        pf = [phf[ks[0]]]
        for kk in ks:
            pf.append(pf[-1] + (phf[kk + 1] - phf[kk]))
        pf = np.array(pf)
        sl = (slice(i0, i1), slice(j0, j1))
        take = lambda a: a[sl][:, :, ks]  # noqa: E731
        bc = [O.DIRICHLET if i0 == 0 else O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX, O.ZEROFLUX,
              O.ZEROFLUX, O.ZEROFLUX]
        D = O.spitzer_tensor(take(w["T"]), w["kappa0"], take(w["br"]), take(w["bt"]),
                             take(w["bp"]))
        op = O.assemble("spherical", rf[i0:i1 + 1], thf[j0:j1 + 1], pf, D, tuple(bc),
                        u_lo=w["T_inner"])
        F = O.apply_F(op, take(w["T"]))
        out.append(F[i - i0, j - j0, half])
    return np.array(out)


def window_op(w, cell, half, kind="spitzer", nu=1.0):
    """The oracle operator on the window of half-width `half` around `cell`
    (clipped at the r and theta walls, phi unwrapped), with the real boundary
    conditions where the window reaches the domain's boundary.  Returns
    (op, take, centre): take() cuts a full-grid field to the window; centre
    is the cell's index in it.  Rows of cells within `half` - 2 of the centre
    are exact rows of the full operator."""
    rf, thf, phf = w["rf"], w["thf"], w["phf"]
    n0, n1, n2 = len(rf) - 1, len(thf) - 1, len(phf) - 1
    i, j, k = cell
    i0, i1 = max(0, i - half), min(n0, i + half + 1)
    j0, j1 = max(0, j - half), min(n1, j + half + 1)
    ks = [(k + d) % n2 for d in range(-half, half + 1)]
    pf = [phf[ks[0]]]
    for kk in ks:
        pf.append(pf[-1] + (phf[kk + 1] - phf[kk]))
    pf = np.array(pf)
    sl = (slice(i0, i1), slice(j0, j1))
    take = lambda a: np.ascontiguousarray(a[sl][:, :, ks])  # noqa: E731
    bc = (O.DIRICHLET if i0 == 0 else O.ZEROFLUX,) + (O.ZEROFLUX,) * 5
    if kind == "spitzer":
        D = O.spitzer_tensor(take(w["T"]), w["kappa0"], take(w["br"]), take(w["bt"]),
                             take(w["bp"]))
        u_lo = w["T_inner"]
    else:
        D = O.isotropic_tensor((i1 - i0, j1 - j0, len(ks)), nu)
        u_lo = 0.0
    op = O.assemble("spherical", rf[i0:i1 + 1], thf[j0:j1 + 1], pf, D, bc, u_lo=u_lo)
    return op, take, (i - i0, j - j0, half)


__all__ = ["oracle_spitzer", "window_op", "gpu_spitzer", "small_shell", "relmax", "window_F", "make_workload"]


def resistivity_window(R, coord, faces, E, lo, hi, eta):
    """The oracle's resistive F on the cells [lo, hi) of a grid, taken as a
    grid of its own with every axis non-periodic.  An edge not on that
    window's boundary has the same four faces, face weights and edge mass as
    in the whole grid, so its F there equals the whole grid's.  E: the whole
    grid's edge values split by component ({'r', 't', 'p'} arrays, whose
    windows must not wrap).  Returns, per component, (F on the window, mask
    of its interior edges, the window's index slices into the whole grid's
    component array)."""
    (i0, j0, k0), (i1, j1, k1) = lo, hi
    f0, f1, f2 = faces
    g = R.edge_grid(coord, f0[i0:i1 + 1], f1[j0:j1 + 1], f2[k0:k1 + 1],
                    periodic=(False, False, False))
    sl = {"r": (slice(i0, i1), slice(j0, j1 + 1), slice(k0, k1 + 1)),
          "t": (slice(i0, i1 + 1), slice(j0, j1), slice(k0, k1 + 1)),
          "p": (slice(i0, i1 + 1), slice(j0, j1 + 1), slice(k0, k1))}
    Ew = {c: E[c][sl[c]] for c in "rtp"}
    for c in "rtp":
        assert Ew[c].shape == g.shapes[c], (c, Ew[c].shape, g.shapes[c])
    F = g.split(R.apply_F(g, R.EdgeGrid.join(Ew), eta))
    return {c: (F[c], ~g.fixed[c], sl[c]) for c in "rtp"}
