"""Resistive diffusion of the vector potential (oracle, test-only).

The induction equation carries the parabolic term -(c^2 eta / 4 pi) curl curl A
(Eq. mhd:a, boxed); MAS advances it by BE + PCG with the diagonal
preconditioner PC1 (Sec. 4.2) and keeps every vector component staggered so
that div B = 0 holds exactly.  eta below stands for the whole constant
c^2 eta / 4 pi.

Discretisation reading (the paper names the staggering, not the scheme):
  * unknowns are the line integrals E = A . dl along the cell edges of the
    grid: E_r on r-edges at (r_c(i), th_f(j), ph_f(k)), shape [n0][n1+1][n2];
    E_t on theta-edges at (r_f(i), th_c(j), ph_f(k)), shape [n0+1][n1][n2];
    E_p on phi-edges at (r_f(i), th_f(j), ph_c(k)), shape [n0+1][n1+1][n2]
    (phi periodic: ph_f(n2) is ph_f(0));
  * face fluxes by Stokes' theorem, Phi = C E with C the signed edge-face
    incidence (normals +r, +theta, +phi, boundaries traversed by the right-
    hand rule), B_f = Phi_f / S_f; the fluxes leaving any cell sum to zero
    identically (div B = 0);
  * energy W = 1/2 sum_f w_f Phi_f^2 with w_f = l*_f / S_f (S_f: face area,
    l*_f: distance between the centres of the two cells the face separates),
    edge mass H_e = S*_e / L_e (L_e: edge length, S*_e: area of the dual
    face through the edge, spanned by the centres of the four cells around
    it), both exact for spherical cells;
  * F(E) = -eta H^-1 dW/dE = -eta H^-1 C^T diag(w) C E on interior edges;
    edges lying in the r and theta boundary surfaces hold their values
    (tangential E given) and F = 0 there; faces all of whose edges are fixed
    carry no unknown and are left out;
  * BE (Eqs. BE, BE_lin): (H + dt eta C^T W C) E^{n+1} = H E^n on interior
    edges, the fixed edges' terms moved to the right-hand side; solved by the
    PCG of pcg.py with PC1 from x0 = E^n.
The same formulas with unit metric give a Cartesian box (every axis may be
periodic; then no edge is fixed).

Pinned by tests/test_oracle_resistivity.py: curl of a discrete gradient is
zero (F vanishes on it), div B = 0 cell by cell, H F is symmetric and
negative semi-definite, the Fourier symbol of a divergence-free mode on a
periodic box, convergence to -curl curl A on the spherical grid, and the BE
solve against a dense direct solve.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import pcg as P


def _centres(f):
    return 0.5 * (f[1:] + f[:-1])


@dataclasses.dataclass
class EdgeGrid:
    coord: str
    f: tuple            # face coordinates (f0, f1, f2)
    periodic: tuple     # per axis
    shapes: dict        # component -> shape (edges 'r', 't', 'p'; faces 'Fr', 'Ft', 'Fp')
    L: dict             # edge lengths per component
    H: dict             # edge masses S*/L (0 on fixed edges)
    w: dict             # face weights l*/S (0 on faces with no unknown)
    fixed: dict         # boolean masks of fixed edges

    @property
    def sizes(self):
        return [int(np.prod(self.shapes[c])) for c in "rtp"]

    def split(self, E):
        E = np.asarray(E, dtype=np.float64).ravel()
        n = self.sizes
        return {"r": E[:n[0]].reshape(self.shapes["r"]),
                "t": E[n[0]:n[0] + n[1]].reshape(self.shapes["t"]),
                "p": E[n[0] + n[1]:].reshape(self.shapes["p"])}

    @staticmethod
    def join(d):
        return np.concatenate([d["r"].ravel(), d["t"].ravel(), d["p"].ravel()])


def _gaps(f, c, periodic):
    """Centre-to-centre distance across face m (between cells m-1 and m), for
    m = 0..n; wraps on a periodic axis, else 0 at the two boundary faces."""
    n = len(c)
    g = np.zeros(n + 1)
    g[1:n] = c[1:] - c[:-1]
    if periodic:
        per = f[-1] - f[0]
        g[0] = g[n] = c[0] + per - c[-1]
    return g


def edge_grid(coord, f0, f1, f2, periodic=(False, False, True)) -> EdgeGrid:
    f0, f1, f2 = (np.asarray(a, dtype=np.float64) for a in (f0, f1, f2))
    n0, n1, n2 = len(f0) - 1, len(f1) - 1, len(f2) - 1
    c0, c1, c2 = _centres(f0), _centres(f1), _centres(f2)
    d0, d1, d2 = np.diff(f0), np.diff(f1), np.diff(f2)
    g0, g1, g2 = _gaps(f0, c0, periodic[0]), _gaps(f1, c1, periodic[1]), _gaps(f2, c2, periodic[2])
    # number of distinct edge / face positions along each axis (faces: n + 1, or n if periodic)
    m0 = n0 if periodic[0] else n0 + 1
    m1 = n1 if periodic[1] else n1 + 1
    m2 = n2 if periodic[2] else n2 + 1
    shapes = {"r": (n0, m1, m2), "t": (m0, n1, m2), "p": (m0, m1, n2),
              "Fr": (m0, n1, n2), "Ft": (n0, m1, n2), "Fp": (n0, n1, m2)}
    I = lambda a: a[:, None, None]  # noqa: E731
    J = lambda a: a[None, :, None]  # noqa: E731
    K = lambda a: a[None, None, :]  # noqa: E731
    f0m, f1m, f2m = f0[:m0], f1[:m1], f2[:m2]        # face positions that carry edges / faces
    g0m, g1m, g2m = g0[:m0], g1[:m1], g2[:m2]
    if coord == "spherical":
        # edge lengths
        Lr = I(d0) * np.ones(shapes["r"])
        Lt = I(f0m) * J(d1) * np.ones(shapes["t"])
        Lp = I(f0m) * J(np.sin(f1m)) * K(d2)
        # face areas and centre distances
        Sr = I(f0m ** 2) * J(np.cos(f1[:-1]) - np.cos(f1[1:])) * K(d2)
        St = I(0.5 * (f0[1:] ** 2 - f0[:-1] ** 2)) * J(np.sin(f1m)) * K(d2)
        Sp = I(0.5 * (f0[1:] ** 2 - f0[:-1] ** 2)) * J(d1) * np.ones((1, 1, m2))
        lr = I(g0m) * np.ones(shapes["Fr"])
        lt = I(c0) * J(g1m) * np.ones(shapes["Ft"])
        lp = I(c0) * J(np.sin(c1)) * K(g2m)
        # dual faces through the edges, spanned by the surrounding cell centres:
        # coordinates of the centres before / after each face (wrapping if
        # periodic; the face itself at a boundary, where the edge is fixed)
        c1m = np.concatenate([[c1[-1] - (f1[-1] - f1[0])], c1])[:m1] if periodic[1] else \
            np.concatenate([[f1[0]], c1])[:m1]
        c1p = np.concatenate([c1, [c1[0] + (f1[-1] - f1[0])]])[:m1] if periodic[1] else \
            np.concatenate([c1, [f1[-1]]])[:m1]
        c0m = np.concatenate([[c0[-1] - (f0[-1] - f0[0])], c0])[:m0] if periodic[0] else \
            np.concatenate([[f0[0]], c0])[:m0]
        c0p = np.concatenate([c0, [c0[0] + (f0[-1] - f0[0])]])[:m0] if periodic[0] else \
            np.concatenate([c0, [f0[-1]]])[:m0]
        Sr_star = I(c0 ** 2) * J(np.cos(c1m) - np.cos(c1p)) * K(g2m)
        St_star = I(0.5 * (c0p ** 2 - c0m ** 2)) * J(np.sin(c1)) * K(g2m)
        Sp_star = I(0.5 * (c0p ** 2 - c0m ** 2)) * J(c1p - c1m) * np.ones((1, 1, n2))
    elif coord == "cartesian":
        one = lambda s: np.ones(s)  # noqa: E731
        Lr = I(d0) * one(shapes["r"])
        Lt = J(d1) * one(shapes["t"])
        Lp = K(d2) * one(shapes["p"])
        Sr = J(d1) * K(d2) * one(shapes["Fr"])
        St = I(d0) * K(d2) * one(shapes["Ft"])
        Sp = I(d0) * J(d1) * one(shapes["Fp"])
        lr = I(g0m) * one(shapes["Fr"])
        lt = J(g1m) * one(shapes["Ft"])
        lp = K(g2m) * one(shapes["Fp"])
        Sr_star = J(g1m) * K(g2m) * one(shapes["r"])
        St_star = I(g0m) * K(g2m) * one(shapes["t"])
        Sp_star = I(g0m) * J(g1m) * one(shapes["p"])
    else:
        raise ValueError(coord)
    # fixed edges: those lying in a non-periodic boundary surface
    fr = np.zeros(shapes["r"], bool)
    ft = np.zeros(shapes["t"], bool)
    fp = np.zeros(shapes["p"], bool)
    if not periodic[1]:
        fr[:, [0, -1], :] = True
        fp[:, [0, -1], :] = True
    if not periodic[0]:
        ft[[0, -1], :, :] = True
        fp[[0, -1], :, :] = True
    if not periodic[2]:
        fr[:, :, [0, -1]] = True
        ft[:, :, [0, -1]] = True
    fixed = {"r": fr, "t": ft, "p": fp}
    with np.errstate(divide="ignore", invalid="ignore"):
        H = {"r": np.where(fr, 0.0, Sr_star / Lr), "t": np.where(ft, 0.0, St_star / Lt),
             "p": np.where(fp, 0.0, Sp_star / Lp)}
        w = {"Fr": lr / Sr, "Ft": lt / St, "Fp": lp / Sp}
    # faces all of whose edges are fixed carry no unknown
    g = EdgeGrid(coord, (f0, f1, f2), tuple(periodic), shapes, {"r": Lr, "t": Lt, "p": Lp}, H,
                 w, fixed)
    live = face_has_unknown(g)
    for k in ("Fr", "Ft", "Fp"):
        g.w[k] = np.where(live[k], np.nan_to_num(g.w[k]), 0.0)
    return g


def _next(a, axis, per):
    """a[.., m+1, ..] for m = 0..n-1 along `axis` (wrapping if periodic; the
    array then has n entries, else n + 1)."""
    sl = [slice(None)] * 3
    if per:
        return np.roll(a, -1, axis=axis)
    sl[axis] = slice(1, None)
    return a[tuple(sl)]


def _cur(a, axis, per):
    sl = [slice(None)] * 3
    if per:
        return a
    sl[axis] = slice(0, -1)
    return a[tuple(sl)]


def curl(g: EdgeGrid, E) -> dict:
    """Face fluxes Phi = C E (right-hand rule, normals +r, +theta, +phi):
      Phi_r = E_t(k) + E_p(j+1) - E_t(k+1) - E_p(j)
      Phi_t = E_r(k+1) - E_r(k) - E_p(i+1) + E_p(i)
      Phi_p = E_t(i+1) - E_t(i) - E_r(j+1) + E_r(j)."""
    e = g.split(E) if not isinstance(E, dict) else E
    p0, p1, p2 = g.periodic
    Er, Et, Ep = e["r"], e["t"], e["p"]
    Fr = _cur(Et, 2, p2) + _next(Ep, 1, p1) - _next(Et, 2, p2) - _cur(Ep, 1, p1)
    Ft = _next(Er, 2, p2) - _cur(Er, 2, p2) - _next(Ep, 0, p0) + _cur(Ep, 0, p0)
    Fp = _next(Et, 0, p0) - _cur(Et, 0, p0) - _next(Er, 1, p1) + _cur(Er, 1, p1)
    return {"Fr": Fr, "Ft": Ft, "Fp": Fp}


def _scatter(target, axis, per, vals, sign, shift):
    """target[.., m + shift, ..] += sign * vals[.., m, ..] (shift 0 or 1)."""
    if per:
        target += sign * (np.roll(vals, shift, axis=axis) if shift else vals)
        return
    sl = [slice(None)] * 3
    sl[axis] = slice(shift, shift + vals.shape[axis])
    target[tuple(sl)] += sign * vals


def curl_T(g: EdgeGrid, Phi: dict) -> dict:
    """C^T Phi (the adjoint of curl): each face adds its signed flux to its
    four edges."""
    p0, p1, p2 = g.periodic
    out = {c: np.zeros(g.shapes[c]) for c in "rtp"}
    Fr, Ft, Fp = Phi["Fr"], Phi["Ft"], Phi["Fp"]
    _scatter(out["t"], 2, p2, Fr, +1, 0)
    _scatter(out["p"], 1, p1, Fr, +1, 1)
    _scatter(out["t"], 2, p2, Fr, -1, 1)
    _scatter(out["p"], 1, p1, Fr, -1, 0)
    _scatter(out["r"], 2, p2, Ft, +1, 1)
    _scatter(out["r"], 2, p2, Ft, -1, 0)
    _scatter(out["p"], 0, p0, Ft, -1, 1)
    _scatter(out["p"], 0, p0, Ft, +1, 0)
    _scatter(out["t"], 0, p0, Fp, +1, 1)
    _scatter(out["t"], 0, p0, Fp, -1, 0)
    _scatter(out["r"], 1, p1, Fp, -1, 1)
    _scatter(out["r"], 1, p1, Fp, +1, 0)
    return out


def face_has_unknown(g: EdgeGrid) -> dict:
    """Faces with at least one interior (not fixed) edge."""
    n = _abs_curl(g, {c: (~g.fixed[c]).astype(np.float64) for c in "rtp"})
    return {k: v > 0 for k, v in n.items()}


def stiffness(g: EdgeGrid, E) -> np.ndarray:
    """K E = C^T diag(w) C E (all edges; rows of fixed edges included)."""
    Phi = curl(g, E)
    return EdgeGrid.join(curl_T(g, {k: g.w[k] * Phi[k] for k in Phi}))


def interior_mask(g: EdgeGrid) -> np.ndarray:
    return EdgeGrid.join({c: ~g.fixed[c] for c in "rtp"})


def apply_F(g: EdgeGrid, E, eta: float) -> np.ndarray:
    """F(E) = -eta H^-1 C^T W C E on interior edges, 0 on fixed edges."""
    KE = stiffness(g, E)
    Hv = EdgeGrid.join(g.H)
    m = interior_mask(g)
    out = np.zeros_like(KE)
    out[m] = -eta * KE[m] / Hv[m]
    return out


def gershgorin_dt_euler(g: EdgeGrid, eta: float) -> float:
    """dt_E = 2 / max_e sum_e' |(eta H^-1 K)_ee'| over interior rows and
    columns (Appendix B's Gershgorin bound applied to this operator).  Two
    distinct edges share at most one face, so the absolute row sum of K is
    sum over the faces f of e of w_f times the number of interior edges of f."""
    free = {c: (~g.fixed[c]).astype(np.float64) for c in "rtp"}
    nfree = _abs_curl(g, free)
    row = EdgeGrid.join(_abs_curl_T(g, {k: g.w[k] * nfree[k] for k in nfree}))
    m = interior_mask(g)
    Hv = EdgeGrid.join(g.H)
    return 2.0 / np.max(eta * row[m] / Hv[m])


def _abs_curl(g: EdgeGrid, e: dict) -> dict:
    """|C| e: the sum of a face's four edge values."""
    p0, p1, p2 = g.periodic
    return {"Fr": _cur(e["t"], 2, p2) + _next(e["p"], 1, p1) + _next(e["t"], 2, p2) +
            _cur(e["p"], 1, p1),
            "Ft": _next(e["r"], 2, p2) + _cur(e["r"], 2, p2) + _next(e["p"], 0, p0) +
            _cur(e["p"], 0, p0),
            "Fp": _next(e["t"], 0, p0) + _cur(e["t"], 0, p0) + _next(e["r"], 1, p1) +
            _cur(e["r"], 1, p1)}


def dense_stiffness(g: EdgeGrid) -> np.ndarray:
    """Dense K = C^T W C by columns (tiny grids only)."""
    n = sum(g.sizes)
    K = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        K[:, c] = stiffness(g, e)
    return K


def be_system(g: EdgeGrid, E_n, dt: float, eta: float):
    """Interior-edge BE system A x = b: A = H + dt eta K restricted to interior
    edges, b = H E^n - dt eta (K E_b) with E_b = E^n on fixed edges, 0 elsewhere.
    Returns (matvec on interior vectors, b, diag(A), interior mask)."""
    E_n = np.asarray(E_n, dtype=np.float64).ravel()
    m = interior_mask(g)
    Hv = EdgeGrid.join(g.H)
    Eb = np.where(m, 0.0, E_n)
    b = (Hv * E_n - dt * eta * stiffness(g, Eb))[m]
    n = len(E_n)

    def matvec(x):
        full = np.zeros(n)
        full[m] = x
        return (Hv * full + dt * eta * stiffness(g, full))[m]

    # diag(K)_e = sum of w_f over the faces of e (incidences are +-1)
    diagK = EdgeGrid.join(_abs_curl_T(g, {k: g.w[k] for k in ("Fr", "Ft", "Fp")}))
    d = (Hv + dt * eta * diagK)[m]
    return matvec, b, d, m


def _abs_curl_T(g: EdgeGrid, wf: dict) -> dict:
    """|C|^T wf: each face adds w_f to each of its four edges (the diagonal of
    C^T W C, since the incidences are +-1)."""
    p0, p1, p2 = g.periodic
    out = {c: np.zeros(g.shapes[c]) for c in "rtp"}
    Fr, Ft, Fp = wf["Fr"], wf["Ft"], wf["Fp"]
    for tgt, ax, per, vals, sh in (("t", 2, p2, Fr, 0), ("p", 1, p1, Fr, 1), ("t", 2, p2, Fr, 1),
                                   ("p", 1, p1, Fr, 0), ("r", 2, p2, Ft, 1), ("r", 2, p2, Ft, 0),
                                   ("p", 0, p0, Ft, 1), ("p", 0, p0, Ft, 0), ("t", 0, p0, Fp, 1),
                                   ("t", 0, p0, Fp, 0), ("r", 1, p1, Fp, 1), ("r", 1, p1, Fp, 0)):
        _scatter(out[tgt], ax, per, vals, +1, sh)
    return out


def be_pcg(g: EdgeGrid, E_n, dt: float, eta: float, rtol=1e-8, maxit=10000, keep=()):
    """BE step by PCG with PC1 from x0 = E^n; returns (E^{n+1} on all edges,
    the pcg.PCGResult of the interior system)."""
    E_n = np.asarray(E_n, dtype=np.float64).ravel()
    matvec, b, d, m = be_system(g, E_n, dt, eta)
    res = P.pcg(matvec, b, E_n[m], lambda r: r / d, rtol, maxit, keep)
    out = E_n.copy()
    out[m] = res.x
    return out, res
