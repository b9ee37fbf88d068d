"""The linearised parabolic operator F(u) (oracle, test-only).

The paper isolates each parabolic term as du/dt = F(u) (Eq. pde) and, for
conduction, freezes the temperature-dependent diffusivity at the previous
step's temperature ("lagged diffusivity", Sec. 1) so that F is linear within a
step.  The conduction term is the Spitzer flux div(kappa0 T^{5/2} b b . grad T)
(Eq. mhd:e1, blue box); the artificial viscosity is div(nu grad v) per
component (Eq. mhd:v, blue box, with rho = 1).  MAS stores these operators as
19-diagonal (conduction) / 15-diagonal (viscosity) DIA matrices (Sec. 4.2,
Appendix B: p = 19, 15).

Discretisation reading (the paper names only "the standard scheme" of its
reference [TCO_STD]): a cell-centred finite-volume form derived as
F(u) = -V^-1 dE/du of the discrete energy

    E(u) = 1/2 sum_faces w_f (u_c' - u_c)^2  +  sum_edges K_e X_e Y_e
           + 1/2 sum_Dirichlet-faces w_b (u_b - u_c)^2

with
  * face weight  w_f = A_f * Dbar_aa / dl_f,  Dbar = mean of D over the two cells;
  * edge (a, b)-plane, corner cells c00 = c, c10 = c+e_a, c01 = c+e_b, c11:
      X = 1/2[(u10-u00)/dl_a(c00) + (u11-u01)/dl_a(c01)]   (a-derivative)
      Y = 1/2[(u01-u00)/dl_b(c00) + (u11-u10)/dl_b(c10)]   (b-derivative)
      K_e = W_e * Dbar_ab,  W_e and Dbar_ab = means over the four cells;
  * D = kappa b b^T in the local (r, theta, phi) basis, kappa = kappa0 T^{5/2};
  * Dirichlet face: w_b = A_b D_aa(c) / (distance centre -> face).

This gives exactly the 19-point pattern with an exactly symmetric S
(S = -Hessian of E, g = -gradient at u = 0), so F(u) = V^-1 (S u + g).
Faces / edges that would reach outside a non-periodic boundary are omitted
(zero flux); the phi axis of the shell is periodic.

The assembled operator is held as 19 stencil slots S19[slot][cell] =
S[cell, cell + OFFSETS[slot]] (the paper's DIA reading of the matrix).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import geometry as geo

# 19-point offsets: self, 6 faces, 12 edges.  Slot 0 is the diagonal.
OFFSETS = [(0, 0, 0)]
for _a in range(3):
    for _s in (-1, 1):
        _o = [0, 0, 0]
        _o[_a] = _s
        OFFSETS.append(tuple(_o))
for _a in range(3):
    for _b in range(_a + 1, 3):
        for _sa in (-1, 1):
            for _sb in (-1, 1):
                _o = [0, 0, 0]
                _o[_a] = _sa
                _o[_b] = _sb
                OFFSETS.append(tuple(_o))
SLOT = {o: s for s, o in enumerate(OFFSETS)}
assert len(OFFSETS) == 19 and len(SLOT) == 19

ZEROFLUX, DIRICHLET, PERIODIC = "zeroflux", "dirichlet", "periodic"
SHELL_BC = (DIRICHLET, ZEROFLUX, ZEROFLUX, ZEROFLUX, PERIODIC, PERIODIC)  # r-, r+, th-, th+, ph-, ph+


def _shift(x: np.ndarray, off) -> np.ndarray:
    """y[c] = x[c - off] (wrapping); used to move values defined at an edge /
    face origin onto the cell at origin + off."""
    return np.roll(x, shift=tuple(off), axis=(0, 1, 2))


def _ahead(x: np.ndarray, off) -> np.ndarray:
    """y[c] = x[c + off] (wrapping)."""
    return np.roll(x, shift=tuple(-o for o in off), axis=(0, 1, 2))


def _unit(a: int):
    o = [0, 0, 0]
    o[a] = 1
    return tuple(o)


def _recip(x: np.ndarray) -> np.ndarray:
    """1/x where x > 0, else 0 (distances across faces that do not exist)."""
    return np.divide(1.0, x, out=np.zeros_like(x), where=x > 0)


def _add(*offs):
    return tuple(sum(x) for x in zip(*offs))


def spitzer_tensor(T, kappa0, br, bt, bp) -> dict:
    """D = kappa b b^T with kappa = kappa0 T^{5/2} (Eq. mhd:e1, lagged: T is the
    temperature at the start of the step).  Keys (a, b) with a <= b."""
    kappa = kappa0 * np.asarray(T, dtype=np.float64) ** 2.5
    b = (np.asarray(br, np.float64), np.asarray(bt, np.float64), np.asarray(bp, np.float64))
    return {(a, c): kappa * b[a] * b[c] for a in range(3) for c in range(a, 3)}


def isotropic_tensor(shape, nu) -> dict:
    """D = nu I: the artificial kinematic viscosity div(nu grad v) per component
    (Eq. mhd:v with rho = 1)."""
    nu_arr = np.broadcast_to(np.asarray(nu, dtype=np.float64), shape).copy()
    z = np.zeros(shape)
    return {(a, c): (nu_arr if a == c else z) for a in range(3) for c in range(a, 3)}


@dataclasses.dataclass
class Operator:
    geom: dict
    S19: np.ndarray        # [19, n0, n1, n2]
    g: np.ndarray          # Dirichlet source term
    face_w: list           # w_a on +a faces (0 where absent)
    edge_K: dict           # K_ab at edges with origin c00 (0 where absent)

    @property
    def V(self):
        return self.geom["V"]

    @property
    def shape(self):
        return self.geom["shape"]


def _axis_periodic(bc, a):
    lo, hi = bc[2 * a], bc[2 * a + 1]
    if (lo == PERIODIC) != (hi == PERIODIC):
        raise ValueError("periodic must be set on both sides of an axis")
    return lo == PERIODIC


def assemble(coord, f0, f1, f2, D: dict, bc=SHELL_BC, u_lo=0.0, u_hi=0.0) -> Operator:
    """Assemble S (19 slots) and g from the discrete energy E (module doc).

    bc: 6 entries (axis0-, axis0+, axis1-, axis1+, axis2-, axis2+) out of
    ZEROFLUX / PERIODIC, and DIRICHLET on the two axis-0 sides only.
    u_lo / u_hi: Dirichlet values (scalar or [n1, n2])."""
    periodic = tuple(_axis_periodic(bc, a) for a in range(3))
    for a in (1, 2):
        if DIRICHLET in (bc[2 * a], bc[2 * a + 1]):
            raise ValueError("Dirichlet boundaries are supported on axis 0 only")
    G = geo.geometry(coord, f0, f1, f2, periodic)
    shape = G["shape"]
    for a in range(3):
        if periodic[a] and shape[a] < 3:
            raise ValueError("a periodic axis needs at least 3 cells")
    V, A, dl = G["V"], G["A"], G["dl"]
    S19 = np.zeros((19,) + shape)
    g = np.zeros(shape)

    def exists_ahead(a):
        """Mask of cells c for which c + e_a is in the domain."""
        m = np.ones(shape, dtype=bool)
        if not periodic[a]:
            idx = [slice(None)] * 3
            idx[a] = -1
            m[tuple(idx)] = False
        return m

    # ---- faces: E_f = 1/2 w (u_{c+a} - u_c)^2 ----
    face_w = []
    for a in range(3):
        ea = _unit(a)
        Daa = D[(a, a)]
        w = A[a] * 0.5 * (Daa + _ahead(Daa, ea)) * _recip(dl[a])
        w = np.where(exists_ahead(a), w, 0.0)
        face_w.append(w)
        # Hessian of 1/2 w (u1 - u0)^2 is w [[1, -1], [-1, 1]]; S = -Hessian
        roles = [(0, 0, 0), ea]
        hess = [[w, -w], [-w, w]]
        for m in range(2):
            for n in range(2):
                slot = SLOT[tuple(np.subtract(roles[n], roles[m]))]
                S19[slot] -= _shift(hess[m][n], roles[m])

    # ---- edges: E_e = K X Y ----
    edge_K = {}
    for a in range(3):
        for b in range(a + 1, 3):
            ea, eb = _unit(a), _unit(b)
            roles = [(0, 0, 0), ea, eb, _add(ea, eb)]  # c00, c10, c01, c11
            ex = exists_ahead(a) & exists_ahead(b)
            Wv = 0.25 * sum(_ahead(V, r) for r in roles)
            Dab = 0.25 * sum(_ahead(D[(a, b)], r) for r in roles)
            K = np.where(ex, Wv * Dab, 0.0)
            edge_K[(a, b)] = K
            ia0 = _recip(dl[a])                 # 1/dl_a(c00)
            ia1 = _recip(_ahead(dl[a], eb))     # 1/dl_a(c01)
            ib0 = _recip(dl[b])                 # 1/dl_b(c00)
            ib1 = _recip(_ahead(dl[b], ea))     # 1/dl_b(c10)
            # X = sum alpha_m u_m, Y = sum beta_m u_m over (c00, c10, c01, c11)
            alpha = [-0.5 * ia0, 0.5 * ia0, -0.5 * ia1, 0.5 * ia1]
            beta = [-0.5 * ib0, -0.5 * ib1, 0.5 * ib0, 0.5 * ib1]
            for m in range(4):
                for n in range(4):
                    h = K * (alpha[m] * beta[n] + beta[m] * alpha[n])  # Hessian of K X Y
                    slot = SLOT[tuple(np.subtract(roles[n], roles[m]))]
                    S19[slot] -= _shift(h, roles[m])

    # ---- Dirichlet faces on axis 0: E_b = 1/2 w_b (u_b - u_c)^2 ----
    for side, (kind, ub) in enumerate(((bc[0], u_lo), (bc[1], u_hi))):
        if kind != DIRICHLET:
            continue
        i = 0 if side == 0 else shape[0] - 1
        wb = G["Ab"][side] * D[(0, 0)][i] / G["db"][side]
        S19[0][i] -= wb
        g[i] += wb * np.broadcast_to(np.asarray(ub, dtype=np.float64), wb.shape)
    return Operator(G, S19, g, face_w, edge_K)


def apply_S(op: Operator, u: np.ndarray) -> np.ndarray:
    """(S u)_c = sum_slots S19[slot][c] u[c + offset]  (homogeneous part)."""
    out = np.zeros(op.shape)
    for s, off in enumerate(OFFSETS):
        out += op.S19[s] * _ahead(u, off)
    return out


def apply_F(op: Operator, u: np.ndarray) -> np.ndarray:
    """F(u) = V^-1 (S u + g)  (Eq. pde with the lagged, linear operator)."""
    return (apply_S(op, u) + op.g) / op.V


def apply_M(op: Operator, u: np.ndarray) -> np.ndarray:
    """M u = V^-1 S u: the homogeneous (matrix) part of F (Eq. BE_lin)."""
    return apply_S(op, u) / op.V


def dense_S(op: Operator) -> np.ndarray:
    """Dense S for tiny grids (tests)."""
    n = int(np.prod(op.shape))
    out = np.zeros((n, n))
    idx = np.arange(n).reshape(op.shape)
    for s, off in enumerate(OFFSETS):
        cols = _ahead(idx, off)
        np.add.at(out, (idx.ravel(), cols.ravel()), op.S19[s].ravel())
    return out


def gershgorin_dt_euler(op: Operator) -> float:
    """dt_Euler = 2 / |lambda|_max with the Gershgorin bound
    |lambda|_max <= max over rows of sum_j |M_ij|, M = V^-1 S (Appendix B,
    Eqs. dteuler and gstb).  Reading: the printed radius sums |A_ij| over i
    for row j; for the symmetric S the row/column distinction only matters
    through V, and M = V^-1 S is summed along its rows."""
    rows = np.zeros(op.shape)
    for s in range(19):
        rows += np.abs(op.S19[s])
    # slots that alias to the same neighbour (tiny periodic axes) would be
    # summed separately here; assemble() forbids periodic axes below 3 cells.
    return 2.0 / float(np.max(rows / op.V))


def ktilde_dt_euler(coord, f0, f1, f2, alpha_max: float) -> float:
    """The looser estimate of Appendix B: |lambda| < max(alpha k~^2) with
    k~^2 = 4 [1/dr^2 + 1/(r dth)^2 + 1/(r sin th dph)^2] (spherical)."""
    f0, f1, f2 = (np.asarray(f, np.float64) for f in (f0, f1, f2))
    c0, c1 = geo.centres(f0), geo.centres(f1)
    d0, d1, d2 = np.diff(f0), np.diff(f1), np.diff(f2)
    if coord == geo.SPHERICAL:
        k2 = 4.0 * (1.0 / d0[:, None, None] ** 2
                    + 1.0 / (c0[:, None, None] * d1[None, :, None]) ** 2
                    + 1.0 / (c0[:, None, None] * np.sin(c1)[None, :, None] * d2[None, None, :]) ** 2)
    else:
        k2 = 4.0 * (1.0 / d0[:, None, None] ** 2 + 1.0 / d1[None, :, None] ** 2
                    + 1.0 / d2[None, None, :] ** 2)
    return 2.0 / float(np.max(alpha_max * k2))


def be_system(op: Operator, u_n: np.ndarray, dt: float):
    """Backward Euler (Eqs. BE, BE_lin, BE_linsolve) in the symmetric form
    A u^{n+1} = b with A = V - dt S (SPD) and b = V u^n + dt g.  Reading: the
    paper's A = 1 - dt M with M "symmetric positive-definite" is a sign slip
    (-M is positive semi-definite); multiplying by V makes A symmetric on a
    non-uniform grid.  Returns (A19, b)."""
    A19 = -dt * op.S19
    A19[0] = A19[0] + op.V
    b = op.V * u_n + dt * op.g
    return A19, b


def apply19(A19: np.ndarray, u: np.ndarray) -> np.ndarray:
    out = np.zeros(u.shape)
    for s, off in enumerate(OFFSETS):
        out += A19[s] * _ahead(u, off)
    return out
