"""Synthetic spherical-shell inputs (FP64, numpy only).

The paper's production case (Sec. 5, Table "tab:grid") is a global coronal
relaxation on a logically rectangular non-uniform (r, theta, phi) grid with
T ~ 1-1.5 MK near the Sun and a field-aligned conduction direction b = B/|B|.
Its data (an ADAPT magnetogram and the MAS state) are not available, so these
seeded stand-ins reproduce the *kind* of input:

* faces uniform in ln r on [1, 2.5] (2.9 % stretch per cell at N_r = 32),
  theta in [0.05 pi, 0.95 pi] (poles excluded), phi periodic on [0, 2 pi);
* T = 1e6 (1 + 0.5 / r^2)(1 + 0.1 n) K with n a smoothed, standardised
  Gaussian field;
* b a unit dipole direction with moment tilted 30 degrees off the polar axis,
  so that all three local components are non-zero (an axis-aligned dipole
  would make b_phi vanish and the 19-point stencil collapse to r-theta planes);
* velocity components for the viscosity operator: smoothed noise, amplitude 1.

Nothing here evaluates the method: no diffusivity, no geometry factors.
Cell centres are arithmetic midpoints of faces (needed to place the fields).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

R_MIN, R_MAX = 1.0, 2.5
TH_MIN, TH_MAX = 0.05 * math.pi, 0.95 * math.pi
T_INNER = 1.5e6  # Dirichlet value on the inner radial boundary (background at r = 1)
KAPPA0 = 1e-15   # Spitzer constant in code units (kappa = O(1)); cancels in dt / dt_Euler


def shell_faces(nr: int, nth: int, nph: int):
    """Face coordinates of the shell grid (host FP64 1D arrays)."""
    i = np.arange(nr + 1, dtype=np.float64)
    rf = R_MAX ** (i / nr)  # R_MIN = 1, uniform in ln r
    j = np.arange(nth + 1, dtype=np.float64)
    thf = TH_MIN + (TH_MAX - TH_MIN) * j / nth
    k = np.arange(nph + 1, dtype=np.float64)
    phf = 2.0 * math.pi * k / nph
    return rf, thf, phf


def box_faces(n0: int, n1: int, n2: int, h=(1.0, 1.0, 1.0)):
    """Face coordinates of a uniform Cartesian box (used for Fourier tests)."""
    return tuple(np.arange(n + 1, dtype=np.float64) * hh for n, hh in zip((n0, n1, n2), h))


def _centres(f):
    return 0.5 * (f[1:] + f[:-1])


def _smooth_axis(a: np.ndarray, axis: int, periodic: bool) -> np.ndarray:
    if periodic:
        lo = np.roll(a, 1, axis=axis)
        hi = np.roll(a, -1, axis=axis)
    else:
        n = a.shape[axis]
        idx_lo = np.concatenate(([0], np.arange(n - 1)))
        idx_hi = np.concatenate((np.arange(1, n), [n - 1]))
        lo = np.take(a, idx_lo, axis=axis)
        hi = np.take(a, idx_hi, axis=axis)
    return 0.25 * lo + 0.5 * a + 0.25 * hi


def smooth_noise(shape, seed: int, passes: int = 4) -> np.ndarray:
    """Standard-normal noise, smoothed by `passes` [1/4, 1/2, 1/4] sweeps per
    axis (phi periodic, r / theta edge-replicated), then standardised."""
    n = np.random.default_rng(seed).standard_normal(shape)
    for _ in range(passes):
        n = _smooth_axis(n, 0, False)
        n = _smooth_axis(n, 1, False)
        n = _smooth_axis(n, 2, True)
    n = n - n.mean()
    s = n.std()
    return n / s if s > 0 else n


def temperature(rf, thf, phf, seed: int) -> np.ndarray:
    nr, nth, nph = len(rf) - 1, len(thf) - 1, len(phf) - 1
    rc = _centres(rf)
    n = smooth_noise((nr, nth, nph), seed)
    return 1e6 * (1.0 + 0.5 / rc[:, None, None] ** 2) * (1.0 + 0.1 * n)


def dipole_bhat(rf, thf, phf, tilt_deg: float = 30.0):
    """Unit vectors of a tilted dipole field at cell centres, as local
    (r, theta, phi) components.  B ~ 3 (m.rhat) rhat - m, which never vanishes."""
    rc, tc, pc = _centres(rf), _centres(thf), _centres(phf)
    del rc  # the direction of a dipole does not depend on r
    t = math.radians(tilt_deg)
    m = np.array([math.sin(t), 0.0, math.cos(t)])
    th = tc[:, None]
    ph = pc[None, :]
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    rhat = (st * cp, st * sp, ct * np.ones_like(ph))
    thhat = (ct * cp, ct * sp, -st * np.ones_like(ph))
    phhat = (-sp * np.ones_like(th), cp * np.ones_like(th), np.zeros_like(th * ph))
    m_r = m[0] * rhat[0] + m[1] * rhat[1] + m[2] * rhat[2]
    m_t = m[0] * thhat[0] + m[1] * thhat[1] + m[2] * thhat[2]
    m_p = m[0] * phhat[0] + m[1] * phhat[1] + m[2] * phhat[2]
    br, bt, bp = 2.0 * m_r, -m_t, -m_p
    nrm = np.sqrt(br * br + bt * bt + bp * bp)
    nr = len(rf) - 1
    shape = (nr,) + br.shape
    return tuple(np.broadcast_to(c / nrm, shape).copy() for c in (br, bt, bp))


def random_unit_vectors(shape, seed: int):
    """Uncorrelated random unit vectors per cell (a rough, adversarial b field)."""
    g = np.random.default_rng(seed).standard_normal((3,) + tuple(shape))
    g /= np.sqrt((g * g).sum(axis=0))
    return g[0].copy(), g[1].copy(), g[2].copy()


def velocity(rf, thf, phf, seeds=(1, 2, 3)):
    nr, nth, nph = len(rf) - 1, len(thf) - 1, len(phf) - 1
    return tuple(smooth_noise((nr, nth, nph), s) for s in seeds)


def edge_potential(nr: int, nth: int, nph: int, seed: int = 4):
    """A seeded vector-potential field on the cell edges of an nr x nth x nph
    shell (phi periodic), in the edge layout [E_r | E_t | E_p] with E_r
    [nr][nth+1][nph], E_t [nr+1][nth][nph], E_p [nr+1][nth+1][nph]: smooth
    noise per component (inputs only; no arithmetic of the method)."""
    shapes = ((nr, nth + 1, nph), (nr + 1, nth, nph), (nr + 1, nth + 1, nph))
    return np.concatenate([smooth_noise(s, seed + q).ravel() for q, s in enumerate(shapes)])


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named synthetic workload (the shapes of the paper-style configs)."""
    name: str
    nr: int
    nth: int
    nph: int
    seed: int
    dt_factor: float  # dt = dt_factor * dt_Euler
    rtol: float
    block: tuple = (8, 8, 8)
    viscosity: bool = False

    @property
    def cells(self) -> int:
        return self.nr * self.nth * self.nph


WORKLOADS = {
    "shell32": Workload("shell32", 32, 32, 64, 0, 50.0, 1e-9),
    "shell128": Workload("shell128", 128, 128, 256, 0, 200.0, 1e-8),
    "shell256": Workload("shell256", 256, 256, 512, 0, 500.0, 1e-8, viscosity=True),
}


def make_workload(w: Workload | str, with_velocity: bool | None = None) -> dict:
    """All inputs of a workload as host FP64 arrays (C-contiguous, phi fastest)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rf, thf, phf = shell_faces(w.nr, w.nth, w.nph)
    T = temperature(rf, thf, phf, w.seed)
    br, bt, bp = dipole_bhat(rf, thf, phf)
    out = dict(rf=rf, thf=thf, phf=phf, T=T, br=br, bt=bt, bp=bp,
               kappa0=KAPPA0, T_inner=T_INNER, workload=w)
    if with_velocity if with_velocity is not None else w.viscosity:
        out["v"] = velocity(rf, thf, phf)
        out["nu"] = 1.0
    return out
