"""Pins for the oracle's RKL2 (Sec. 3: Fig. rkl2, coefficient block, Eq. rkl2_s)."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import operator as O
from oracle import rkl2
from workloads import box_faces


def closed_form(z, s):
    """RKL2 stability polynomial of the paper's reference [RKL2_2014]:
    R_s(z) = 1 - b_s + b_s P_s(1 + w1 z), w1 = 4 / (s^2 + s - 2) (Legendre P_s)."""
    bs = (s * s + s - 2.0) / (2.0 * s * (s + 1.0)) if s > 2 else 1.0 / 3.0
    w1 = 4.0 / (s * s + s - 2.0)
    return 1.0 - bs + bs * eval_legendre(s, 1.0 + w1 * np.asarray(z))


@pytest.mark.parametrize("s", [2, 3, 4, 7, 14, 28, 45, 60])
def test_recurrence_matches_legendre_closed_form(s):
    zmin = -(s * s + s - 2.0) / 2.0
    z = np.linspace(zmin, 0.0, 801)
    R = rkl2.amplification(z, s)
    assert np.max(np.abs(R - closed_form(z, s))) <= 1e-11


@pytest.mark.parametrize("s", [3, 14, 28, 45])
def test_stable_on_interval_and_second_order(s):
    zmin = -(s * s + s - 2.0) / 2.0
    z = np.linspace(zmin, 0.0, 4001)
    assert np.max(np.abs(rkl2.amplification(z, s))) <= 1.0 + 1e-12
    # R(z) = 1 + z + z^2/2 + O(z^3): second-order accuracy
    for h in (1e-2, 5e-3):
        R = rkl2.amplification(np.array([-h]), s)[0]
        taylor = 1.0 - h + 0.5 * h * h
        assert abs(R - taylor) <= 10 * (s ** 4) * h ** 3


def test_literal_gamma_index_is_unstable():
    """The printed last term (b_k - 1) mu~_k leaves the recurrence unstable,
    which is why the index is read as k - 1."""
    s = 28
    c = rkl2.coefficients(s)
    z = np.linspace(-(s * s + s - 2.0) / 2.0, 0.0, 2001)
    u0 = np.ones_like(z)
    F0 = z * u0
    um2, um1 = u0, u0 + c["mut"][1] * F0
    for k in range(2, s + 1):
        lit = (c["b"][k] - 1.0) * c["mut"][k]
        uk = c["mu"][k] * um1 + c["nu"][k] * um2 + (1 - c["mu"][k] - c["nu"][k]) * u0 \
            + c["mut"][k] * z * um1 + lit * F0
        um2, um1 = um1, uk
    assert np.max(np.abs(um1)) > 1.5


@pytest.mark.parametrize("ratio,s", [(50, 14), (200, 28), (500, 45), (0.2, 2), (1.0, 2), (2.5, 3)])
def test_stage_count(ratio, s):
    got = rkl2.stage_count(ratio)
    assert got == s
    assert got * got + got - 2 >= 4 * ratio
    if got > 2:
        assert (got - 1) ** 2 + (got - 1) - 2 < 4 * ratio


def test_stage_count_odd_option():
    assert rkl2.stage_count(200, odd=True) == 29
    assert rkl2.stage_count(500, odd=True) == 45


def _golden_substeps():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_rkl2_substeps.txt")
    rows = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, s, r = line.split()
                rows[name] = (int(s), float(r))
    return rows


def test_paper_substep_counts_consistent():
    """The printed average sub-step counts (Fig. iters caption) are stage counts
    of Eq. rkl2_s: 195 for dt/dt_E in (9457, 9554.5], 49 in (587.5, 612]; the
    printed maximal ratios (Sec. 6) need at least as many stages as the averages."""
    g = _golden_substeps()
    s_c, r_c = g["conduction"]
    s_v, r_v = g["viscosity"]
    assert (s_c, s_v) == (195, 49)
    assert rkl2.stage_count(9554) == s_c and rkl2.stage_count(9458) == s_c
    assert rkl2.stage_count(9457) == s_c - 1 and rkl2.stage_count(9555) == s_c + 1
    assert rkl2.stage_count(612) == s_v and rkl2.stage_count(588) == s_v
    assert rkl2.stage_count(587) == s_v - 1 and rkl2.stage_count(613) == s_v + 1
    assert rkl2.stage_count(r_c) >= s_c and rkl2.stage_count(r_v) >= s_v


@pytest.mark.parametrize("ratio,lo,hi", [(5, 0.3, 0.7), (50, 0.3, 0.7), (500, 0.3, 0.7)])
def test_high_mode_damping_about_half_not_L_stable(ratio, lo, hi):
    """Sec. 6 / Fig. ampfac: at large dt/dt_E the highest modes are damped by
    only ~0.5 (not L-stable), while BE damps them towards 0."""
    s = rkl2.stage_count(ratio)
    zhigh = -2.0 * ratio  # the Gershgorin-extreme mode, dt |lambda|_max = 2 dt/dt_E
    R = rkl2.amplification(np.array([zhigh]), s)[0]
    assert lo < abs(R) < hi
    assert abs(rkl2.be_amplification(zhigh)) < 1.0 / (2 * ratio)


def test_speedup_over_euler():
    """Fig. rkl2speedup: speedup = ceil(dt/dt_E) / s."""
    for r in (10, 100, 1000):
        s = rkl2.stage_count(r)
        assert math.ceil(r) / s > 1.0
    assert math.ceil(500) / rkl2.stage_count(500) == pytest.approx(500 / 45)


@pytest.mark.parametrize("modes", [(1, 2, 3), (3, 4, 5), (0, 1, 6)])
def test_rkl2_on_fourier_mode_of_periodic_box(modes):
    """The full rkl2_step on one cosine mode returns R_s(dt lambda) times the mode."""
    n, h = (8, 10, 12), (1.0, 0.8, 1.2)
    bvec = np.array([0.4, 0.5, -0.7])
    bvec /= np.linalg.norm(bvec)
    shape = n
    D = {(a, b): np.full(shape, 2.0 * bvec[a] * bvec[b]) for a in range(3) for b in range(a, 3)}
    op = O.assemble("cartesian", *box_faces(*n, h=h), D, (O.PERIODIC,) * 6)
    theta = [2 * math.pi * m / nn for m, nn in zip(modes, n)]
    idx = np.meshgrid(*[np.arange(nn) for nn in n], indexing="ij")
    u = np.cos(sum(t * i for t, i in zip(theta, idx)))
    lam = 0.0
    for a in range(3):
        lam -= 4 * 2.0 * bvec[a] ** 2 * math.sin(theta[a] / 2) ** 2 / h[a] ** 2
    for a in range(3):
        for b in range(a + 1, 3):
            lam -= 2 * 2.0 * bvec[a] * bvec[b] * math.sin(theta[a]) * math.sin(theta[b]) / (h[a] * h[b])
    dtE = O.gershgorin_dt_euler(op)
    dt = 37.0 * dtE
    s = rkl2.stage_count(37.0)
    out = rkl2.rkl2_step(lambda v: O.apply_F(op, v), u, dt, s)
    assert np.max(np.abs(out - closed_form(dt * lam, s) * u)) <= 1e-12
