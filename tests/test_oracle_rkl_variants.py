"""Pins for the super-step variants of Sec. 6 (oracle/rkl_variants.py): the
Legendre closed form and consistency of RKL1, its stability bound, the
paper's remarks on RKL1 with extra stages, on sub-cycling RKL2 and on
explicit Euler sub-steps against backward Euler, and the convergence order
of sub-cycled steps on a smooth mode."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as Lg

from oracle import rkl2 as R2
from oracle import rkl_variants as V


@pytest.mark.parametrize("s", [1, 2, 3, 7, 16, 40])
def test_rkl1_is_legendre(s):
    z = np.linspace(-(s * s + s), 0.0, 257)
    c = np.zeros(s + 1)
    c[s] = 1.0
    ref = Lg.legval(1.0 + 2.0 * z / (s * s + s), c)
    assert np.max(np.abs(V.rkl1_amplification(z, s) - ref)) < 1e-12


@pytest.mark.parametrize("s", [2, 5, 11])
def test_rkl1_first_order_and_stable(s):
    h = 1e-6
    d = (V.rkl1_amplification(np.array([h]), s)[0] - V.rkl1_amplification(np.array([-h]), s)[0]) / (2 * h)
    assert d == pytest.approx(1.0, rel=1e-8)
    z = np.linspace(-(s * s + s), 0.0, 2001)
    assert np.max(np.abs(V.rkl1_amplification(z, s))) <= 1.0 + 1e-12


@pytest.mark.parametrize("r", [0.3, 1.0, 2.5, 50.0, 612.0, 9554.0])
def test_rkl1_stage_count_minimal(r):
    s = V.rkl1_stage_count(r)
    assert s * s + s >= 2 * r
    if s > 1:
        assert (s - 1) * s < 2 * r
    assert V.rkl1_stage_count(r, extra=3) == s + 3


@pytest.mark.parametrize("s", range(1, 30))
def test_rkl1_extra_stages_leave_the_top_mode(s):
    """Sec. 6: with s matched exactly to the step, |R| = 1 at the highest
    mode; any extra stage brings it below 1."""
    r = (s * s + s) / 2.0  # dt/dt_E for which s is exact
    z = -2.0 * r           # dt times the Gershgorin-extreme eigenvalue
    assert abs(V.rkl1_amplification(np.array([z]), s)[0]) == pytest.approx(1.0, abs=1e-9)
    for e in range(1, 6):
        assert abs(V.rkl1_amplification(np.array([z]), s + e)[0]) < 1.0 - 1e-3


@pytest.mark.parametrize("r", [50.0, 500.0])
def test_subcycling_damps_high_modes(r):
    """Sec. 6: about ten sub-cycles bring RKL2 close to BE on the upper half
    of the spectrum (dt lambda in [-2r, -r]): the worst amplification drops
    more than 20-fold and to within 15x of BE's."""
    z = -np.linspace(r, 2 * r, 400)

    def sub(m):
        s = R2.stage_count(r / m)
        return np.abs(R2.amplification(z / m, s)) ** m

    one, ten = sub(1).max(), sub(10).max()
    be = np.abs(R2.be_amplification(z)).max()
    assert ten < one / 20 and ten < 15 * be
    # the super-step with nsub = 10 applies exactly these sub-steps
    dte = 1.0
    lam = z / r  # dt = r dt_E
    u, napply = V.super_step(lambda v: lam * v, np.ones_like(z), r, dte, nsub=10)
    assert np.allclose(np.abs(u), sub(10), rtol=1e-12, atol=1e-300)
    assert napply == 10 * R2.stage_count(r / 10)


@pytest.mark.parametrize("r", [50.0, 500.0])
def test_euler_quarter_step_damps_more_than_be(r):
    """Sec. 6: explicit Euler sub-steps over a quarter of the step damp the
    upper half of the spectrum more than a full BE step."""
    n, h = V.euler_substeps(r, 1.0, 0.25)
    assert n * h == pytest.approx(0.25 * r) and h <= 0.5 + 1e-15
    zs = -np.linspace(r, 2 * r, 400)
    lam = zs / r  # eigenvalues in units of 1/dt_E
    euler = np.abs((1.0 + h * lam) ** n)
    assert np.all(euler < np.abs(R2.be_amplification(zs)))


def test_subcycled_error_orders():
    """On a smooth mode the sub-cycled RKL2 error falls ~m^-2 (second order)
    and RKL1's ~m^-1 (first order)."""
    lam = -0.7
    dt = 3.0
    exact = math.exp(lam * dt)

    def err(scheme, m):
        u, _ = V.super_step(lambda v: lam * v, np.array([1.0]), dt, 1.0, scheme=scheme, nsub=m)
        return abs(u[0] - exact)

    e2 = [err(2, m) for m in (4, 8, 16)]
    e1 = [err(1, m) for m in (4, 8, 16)]
    assert 3.0 < e2[0] / e2[1] < 5.5 and 3.0 < e2[1] / e2[2] < 5.5
    assert 1.6 < e1[0] / e1[1] < 2.6 and 1.6 < e1[1] / e1[2] < 2.6


def test_super_step_defaults_reduce_to_rkl2():
    rng = np.random.default_rng(0)
    A = -np.diag(rng.random(6) * 40)
    u0 = rng.standard_normal(6)
    F = lambda v: A @ v  # noqa: E731
    u, n = V.super_step(F, u0, 20.0, 1.0)
    s = R2.stage_count(20.0)
    assert np.array_equal(u, R2.rkl2_step(F, u0, 20.0, s)) and n == s
