"""Pins for the resistive curl-curl operator (oracle/resistivity.py).

Independent of the oracle's assembly: the curl of a discrete gradient
(exact incidence identity), div B = 0 cell by cell, symmetry and the exact
null space (gradients of interior node potentials), the closed-form
spectrum on a periodic box, convergence to -curl curl A on the spherical
grid for an analytic field, BE against a dense direct solve, and the
Gershgorin bound against dense row sums.
"""
import math

import numpy as np
import pytest

from oracle import resistivity as R
from workloads import box_faces, shell_faces


def _shell(n=(3, 4, 5)):
    rf, thf, phf = shell_faces(*n)
    return R.edge_grid("spherical", rf, thf, phf)


def _node_gradient(g, phi):
    """E = differences of a node potential phi[m0][m1][m2] along each edge."""
    p0, p1, p2 = g.periodic
    nxt = lambda a, ax, per: np.roll(a, -1, ax) if per else np.take(  # noqa: E731
        a, range(1, a.shape[ax]), axis=ax)
    cur = lambda a, ax, per: a if per else np.take(a, range(0, a.shape[ax] - 1), axis=ax)  # noqa
    return {"r": nxt(phi, 0, p0) - cur(phi, 0, p0), "t": nxt(phi, 1, p1) - cur(phi, 1, p1),
            "p": nxt(phi, 2, p2) - cur(phi, 2, p2)}


def _node_shape(g):
    return (g.shapes["t"][0], g.shapes["r"][1], g.shapes["r"][2])


@pytest.mark.parametrize("coord", ["spherical", "cartesian"])
def test_curl_of_gradient_vanishes(coord):
    f = shell_faces(3, 4, 5) if coord == "spherical" else box_faces(3, 4, 5, h=(0.5, 0.7, 0.9))
    g = R.edge_grid(coord, *f)
    phi = np.random.default_rng(1).standard_normal(_node_shape(g))
    E = R.EdgeGrid.join(_node_gradient(g, phi))
    Phi = R.curl(g, E)
    assert max(np.max(np.abs(v)) for v in Phi.values()) <= 1e-13
    assert np.max(np.abs(R.apply_F(g, E, 2.0))) <= 1e-10


def test_div_B_vanishes():
    g = _shell()
    E = np.random.default_rng(2).standard_normal(sum(g.sizes))
    P = R.curl(g, E)
    div = (P["Fr"][1:] - P["Fr"][:-1]) + (P["Ft"][:, 1:] - P["Ft"][:, :-1]) + \
        (np.roll(P["Fp"], -1, axis=2) - P["Fp"])
    assert np.max(np.abs(div)) <= 1e-13


def test_symmetric_psd_and_null_space():
    """K = C^T W C is symmetric PSD on interior edges; its null space is
    exactly the gradients of interior node potentials (no harmonic fields
    with the tangential boundary values fixed on this domain)."""
    g = _shell((3, 4, 5))
    K = R.dense_stiffness(g)
    m = R.interior_mask(g)
    Ki = K[np.ix_(m, m)]
    assert np.max(np.abs(Ki - Ki.T)) == 0.0
    ev = np.linalg.eigvalsh(Ki)
    assert ev.min() >= -1e-12 * ev.max()
    null = int(np.sum(ev <= 1e-10 * ev.max()))
    n0, n1, n2 = 3, 4, 5
    interior_nodes = (n0 - 1) * (n1 - 1) * n2  # nodes off the r and theta boundary surfaces
    assert null == interior_nodes


def test_periodic_box_spectrum():
    """On a fully periodic uniform box the generalised eigenvalues of
    K v = mu H v are 0 (gradients and the three constant fields) and, for
    each wavevector k != 0, |kappa|^2 = sum_a (2/h_a)^2 sin^2(k_a h_a / 2)
    twice (the two divergence-free polarisations)."""
    n, h = (4, 5, 3), (0.6, 0.9, 1.3)
    g = R.edge_grid("cartesian", *box_faces(*n, h=h), periodic=(True, True, True))
    K = R.dense_stiffness(g)
    Hv = R.EdgeGrid.join(g.H)
    Hs = 1.0 / np.sqrt(Hv)
    mu = np.sort(np.linalg.eigvalsh(Hs[:, None] * K * Hs[None, :]))
    ref = []
    for m0 in range(n[0]):
        for m1 in range(n[1]):
            for m2 in range(n[2]):
                kap = sum((2.0 / hh) ** 2 * math.sin(math.pi * mm / nn) ** 2
                          for hh, mm, nn in zip(h, (m0, m1, m2), n))
                ref += [0.0, kap, kap]  # gradient mode + two transverse modes
    ref = np.sort(np.array(ref))
    assert np.max(np.abs(mu - ref)) <= 1e-10 * ref.max()


def _cart(r, th, ph):
    return r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)


def _basis(th, ph):
    er = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)])
    return er, et, ep


def _A(x, y, z):
    return np.stack([y * y * z, z * z * x, x * x * y])


def _minus_curlcurl_A(x, y, z):
    return np.stack([2 * z, 2 * x, 2 * y])


def _edge_integrals(g, field, average=False):
    """Gauss-Legendre line integrals of field . t along every edge (or their
    averages over the edge length)."""
    rf, thf, phf = g.f
    rc, thc, phc = (0.5 * (a[1:] + a[:-1]) for a in (rf, thf, phf))
    xg, wg = np.polynomial.legendre.leggauss(8)
    out = {}
    n0, m1, m2 = g.shapes["r"]
    # r-edges: r from rf[i] to rf[i+1] at (thf[j], phf[k])
    I, Jn, Kn = np.meshgrid(np.arange(n0), np.arange(m1), np.arange(m2), indexing="ij")
    a, b = rf[I], rf[I + 1]
    acc = 0.0
    for s, wq in zip(xg, wg):
        r = 0.5 * (a + b) + 0.5 * (b - a) * s
        th, ph = thf[Jn], phf[Kn]
        er, _, _ = _basis(th, ph)
        acc = acc + wq * 0.5 * (b - a) * np.sum(field(*_cart(r, th, ph)) * er, axis=0)
    out["r"] = acc / (b - a) if average else acc
    m0, n1, m2 = g.shapes["t"]
    I, Jn, Kn = np.meshgrid(np.arange(m0), np.arange(n1), np.arange(m2), indexing="ij")
    a, b = thf[Jn], thf[Jn + 1]
    acc = 0.0
    for s, wq in zip(xg, wg):
        th = 0.5 * (a + b) + 0.5 * (b - a) * s
        r, ph = rf[I], phf[Kn]
        _, et, _ = _basis(th, ph)
        acc = acc + wq * 0.5 * (b - a) * r * np.sum(field(*_cart(r, th, ph)) * et, axis=0)
    out["t"] = acc / (rf[I] * (b - a)) if average else acc
    m0, m1, n2 = g.shapes["p"]
    I, Jn, Kn = np.meshgrid(np.arange(m0), np.arange(m1), np.arange(n2), indexing="ij")
    a, b = phf[Kn], phf[Kn + 1]
    acc = 0.0
    for s, wq in zip(xg, wg):
        ph = 0.5 * (a + b) + 0.5 * (b - a) * s
        r, th = rf[I], thf[Jn]
        _, _, ep = _basis(th, ph)
        acc = acc + wq * 0.5 * (b - a) * r * np.sin(th) * np.sum(
            field(*_cart(r, th, ph)) * ep, axis=0)
    out["p"] = acc / (rf[I] * np.sin(thf[Jn]) * (b - a)) if average else acc
    return out


def _shell_error(n):
    rf = np.linspace(1.0, 2.0, n + 1)
    thf = np.linspace(0.3 * math.pi, 0.7 * math.pi, n + 1)
    phf = np.linspace(0.0, 2 * math.pi, 2 * n + 1)
    g = R.edge_grid("spherical", rf, thf, phf)
    E = R.EdgeGrid.join(_edge_integrals(g, _A))
    F = g.split(R.apply_F(g, E, 1.0))
    ref = _edge_integrals(g, _minus_curlcurl_A, average=True)
    err = 0.0
    t = max(2, n // 4)
    for c in "rtp":
        got = F[c] / g.L[c]
        sl = (slice(t, -t), slice(t, -t), slice(None))
        err = max(err, np.max(np.abs(got - ref[c])[sl]))
    return err / 4.0  # |-curl curl A| <= 2 |x| ~ 4 on this shell


def test_spherical_convergence_to_curl_curl():
    errs = [_shell_error(n) for n in (8, 16, 32)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.01 and min(rates) > 1.7, (errs, rates)


def test_be_pcg_matches_direct_solve():
    g = _shell((3, 4, 5))
    rng = np.random.default_rng(3)
    E_n = rng.standard_normal(sum(g.sizes))
    eta = 0.7
    dt = 40.0 * R.gershgorin_dt_euler(g, eta)
    x, res = R.be_pcg(g, E_n, dt, eta, rtol=1e-14)
    m = R.interior_mask(g)
    K = R.dense_stiffness(g)
    Hv = R.EdgeGrid.join(g.H)
    A = np.diag(Hv[m]) + dt * eta * K[np.ix_(m, m)]
    Eb = np.where(m, 0.0, E_n)
    b = Hv[m] * E_n[m] - dt * eta * (K @ Eb)[m]
    ref = np.linalg.solve(A, b)
    assert res.converged
    assert np.max(np.abs(x[m] - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert np.array_equal(x[~m], E_n[~m])  # fixed edges untouched
    # one BE step damps: the curl energy decreases
    W = lambda E: float(E @ (K @ E))  # noqa: E731
    assert W(x) < W(E_n)


def test_gershgorin_matches_dense_row_sums():
    g = _shell((3, 4, 5))
    K = R.dense_stiffness(g)
    m = R.interior_mask(g)
    Hv = R.EdgeGrid.join(g.H)
    A = 1.3 * K[np.ix_(m, m)] / Hv[m][:, None]
    dense = 2.0 / np.max(np.sum(np.abs(A), axis=1))
    assert R.gershgorin_dt_euler(g, 1.3) == pytest.approx(dense, rel=1e-13)
    lam = np.max(np.abs(np.linalg.eigvals(A)))
    assert 2.0 / lam >= dense  # Gershgorin bounds |lambda|_max from above


@pytest.mark.parametrize("lo,hi", [((0, 0, 0), (5, 6, 7)), ((2, 3, 4), (7, 9, 12)),
                                   ((5, 6, 12), (10, 12, 19))])
def test_window_F_equals_whole_grid(lo, hi):
    """F on a window of cells, as a non-periodic grid of its own, equals the
    whole grid's F at the window's interior edges (the check the full-size
    GPU test makes on sampled windows)."""
    from helpers import resistivity_window
    faces = shell_faces(10, 12, 20)
    g = R.edge_grid("spherical", *faces)
    E = np.random.default_rng(3).standard_normal(sum(g.sizes))
    F = g.split(R.apply_F(g, E, 0.8))
    win = resistivity_window(R, "spherical", faces, g.split(E), lo, hi, 0.8)
    scale = max(np.max(np.abs(F[c])) for c in "rtp")
    for c, (Fw, m, sl) in win.items():
        assert m.any()
        assert np.max(np.abs(Fw[m] - F[c][sl][m])) <= 1e-14 * scale, c
