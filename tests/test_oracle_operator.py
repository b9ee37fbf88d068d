"""Pins for the oracle's operator F(u), Gershgorin dt_Euler and geometry.

Each check is independent of the oracle's own assembly code: a brute-force
loop energy, closed-form Fourier symbols, polynomial exactness, grid
convergence to the continuous operator, and invariants of the paper's
operator (self-adjointness, conservation, negative semi-definiteness).
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import operator as O
from workloads import make_workload, shell_faces, temperature, dipole_bhat, box_faces
from workloads import random_unit_vectors

ZF, DI, PE = O.ZEROFLUX, O.DIRICHLET, O.PERIODIC


def tiny_shell(nr=4, nth=5, nph=6, seed=3, bc=O.SHELL_BC, u_lo=1.5e6):
    rf, thf, phf = shell_faces(nr, nth, nph)
    T = temperature(rf, thf, phf, seed)
    br, bt, bp = dipole_bhat(rf, thf, phf)
    D = O.spitzer_tensor(T, 1e-15, br, bt, bp)
    return O.assemble("spherical", rf, thf, phf, D, bc, u_lo=u_lo), (rf, thf, phf, D)


# --------------------------------------------------------------------------------------------
# brute-force energy: the definition E(u), written as plain loops over faces and edges
# --------------------------------------------------------------------------------------------
def loop_energy(coord, f0, f1, f2, D, bc, u, u_lo=0.0):
    periodic = tuple(bc[2 * a] == PE for a in range(3))
    G = geo.geometry(coord, f0, f1, f2, periodic)
    n = G["shape"]
    V, A, dl = G["V"], G["A"], G["dl"]
    E = 0.0

    def nb(c, a, s=1):
        m = list(c)
        m[a] += s
        if periodic[a]:
            m[a] %= n[a]
        elif not (0 <= m[a] < n[a]):
            return None
        return tuple(m)

    for c in np.ndindex(*n):
        for a in range(3):
            c1 = nb(c, a)
            if c1 is None:
                continue
            w = A[a][c] * 0.5 * (D[(a, a)][c] + D[(a, a)][c1]) / dl[a][c]
            E += 0.5 * w * (u[c1] - u[c]) ** 2
        for a in range(3):
            for b in range(a + 1, 3):
                c10, c01 = nb(c, a), nb(c, b)
                if c10 is None or c01 is None:
                    continue
                c11 = nb(c10, b)
                cells = (c, c10, c01, c11)
                W = sum(V[x] for x in cells) / 4
                Dab = sum(D[(a, b)][x] for x in cells) / 4
                X = 0.5 * ((u[c10] - u[c]) / dl[a][c] + (u[c11] - u[c01]) / dl[a][c01])
                Y = 0.5 * ((u[c01] - u[c]) / dl[b][c] + (u[c11] - u[c10]) / dl[b][c10])
                E += W * Dab * X * Y
    if bc[0] == DI:
        for j in range(n[1]):
            for k in range(n[2]):
                wb = G["Ab"][0][j, k] * D[(0, 0)][0, j, k] / G["db"][0]
                E += 0.5 * wb * (u_lo - u[0, j, k]) ** 2
    return E


@pytest.mark.parametrize("bc", [O.SHELL_BC, (ZF, ZF, ZF, ZF, ZF, ZF)])
def test_assembly_equals_energy_hessian(bc):
    """S = -Hessian(E), g = -grad E(0), by exact second differences of the loop energy."""
    u_lo = 2.0
    op, (rf, thf, phf, D) = tiny_shell(3, 4, 5, bc=bc, u_lo=u_lo)
    # rescale to O(1) so the second differences are well conditioned
    scale = 1.0 / np.max(np.abs(D[(0, 0)]))
    D = {k: v * scale for k, v in D.items()}
    op = O.assemble("spherical", rf, thf, phf, D, bc, u_lo=u_lo)
    n = int(np.prod(op.shape))
    E = lambda u: loop_energy("spherical", rf, thf, phf, D, bc, u.reshape(op.shape), u_lo)  # noqa
    E0 = E(np.zeros(n))
    Ei = np.array([E(np.eye(n)[i]) for i in range(n)])
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            e = np.zeros(n)
            e[i] += 1.0
            e[j] += 1.0
            H[i, j] = H[j, i] = E(e) - Ei[i] - Ei[j] + E0
    Ss = O.dense_S(op)
    assert np.max(np.abs(Ss + H)) <= 1e-10 * np.max(np.abs(H))
    Em = np.array([E(-np.eye(n)[i]) for i in range(n)])
    grad0 = (Ei - Em) / 2.0
    assert np.max(np.abs(op.g.ravel() + grad0)) <= 1e-10 * max(1.0, np.max(np.abs(grad0)))


def test_nineteen_point_pattern_with_tilted_dipole():
    """A tilted dipole gives all 19 couplings (Appendix B: p = 19) in the interior."""
    op, _ = tiny_shell(5, 5, 6)
    interior = op.S19[:, 1:-1, 1:-1, :]
    assert np.all(np.abs(interior) > 0)


def test_self_adjoint_volume_weighted():
    """u . V F(v) = v . V F(u) for the homogeneous part (self-adjointness)."""
    w = make_workload("shell32")
    D = O.spitzer_tensor(w["T"], w["kappa0"], w["br"], w["bt"], w["bp"])
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], D, O.SHELL_BC, u_lo=w["T_inner"])
    rng = np.random.default_rng(7)
    u, v = rng.standard_normal((2,) + op.shape)
    lhs = np.sum(u * op.V * O.apply_M(op, v))
    rhs = np.sum(v * op.V * O.apply_M(op, u))
    scale = np.sum(np.abs(u * op.V * O.apply_M(op, v)))
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_negative_semidefinite_tiny_config_fields():
    """Spectrum of V^-1/2 S V^-1/2 <= 0 on tiny grids built like the workloads."""
    for seed, shape in [(0, (4, 6, 8)), (5, (5, 5, 6)), (11, (3, 7, 8))]:
        op, _ = tiny_shell(*shape, seed=seed)
        S = O.dense_S(op)
        v = 1.0 / np.sqrt(op.V.ravel())
        lam = np.linalg.eigvalsh(v[:, None] * S * v[None, :])
        assert lam.max() <= 1e-12 * np.abs(lam).max()


def test_random_bhat_is_not_guaranteed_nsd_but_conservative():
    """The form is exact-symmetric and conservative for any b; uncorrelated
    random b per cell may break semi-definiteness (documented risk)."""
    rf, thf, phf = shell_faces(4, 6, 8)
    T = temperature(rf, thf, phf, 2)
    br, bt, bp = random_unit_vectors(T.shape, 9)
    D = O.spitzer_tensor(T, 1e-15, br, bt, bp)
    op = O.assemble("spherical", rf, thf, phf, D, (ZF,) * 4 + (PE, PE))
    S = O.dense_S(op)
    assert np.allclose(S, S.T, rtol=0, atol=1e-14 * np.abs(S).max())
    assert np.max(np.abs(S.sum(axis=1))) <= 1e-12 * np.abs(S).max()


def test_conservation_zero_flux():
    """sum_c V_c F(u)_c = 0 when every boundary is zero-flux."""
    w = make_workload("shell32")
    D = O.spitzer_tensor(w["T"], w["kappa0"], w["br"], w["bt"], w["bp"])
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], D, (ZF,) * 4 + (PE, PE))
    F = O.apply_F(op, w["T"])
    tot = np.sum(op.V * F)
    assert abs(tot) <= 1e-13 * np.sum(np.abs(op.V * F))


def test_dirichlet_constant_state_is_steady():
    """u = u_b everywhere is a steady state; u = const != u_b only drives the
    Dirichlet layer, by w_b (u_b - u) / V."""
    op, (rf, thf, phf, D) = tiny_shell(4, 5, 6, u_lo=3.0)
    F = O.apply_F(op, np.full(op.shape, 3.0))
    assert np.max(np.abs(F)) <= 1e-12 * np.max(np.abs(op.S19[0] / op.V))
    F2 = O.apply_F(op, np.full(op.shape, 1.0))
    assert np.max(np.abs(F2[1:])) <= 1e-12 * np.max(np.abs(F2))
    G = geo.geometry("spherical", rf, thf, phf, (False, False, True))
    wb = G["Ab"][0] * D[(0, 0)][0] / G["db"][0]
    assert np.allclose(F2[0], wb * 2.0 / G["V"][0], rtol=1e-13)


def _box_op(n, h, D_const, bc):
    f = box_faces(*n, h=h)
    shape = tuple(n)
    D = {k: np.full(shape, v) for k, v in D_const.items()}
    return O.assemble("cartesian", *f, D, bc), f


def fourier_symbol(theta, h, Dc):
    """Closed form of the discrete operator's eigenvalue for constant D on a
    periodic uniform box (derived from E by Fourier analysis)."""
    lam = 0.0
    for a in range(3):
        lam -= 4.0 * Dc[(a, a)] * math.sin(theta[a] / 2) ** 2 / h[a] ** 2
    for a in range(3):
        for b in range(a + 1, 3):
            lam -= 2.0 * Dc[(a, b)] * math.sin(theta[a]) * math.sin(theta[b]) / (h[a] * h[b])
    return lam


def _rank1_D(bvec, kappa=1.7):
    bvec = np.asarray(bvec, float) / np.linalg.norm(bvec)
    return {(a, b): kappa * bvec[a] * bvec[b] for a in range(3) for b in range(a, 3)}


@pytest.mark.parametrize("modes", [(1, 2, 3), (4, 0, 5), (3, 4, 1), (0, 5, 6), (4, 5, 6)])
def test_fourier_symbol_periodic_box(modes):
    n, h = (8, 10, 12), (0.7, 1.1, 0.9)
    Dc = _rank1_D([0.3, -0.8, 0.5])
    op, f = _box_op(n, h, Dc, (PE,) * 6)
    theta = [2 * math.pi * m / nn for m, nn in zip(modes, n)]
    idx = np.meshgrid(*[np.arange(nn) for nn in n], indexing="ij")
    u = np.cos(sum(t * i for t, i in zip(theta, idx)))
    lam = fourier_symbol(theta, h, Dc)
    F = O.apply_F(op, u)
    assert np.max(np.abs(F - lam * u)) <= 1e-12 * max(1.0, abs(lam))


def test_quadratic_exactness_uniform_box():
    """On a uniform box with constant full D, F(u) = tr(D Q) exactly for
    u = 1/2 x^T Q x + c.x at every cell whose neighbours all exist."""
    n, h = (6, 7, 8), (0.5, 0.8, 0.6)
    rng = np.random.default_rng(3)
    Bm = rng.standard_normal((3, 3))
    Dm = Bm @ Bm.T + 0.5 * np.eye(3)
    Dc = {(a, b): Dm[a, b] for a in range(3) for b in range(a, 3)}
    op, f = _box_op(n, h, Dc, (ZF,) * 6)
    Q = rng.standard_normal((3, 3))
    Q = Q + Q.T
    cvec = rng.standard_normal(3)
    x = np.meshgrid(*[geo.centres(ff) for ff in f], indexing="ij")
    u = sum(0.5 * Q[a, b] * x[a] * x[b] for a in range(3) for b in range(3)) + sum(
        cvec[a] * x[a] for a in range(3))
    F = O.apply_F(op, u)
    exact = np.trace(Dm @ Q)
    assert np.max(np.abs(F[1:-1, 1:-1, 1:-1] - exact)) <= 1e-10 * (1 + abs(exact))


def _shell_F_error(n, mode):
    rf = np.linspace(1.0, 2.0, n + 1)
    thf = np.linspace(0.3 * math.pi, 0.7 * math.pi, n + 1)
    phf = np.linspace(0.0, 2 * math.pi, 2 * n + 1)
    shape = (n, n, 2 * n)
    x, y, z = geo.cartesian_position("spherical", rf, thf, phf)
    Q = np.array([[2.0, 1.0, 0.0], [1.0, 4.0, -0.5], [0.0, -0.5, 6.0]])
    u = 0.5 * (Q[0, 0] * x * x + Q[1, 1] * y * y + Q[2, 2] * z * z) + Q[0, 1] * x * y \
        + Q[0, 2] * x * z + Q[1, 2] * y * z
    if mode == "isotropic":
        D = O.isotropic_tensor(shape, 1.0)
        exact = np.trace(Q)
    else:
        bc_ = np.array([0.36, -0.48, 0.8])  # constant Cartesian unit vector
        er, et, ep = geo.local_basis("spherical", rf, thf, phf)
        comps = [sum(bc_[m] * e[m] for m in range(3)) for e in (er, et, ep)]
        D = {(a, b): comps[a] * comps[b] for a in range(3) for b in range(a, 3)}
        exact = bc_ @ Q @ bc_
    op = O.assemble("spherical", rf, thf, phf, D, (ZF,) * 4 + (PE, PE))
    F = O.apply_F(op, u)
    return np.max(np.abs(F[2:-2, 2:-2, :] - exact)) / abs(exact)


@pytest.mark.parametrize("mode", ["isotropic", "anisotropic"])
def test_spherical_grid_convergence(mode):
    """On the spherical grid F(u) converges to div(D grad u) for a Cartesian
    quadratic u (isotropic D = I, and D = b b^T with a constant Cartesian b)."""
    errs = [_shell_F_error(n, mode) for n in (8, 16, 32)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.02
    assert min(rates) > 0.9, (errs, rates)


def test_gershgorin_bounds_spectrum():
    """|lambda|_max <= G and G <= sqrt(19) |lambda|_max (Appendix B, Eq. gstb
    and the sqrt(p) accuracy it quotes)."""
    for seed, shape in [(0, (4, 6, 8)), (4, (5, 4, 6))]:
        op, _ = tiny_shell(*shape, seed=seed)
        S = O.dense_S(op)
        v = 1.0 / np.sqrt(op.V.ravel())
        lam = np.abs(np.linalg.eigvalsh(v[:, None] * S * v[None, :])).max()
        G = 2.0 / O.gershgorin_dt_euler(op)
        assert G >= lam * (1 - 1e-12)
        assert G <= math.sqrt(19) * lam


def test_gershgorin_tighter_than_ktilde_for_anisotropic():
    """Appendix B: the k~ estimate underestimates dt_Euler for anisotropic
    diffusion; the Gershgorin estimate is the larger (closer) one."""
    w = make_workload("shell32")
    D = O.spitzer_tensor(w["T"], w["kappa0"], w["br"], w["bt"], w["bp"])
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], D, O.SHELL_BC, u_lo=w["T_inner"])
    kappa = w["kappa0"] * w["T"] ** 2.5
    dt_g = O.gershgorin_dt_euler(op)
    dt_k = O.ktilde_dt_euler("spherical", w["rf"], w["thf"], w["phf"], kappa.max())
    assert dt_k < dt_g
