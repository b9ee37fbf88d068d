"""Pins for the oracle's learned factored preconditioner M^-1 = G G^T
(oracle/learned_pc.py): dense construction, SPD by construction, the
stencil applications against dense products, point Jacobi at zero outputs,
the objective's gradient against finite differences, and PCG with the
factor against a dense solve."""
import numpy as np
import pytest

from oracle import learned_pc as LP
from oracle import operator as O
from oracle import pcg
from workloads import dipole_bhat, shell_faces, temperature


def shell_system(shape, seed=1, ratio=80.0):
    rf, thf, phf = shell_faces(*shape)
    T = temperature(rf, thf, phf, seed)
    br, bt, bp = dipole_bhat(rf, thf, phf)
    op = O.assemble("spherical", rf, thf, phf, O.spitzer_tensor(T, 1e-15, br, bt, bp),
                    O.SHELL_BC, u_lo=1.5e6)
    dt = ratio * O.gershgorin_dt_euler(op)
    A19, b = O.be_system(op, T, dt)
    return op, T, dt, A19, b


def dense_A(A19, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    idx = np.arange(n).reshape(shape)
    for s, off in enumerate(O.OFFSETS):
        cols = np.roll(idx, tuple(-o for o in off), axis=(0, 1, 2))
        np.add.at(A, (idx.ravel(), cols.ravel()), A19[s].ravel())
    return A


def outputs(shape, seed, scale=0.3):
    return scale * np.random.default_rng(seed).standard_normal((4,) + tuple(shape))


def test_factor_lower_triangular_spd():
    shape = (3, 4, 5)  # phi periodic with 5 cells: the seam must not couple
    _, T, _, A19, _ = shell_system(shape)
    g = LP.factor_entries(outputs(shape, 2), A19[0])
    G = LP.dense_G(g)
    assert np.all(np.triu(G, 1) == 0.0)
    assert np.all(np.diag(G) > 0.0)
    M = G @ G.T
    assert np.array_equal(M, M.T) or np.max(np.abs(M - M.T)) <= 1e-15 * np.max(np.abs(M))
    assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > 0.0
    # the entries are the defined functions of the outputs
    o = outputs(shape, 2)
    d = 1.0 / np.sqrt(A19[0])
    assert np.allclose(np.diag(G).reshape(shape), d * np.exp(o[0]), rtol=1e-15, atol=0)
    # no coupling across the periodic seam, across the r and theta walls
    assert np.all(g[3][:, :, 0] == 0.0) and np.all(g[1][0] == 0.0) and np.all(g[2][:, 0] == 0.0)


def test_stencil_applications_match_dense():
    shape = (3, 4, 5)
    _, _, _, A19, _ = shell_system(shape)
    g = LP.factor_entries(outputs(shape, 3), A19[0])
    G = LP.dense_G(g)
    x = np.random.default_rng(4).standard_normal(shape)
    for got, ref in ((LP.apply_G(g, x), G @ x.ravel()), (LP.apply_GT(g, x), G.T @ x.ravel()),
                     (LP.apply_Minv(g, x), G @ (G.T @ x.ravel()))):
        assert np.max(np.abs(got.ravel() - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_zero_outputs_is_point_jacobi():
    shape = (4, 6, 8)
    op, T, dt, A19, _ = shell_system(shape)
    g = LP.factor_entries(np.zeros((4,) + shape), A19[0])
    r = np.random.default_rng(5).standard_normal(shape)
    assert np.max(np.abs(LP.apply_Minv(g, r) - r / A19[0])) <= 1e-15 * np.max(np.abs(r / A19[0]))
    a = LP.be_pcg_factor(op, T, dt, g, rtol=1e-10, keep=(1, 3, 8))
    b = pcg.be_pcg(op, T, dt, "jacobi", rtol=1e-10, keep=(1, 3, 8))
    assert a.iters == b.iters
    for xa, xb in zip(a.iterates, b.iterates):
        assert np.max(np.abs(xa - xb)) <= 1e-13 * np.max(np.abs(xb))


def _loss_of_outputs(o, A19, z):
    g = LP.factor_entries(o, A19[0])
    return LP.loss_and_grad(g, lambda v: O.apply19(A19, v), z)[0]


def test_objective_matches_definition_and_gradient_matches_differences():
    shape = (2, 3, 4)
    _, _, _, A19, _ = shell_system(shape, ratio=20.0)
    rng = np.random.default_rng(6)
    o = 0.2 * rng.standard_normal((4,) + shape)
    z = rng.choice([-1.0, 1.0], size=shape)
    g = LP.factor_entries(o, A19[0])
    L, dg = LP.loss_and_grad(g, lambda v: O.apply19(A19, v), z)
    # L against the dense definition ||G^T A G z - z||^2 / N
    G, A = LP.dense_G(g), dense_A(A19, shape)
    e = G.T @ A @ G @ z.ravel() - z.ravel()
    assert abs(L - e @ e / z.size) <= 1e-13 * L
    # dL/dG on the pattern against central differences in the entries
    h = 1e-6
    for q in range(4):
        for idx in [(0, 0, 0), (1, 2, 3), (1, 1, 0), (0, 2, 1)]:
            if q > 0 and not LP.has_lower(shape)[q - 1][idx]:
                assert dg[q][idx] == 0.0
                continue
            gp, gm = g.copy(), g.copy()
            gp[q][idx] += h
            gm[q][idx] -= h
            fd = (LP.loss_and_grad(gp, lambda v: O.apply19(A19, v), z)[0]
                  - LP.loss_and_grad(gm, lambda v: O.apply19(A19, v), z)[0]) / (2 * h)
            assert abs(fd - dg[q][idx]) <= 1e-6 * np.max(np.abs(dg)), (q, idx)
    # dL/do (through the entry maps) against central differences in o
    do = LP.grad_outputs(dg, g, A19[0])
    for q in range(4):
        for idx in [(0, 1, 2), (1, 0, 3), (1, 2, 1)]:
            op_, om = o.copy(), o.copy()
            op_[q][idx] += h
            om[q][idx] -= h
            fd = (_loss_of_outputs(op_, A19, z) - _loss_of_outputs(om, A19, z)) / (2 * h)
            assert abs(fd - do[q][idx]) <= 1e-6 * np.max(np.abs(do)), (q, idx)


def test_objective_vanishes_for_an_exact_inverse_factor():
    """With A = L L^T (Cholesky) and G = L^-T the preconditioned operator is
    the identity, so L(z) = 0 -- checked on the dense formula the gradient
    derivation starts from (G^T A G = I)."""
    shape = (2, 3, 4)
    _, _, _, A19, _ = shell_system(shape, ratio=20.0)
    A = dense_A(A19, shape)
    Lc = np.linalg.cholesky(A)
    G = np.linalg.inv(Lc).T
    assert np.max(np.abs(G.T @ A @ G - np.eye(A.shape[0]))) <= 1e-12


def test_pcg_with_factor_equals_dense_solve():
    shape = (4, 6, 8)
    op, T, dt, A19, b = shell_system(shape)
    g = LP.factor_entries(outputs(shape, 7, scale=0.2), A19[0])
    res = LP.be_pcg_factor(op, T, dt, g, rtol=1e-13)
    A = dense_A(A19, shape)
    xd = np.linalg.solve(A, b.ravel()).reshape(shape)
    assert res.converged
    assert np.max(np.abs(res.x - xd)) <= 10 * np.linalg.cond(A) * 1e-13 * np.max(np.abs(xd))


@pytest.mark.parametrize("seed", [8, 9])
def test_preconditioned_operator_spectrum_is_positive(seed):
    """G^T A G is symmetric positive definite (A SPD, G nonsingular), so PCG
    with M^-1 = G G^T cannot break down: checked by dense eigenvalues."""
    shape = (3, 3, 4)
    _, _, _, A19, _ = shell_system(shape)
    g = LP.factor_entries(outputs(shape, seed, scale=1.0), A19[0])
    G, A = LP.dense_G(g), dense_A(A19, shape)
    P = G.T @ A @ G
    assert np.min(np.linalg.eigvalsh(0.5 * (P + P.T))) > 0.0
