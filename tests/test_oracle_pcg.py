"""Pins for the oracle's backward Euler + PCG and block ILU0 (Sec. 2, App. A)."""
import math

import numpy as np
import pytest

from oracle import ilu0
from oracle import operator as O
from oracle import pcg
from workloads import shell_faces, temperature, dipole_bhat, box_faces, make_workload


def shell_op(shape, seed=1, bc=O.SHELL_BC):
    rf, thf, phf = shell_faces(*shape)
    T = temperature(rf, thf, phf, seed)
    br, bt, bp = dipole_bhat(rf, thf, phf)
    D = O.spitzer_tensor(T, 1e-15, br, bt, bp)
    return O.assemble("spherical", rf, thf, phf, D, bc, u_lo=1.5e6), T


@pytest.mark.parametrize("precond", ["jacobi", "ilu0", "none"])
def test_be_pcg_equals_dense_solve(precond):
    op, T = shell_op((4, 6, 8))
    dt = 80.0 * O.gershgorin_dt_euler(op)
    res = pcg.be_pcg(op, T, dt, precond, rtol=1e-13, block=(2, 3, 4))
    A19, b = O.be_system(op, T, dt)
    n = T.size
    A = np.zeros((n, n))
    idx = np.arange(n).reshape(T.shape)
    for s, off in enumerate(O.OFFSETS):
        cols = np.roll(idx, tuple(-o for o in off), axis=(0, 1, 2))
        np.add.at(A, (idx.ravel(), cols.ravel()), A19[s].ravel())
    xd = np.linalg.solve(A, b.ravel()).reshape(T.shape)
    cond = np.linalg.cond(A)
    assert res.converged
    assert np.max(np.abs(res.x - xd)) <= 10 * cond * 1e-13 * np.max(np.abs(xd))
    # the BE step itself: (u^{n+1} - u^n)/dt = F(u^{n+1})  (Eq. BE)
    lhs = (res.x - T) / dt
    rhs = O.apply_F(op, res.x)
    assert np.max(np.abs(lhs - rhs)) <= 1e-7 * np.max(np.abs(rhs))


def test_be_single_fourier_mode_one_iteration():
    """On a periodic box with constant D, BE maps a cosine mode to
    mode / (1 - dt lambda); Jacobi-PCG from 0 gets it in one iteration."""
    n, h = (8, 10, 12), (1.0, 1.0, 1.0)
    bvec = np.array([0.6, 0.0, 0.8])
    D = {(a, b): np.full(n, bvec[a] * bvec[b]) for a in range(3) for b in range(a, 3)}
    op = O.assemble("cartesian", *box_faces(*n, h=h), D, (O.PERIODIC,) * 6)
    theta = [2 * math.pi * m / nn for m, nn in zip((2, 3, 4), n)]
    idx = np.meshgrid(*[np.arange(nn) for nn in n], indexing="ij")
    u = np.cos(sum(t * i for t, i in zip(theta, idx)))
    lam = -sum(4 * bvec[a] ** 2 * math.sin(theta[a] / 2) ** 2 for a in range(3)) - sum(
        2 * bvec[a] * bvec[b] * math.sin(theta[a]) * math.sin(theta[b])
        for a in range(3) for b in range(a + 1, 3))
    dt = 50 * O.gershgorin_dt_euler(op)
    res = pcg.be_pcg(op, u, dt, "jacobi", rtol=1e-14, x0=np.zeros(n))
    assert res.iters == 1
    assert np.max(np.abs(res.x - u / (1 - dt * lam))) <= 1e-13


def test_true_residual_meets_tolerance():
    op, T = shell_op((6, 8, 12))
    dt = 200 * O.gershgorin_dt_euler(op)
    for pc in ("jacobi", "ilu0"):
        res = pcg.be_pcg(op, T, dt, pc, rtol=1e-9, block=(4, 4, 4))
        A19, b = O.be_system(op, T, dt)
        true = np.linalg.norm(b - O.apply19(A19, res.x)) / np.linalg.norm(b)
        assert res.converged and true <= 2e-9


def test_ilu0_unit_blocks_equal_jacobi():
    """Sec. 2.3: with one grid point per subdomain PC2 is PC1."""
    op, T = shell_op((4, 6, 8))
    A19, b = O.be_system(op, T, 60 * O.gershgorin_dt_euler(op))
    fac = ilu0.factor(A19, (1, 1, 1))
    r = np.random.default_rng(0).standard_normal(T.shape)
    z = ilu0.apply(fac, r)
    # the triangular solver divides by the pivot up to its own rounding (1 ulp)
    jac = r / A19[0]
    assert np.max(np.abs(z - jac) / np.abs(jac)) <= 2.3e-16


def test_ilu0_reproduces_A_on_pattern():
    """Zero-fill ILU: (L U)_ij = A_ij for every (i, j) in the pattern."""
    op, T = shell_op((4, 6, 8))
    A19, b = O.be_system(op, T, 60 * O.gershgorin_dt_euler(op))
    block = (3, 4, 5)
    fac = ilu0.factor(A19, block)
    for gi, grp in enumerate(fac["groups"]):
        for bi in range(len(grp["origins"])):
            L, U = ilu0.lower_upper_dense(fac, gi, bi)
            Ab, pat = ilu0.block_dense_A(A19, block, grp["origins"][bi])
            LU = L @ U
            mask = np.zeros_like(Ab, dtype=bool)
            for i, d in enumerate(pat):
                mask[i, list(d.keys())] = True
            assert np.max(np.abs((LU - Ab)[mask])) <= 1e-12 * np.abs(Ab).max()


def test_ilu0_on_chain_block_is_exact_lu():
    """A 1 x 1 x m block is tridiagonal: ILU0 needs no fill and equals the
    exact LU factorisation (compared with the Cholesky factor)."""
    op, T = shell_op((3, 4, 10))
    A19, b = O.be_system(op, T, 60 * O.gershgorin_dt_euler(op))
    block = (1, 1, 10)
    fac = ilu0.factor(A19, block)
    L, U = ilu0.lower_upper_dense(fac, 0, 5)
    Ab, _ = ilu0.block_dense_A(A19, block, fac["groups"][0]["origins"][5])
    C = np.linalg.cholesky(Ab)
    d = np.diag(C)
    assert np.allclose(L, C / d[None, :], rtol=1e-12, atol=1e-14)
    assert np.allclose(U, (C * d[None, :]).T, rtol=1e-12, atol=1e-12 * np.abs(Ab).max())


def test_ilu0_symmetric_A_gives_U_equal_D_Lt():
    op, T = shell_op((4, 6, 8))
    A19, b = O.be_system(op, T, 60 * O.gershgorin_dt_euler(op))
    fac = ilu0.factor(A19, (4, 6, 8))
    L, U = ilu0.lower_upper_dense(fac, 0, 0)
    Dg = np.diag(np.diag(U))
    assert np.max(np.abs(U - Dg @ L.T)) <= 1e-12 * np.abs(U).max()


def test_ilu0_iterations_fall_with_block_size():
    """PC2 weakens as the subdomains shrink (Sec. 2.3, Sec. 7); block 1 = PC1."""
    op, T = shell_op((8, 16, 16))
    dt = 200 * O.gershgorin_dt_euler(op)
    its = {}
    for blk in [(1, 1, 1), (2, 2, 2), (4, 4, 4), (8, 8, 8)]:
        its[blk] = pcg.be_pcg(op, T, dt, "ilu0", rtol=1e-9, block=blk).iters
    jac = pcg.be_pcg(op, T, dt, "jacobi", rtol=1e-9).iters
    assert its[(1, 1, 1)] == jac
    assert its[(1, 1, 1)] > its[(2, 2, 2)] > its[(4, 4, 4)] >= its[(8, 8, 8)]


def test_workload_shell32_solvers_agree():
    """Config-1 style step: RKL2, BE-Jacobi and BE-ILU0 all run; BE solutions
    agree within the solver tolerance."""
    w = make_workload("shell32")
    D = O.spitzer_tensor(w["T"], w["kappa0"], w["br"], w["bt"], w["bp"])
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], D, O.SHELL_BC, u_lo=w["T_inner"])
    dt = 50 * O.gershgorin_dt_euler(op)
    rj = pcg.be_pcg(op, w["T"], dt, "jacobi", rtol=1e-9)
    ri = pcg.be_pcg(op, w["T"], dt, "ilu0", rtol=1e-9)
    assert rj.converged and ri.converged and ri.iters < rj.iters
    assert np.max(np.abs(rj.x - ri.x)) <= 1e-6 * np.max(np.abs(rj.x))


@pytest.mark.parametrize("shape,block", [((4, 6, 8), (3, 4, 5)), ((8, 16, 16), (8, 8, 8)),
                                         ((5, 7, 9), (2, 3, 4))])
def test_ilu0_apply_equals_dense_solve_per_block(shape, block):
    """z = (L U)^-1 r on every block, L and U taken densely from the factor and
    solved by a dense LU of their product: a substitution that used the wrong
    entries (e.g. r_j instead of z_j, or the diagonal in the forward sweep)
    fails here, including on ragged blocks."""
    op, T = shell_op(shape)
    A19, _ = O.be_system(op, T, 60 * O.gershgorin_dt_euler(op))
    fac = ilu0.factor(A19, block)
    r = np.random.default_rng(3).standard_normal(T.shape)
    z = ilu0.apply(fac, r)
    nblocks = 0
    for gi, grp in enumerate(fac["groups"]):
        idx = grp["idx"]
        for bi in range(len(grp["origins"])):
            L, U = ilu0.lower_upper_dense(fac, gi, bi)
            rb = r[idx[0][bi], idx[1][bi], idx[2][bi]]
            zd = np.linalg.solve(L @ U, rb)
            zb = z[idx[0][bi], idx[1][bi], idx[2][bi]]
            assert np.max(np.abs(zb - zd)) <= 1e-13 * np.max(np.abs(zd))
            nblocks += 1
    assert nblocks == np.prod([-(-n // b) for n, b in zip(shape, block)])


def test_ilu0_whole_block_is_dense_zero_fill_lu():
    """One block covering a tiny grid: the factor equals a dense textbook
    zero-fill ILU (IKJ elimination on a dense copy, fill outside the pattern
    discarded) of the dense block matrix."""
    shape = (3, 4, 5)
    op, T = shell_op(shape)
    A19, _ = O.be_system(op, T, 60 * O.gershgorin_dt_euler(op))
    fac = ilu0.factor(A19, shape)
    Ab, pat = ilu0.block_dense_A(A19, shape, (0, 0, 0))
    n = Ab.shape[0]
    mask = Ab != 0
    for i, d in enumerate(pat):
        mask[i, list(d.keys())] = True
    W = Ab.copy()
    for i in range(1, n):
        for k in range(i):
            if not mask[i, k]:
                continue
            W[i, k] /= W[k, k]
            W[i, k + 1:] -= W[i, k] * W[k, k + 1:] * mask[i, k + 1:]
    L, U = ilu0.lower_upper_dense(fac, 0, 0)
    assert np.max(np.abs(np.tril(W, -1) - (L - np.eye(n)))) <= 1e-13 * np.abs(Ab).max()
    assert np.max(np.abs(np.triu(W) - U)) <= 1e-13 * np.abs(Ab).max()
