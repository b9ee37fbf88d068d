"""GPU parity of the resistive curl-curl operator and its BE + PC1 solve
(sts_set_resistivity, apply_F_resistivity, resistivity_dt_euler,
resistivity_be_pcg_solve) against the oracle (oracle/resistivity.py):
F and dt_E to 1e-12 relative, PCG iterates to 1e-12 relative, converged
solves with iteration counts within one and within the residual bound of
each other, on small and ragged shells, boxes with every periodicity
pattern, and the 128 x 128 x 256 shell (12.7M edges, the whole field
checked); at 256 x 256 x 512 (101.2M edges, the benchmark's launch), F
against the oracle on windows of cells and the curl of a gradient on every
edge."""
import numpy as np
import pytest

from helpers import relmax, resistivity_window
from oracle import resistivity as R
from workloads import box_faces, make_workload, shell_faces

pytestmark = pytest.mark.gpu
SHELL_BC = (1, 0, 0, 0, 2, 2)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _pair(sts, coord, f, bc, eta):
    periodic = tuple(bc[2 * a] == 2 for a in range(3))
    g = R.edge_grid(coord, *f, periodic=periodic)
    ctx = sts.Context(sts.SPHERICAL if coord == "spherical" else sts.CARTESIAN, *f, bc)
    ctx.set_resistivity(eta)
    assert ctx.resistivity_sizes() == tuple(g.sizes)
    return g, ctx


def _smooth_E(g, seed):
    """A rough-plus-smooth edge field: random values plus a smooth mode."""
    rng = np.random.default_rng(seed)
    n = sum(g.sizes)
    return rng.standard_normal(n) + 3.0 * np.sin(np.arange(n) * 2e-3)


CASES = [
    ("spherical", (6, 7, 9), SHELL_BC),
    ("spherical", (5, 13, 70), SHELL_BC),
    ("spherical", (1, 3, 4), SHELL_BC),
    ("spherical", (4, 5, 6), (0, 0, 0, 0, 0, 0)),
    ("cartesian", (5, 6, 7), (2, 2, 2, 2, 2, 2)),
    ("cartesian", (5, 6, 7), (0, 0, 2, 2, 0, 0)),
    ("cartesian", (4, 3, 5), (2, 2, 0, 0, 2, 2)),
    # several tiles, theta strips and runs of the fused sweep: phi wrapping
    # across tiles, theta wrapping across strips, r wrapping at a run's start,
    # a ragged last phi tile
    ("spherical", (9, 37, 130), SHELL_BC),
    ("cartesian", (5, 19, 70), (0, 0, 2, 2, 2, 2)),
    ("cartesian", (6, 9, 66), (2, 2, 0, 0, 0, 0)),
]


def _faces(coord, n):
    return shell_faces(*n) if coord == "spherical" else box_faces(*n, h=(0.6, 0.9, 1.3))


@pytest.mark.parametrize("coord,n,bc", CASES, ids=[f"{c}-{n}-{b}" for c, n, b in CASES])
def test_F_and_dt_euler(gpu_lib, coord, n, bc):
    g, ctx = _pair(gpu_lib, coord, _faces(coord, n), bc, 0.7)
    E = _smooth_E(g, sum(n))
    got = _host(ctx.apply_F_resistivity(_cuda(E)))
    ref = R.apply_F(g, E, 0.7)
    assert relmax(got, ref) <= 1e-12
    m = R.interior_mask(g)
    if m.any():
        assert ctx.resistivity_dt_euler() == pytest.approx(R.gershgorin_dt_euler(g, 0.7),
                                                           rel=1e-12)


def test_F_of_gradient_vanishes(gpu_lib):
    """The curl of a discrete gradient is zero on the GPU too."""
    f = shell_faces(8, 9, 16)
    g, ctx = _pair(gpu_lib, "spherical", f, SHELL_BC, 1.0)
    phi = np.random.default_rng(0).standard_normal((9, 10, 16))
    E = R.EdgeGrid.join({"r": phi[1:] - phi[:-1], "t": phi[:, 1:] - phi[:, :-1],
                         "p": np.roll(phi, -1, axis=2) - phi})
    F = _host(ctx.apply_F_resistivity(_cuda(E)))
    scale = np.max(np.abs(R.apply_F(g, np.random.default_rng(1).standard_normal(E.size), 1.0)))
    assert np.max(np.abs(F)) <= 1e-12 * scale


@pytest.mark.parametrize("coord,n,bc", CASES[:2] + CASES[4:5],
                         ids=[f"{c}-{n}-{b}" for c, n, b in CASES[:2] + CASES[4:5]])
@pytest.mark.parametrize("ratio", [5.0, 60.0])
def test_be_pcg(gpu_lib, coord, n, bc, ratio):
    """Converged solutions: the same iteration count (within one), and both
    within the residual bound of the exact solution: ||b - A x|| <= rtol ||b||
    and A >= H give ||x_gpu - x_ref|| <= 2 rtol ||b|| / min H.  (After
    ~100 iterations the two recurrences' rounding no longer agrees to 1e-12;
    the iterates themselves are compared in test_be_pcg_iterates.)"""
    g, ctx = _pair(gpu_lib, coord, _faces(coord, n), bc, 0.7)
    E_n = _smooth_E(g, 7)
    dt = ratio * R.gershgorin_dt_euler(g, 0.7)
    rtol = 1e-10
    ref, res = R.be_pcg(g, E_n, dt, 0.7, rtol=rtol)
    x = _cuda(E_n)
    it, rel, st = ctx.resistivity_be_pcg_solve(_cuda(E_n), x, dt, rtol=rtol)
    assert st == 0 and abs(it - res.iters) <= 1 and rel <= rtol
    got = _host(x)
    _, b, _, m = R.be_system(g, E_n, dt, 0.7)
    hmin = np.min(R.EdgeGrid.join(g.H)[m])
    assert np.linalg.norm(got[m] - ref[m]) <= 2.0 * rtol * np.linalg.norm(b) / hmin
    assert np.array_equal(got[~m], E_n[~m])


ITER_CASES = [("spherical", (6, 7, 9), SHELL_BC, k) for k in (1, 5, 12)] + \
    [c + (k,) for c in CASES[7:] for k in (1, 12)]


@pytest.mark.parametrize("coord,n,bc,k", ITER_CASES,
                         ids=[f"{c}-{n}-{b}-{k}" for c, n, b, k in ITER_CASES])
def test_be_pcg_iterates(gpu_lib, coord, n, bc, k):
    """The k-th PCG iterate equals the oracle's (same recurrence, same PC1)."""
    g, ctx = _pair(gpu_lib, coord, _faces(coord, n), bc, 0.7)
    E_n = _smooth_E(g, 5)
    dt = 60.0 * R.gershgorin_dt_euler(g, 0.7)
    ref, res = R.be_pcg(g, E_n, dt, 0.7, rtol=0.0, maxit=k)
    x = _cuda(E_n)
    it, rel, st = ctx.resistivity_be_pcg_solve(_cuda(E_n), x, dt, rtol=0.0, maxit=k,
                                               allow_not_converged=True)
    assert it == k == res.iters
    assert relmax(_host(x), ref) <= 1e-12


def test_be_pcg_guess_and_errors(gpu_lib):
    g, ctx = _pair(gpu_lib, "spherical", shell_faces(6, 7, 9), SHELL_BC, 0.7)
    E_n = _smooth_E(g, 3)
    dt = 30.0 * R.gershgorin_dt_euler(g, 0.7)
    ref, _ = R.be_pcg(g, E_n, dt, 0.7, rtol=1e-12)
    # any initial guess on the interior edges converges to the same solution;
    # the fixed edges take E^n's values
    x = _cuda(np.zeros_like(E_n))
    it, rel, st = ctx.resistivity_be_pcg_solve(_cuda(E_n), x, dt, rtol=1e-12)
    assert st == 0 and relmax(_host(x), ref) <= 1e-10
    x = _cuda(E_n)
    it, rel, st = ctx.resistivity_be_pcg_solve(_cuda(E_n), x, dt, rtol=1e-12, maxit=2,
                                               allow_not_converged=True)
    assert st == 1 and it == 2
    En = _cuda(E_n)
    for kw in (dict(dt=-1.0), dict(dt=dt, rtol=-1.0)):
        with pytest.raises(gpu_lib.StsError):
            ctx.resistivity_be_pcg_solve(En, _cuda(E_n), **kw)
    with pytest.raises(gpu_lib.StsError):
        ctx.resistivity_be_pcg_solve(En, En, dt)
    ctx2 = gpu_lib.Context(gpu_lib.SPHERICAL, *shell_faces(6, 7, 9), SHELL_BC)
    with pytest.raises(gpu_lib.StsError):
        ctx2.apply_F_resistivity(En)  # not set
    with pytest.raises(gpu_lib.StsError):
        ctx2.set_resistivity(0.0)


# ----------------------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def shell128(gpu_lib):
    w = make_workload("shell128")
    return _pair(gpu_lib, "spherical", (w["rf"], w["thf"], w["phf"]), SHELL_BC, 1.0)


def test_shell128_F_and_dt(shell128):
    g, ctx = shell128
    E = _smooth_E(g, 11)
    got = _host(ctx.apply_F_resistivity(_cuda(E)))
    assert relmax(got, R.apply_F(g, E, 1.0)) <= 1e-12
    assert ctx.resistivity_dt_euler() == pytest.approx(R.gershgorin_dt_euler(g, 1.0), rel=1e-12)


def test_shell128_be_pcg(shell128):
    g, ctx = shell128
    E_n = _smooth_E(g, 12)
    dt = 20.0 * R.gershgorin_dt_euler(g, 1.0)
    rtol = 1e-8
    ref, res = R.be_pcg(g, E_n, dt, 1.0, rtol=rtol)
    x = _cuda(E_n)
    it, rel, st = ctx.resistivity_be_pcg_solve(_cuda(E_n), x, dt, rtol=rtol)
    assert st == 0 and abs(it - res.iters) <= 1 and rel <= rtol
    got = _host(x)
    _, b, _, m = R.be_system(g, E_n, dt, 1.0)
    hmin = np.min(R.EdgeGrid.join(g.H)[m])
    assert np.linalg.norm(got[m] - ref[m]) <= 2.0 * rtol * np.linalg.norm(b) / hmin


# ----------------------------------------------------------------------------- 256 x 256 x 512
@pytest.fixture(scope="module")
def shell256_res(gpu_lib):
    """The benchmark's resistivity grid: 256 x 256 x 512 cells, 101.2M edges,
    the fused sweep in the benchmark's launch (tiles, strips and runs)."""
    faces = shell_faces(256, 256, 512)
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, *faces, SHELL_BC)
    ctx.set_resistivity(1.0)
    yield faces, ctx
    ctx.close()


def _split_full(sizes, shapes, v):
    out, o = {}, 0
    for c, n, sh in zip("rtp", sizes, shapes):
        out[c] = v[o:o + n].reshape(sh)
        o += n
    return out


SHAPES256 = [(256, 257, 512), (257, 256, 512), (257, 257, 512)]


def test_shell256_F_windows(shell256_res):
    """F at full size against the oracle on windows of cells, each taken as a
    grid of its own (its interior edges have the whole grid's F): at the inner
    r and theta boundaries, across a run, a tile, a theta tile and strip
    boundary, and at the outer r and theta corner."""
    faces, ctx = shell256_res
    sizes = ctx.resistivity_sizes()
    assert [int(np.prod(s)) for s in SHAPES256] == list(sizes)
    E = np.random.default_rng(21).standard_normal(sum(sizes))
    F = _split_full(sizes, SHAPES256, _host(ctx.apply_F_resistivity(_cuda(E))))
    Es = _split_full(sizes, SHAPES256, E)
    windows = [((0, 0, 0), (6, 7, 9)), ((14, 12, 58), (22, 21, 70)),
               ((127, 30, 250), (133, 36, 262)), ((250, 249, 500), (256, 256, 511))]
    for lo, hi in windows:
        win = resistivity_window(R, "spherical", faces, Es, lo, hi, 1.0)
        scale = max(np.max(np.abs(w[0])) for w in win.values())
        for c, (Fw, m, sl) in win.items():
            assert m.any()
            err = np.max(np.abs(F[c][sl][m] - Fw[m]))
            assert err <= 1e-12 * scale, (lo, hi, c, err / scale)


def test_shell256_F_of_gradient_vanishes(shell256_res):
    """At full size the curl of a discrete gradient is zero on every edge."""
    faces, ctx = shell256_res
    sizes = ctx.resistivity_sizes()
    phi = np.random.default_rng(22).standard_normal((257, 257, 512))
    E = R.EdgeGrid.join({"r": phi[1:] - phi[:-1], "t": phi[:, 1:] - phi[:, :-1],
                         "p": np.roll(phi, -1, axis=2) - phi})
    del phi
    F = _host(ctx.apply_F_resistivity(_cuda(E)))
    scale = float(np.max(np.abs(_host(ctx.apply_F_resistivity(
        _cuda(np.random.default_rng(23).standard_normal(sum(sizes))))))))
    assert np.max(np.abs(F)) <= 1e-12 * scale
