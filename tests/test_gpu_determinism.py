"""Run-to-run reproducibility at the benchmark's size (128 x 128 x 256): the
reductions (Gershgorin maximum, PCG dot products and norms) sum per-workgroup
partials in a fixed order, so repeating a call, on the same or on a fresh
context, gives bitwise-identical results and equal iteration counts."""
import numpy as np
import pytest

from workloads import edge_potential, make_workload

pytestmark = pytest.mark.gpu
SHELL_BC = (1, 0, 0, 0, 2, 2)


def _cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dtype) if dtype is not None else t


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def w():
    return make_workload("shell128")


def _ctx(sts, w):
    c = sts.Context(sts.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    c.set_dirichlet(0, value=w["T_inner"])
    c.set_spitzer(_cuda(w["T"]), w["kappa0"], _cuda(w["br"]), _cuda(w["bt"]), _cuda(w["bp"]))
    return c


def _run(sts, ctx, w):
    T = _cuda(w["T"])
    out = {"dt": ctx.dt_euler()}
    dt = 200.0 * out["dt"]
    out["F"] = _host(ctx.apply_F(T))
    u = T.clone()
    out["s"] = ctx.rkl2_step(u, dt)
    out["rkl2"] = _host(u)
    for pc in (sts.PC_JACOBI, sts.PC_BLOCK_ILU0):
        x = T.clone()
        it, rel, st = ctx.be_pcg_solve(T, x, dt, pc=pc, rtol=1e-8)
        assert st == 0
        out[f"pcg{pc}"] = (it, rel, _host(x))
    return out


def test_solver_path_is_bitwise_reproducible(gpu_lib, w):
    a = _ctx(gpu_lib, w)
    r1, r2 = _run(gpu_lib, a, w), _run(gpu_lib, a, w)
    b = _ctx(gpu_lib, w)
    r3 = _run(gpu_lib, b, w)
    for r in (r2, r3):
        assert r["dt"] == r1["dt"] and r["s"] == r1["s"]
        assert np.array_equal(r["F"], r1["F"]) and np.array_equal(r["rkl2"], r1["rkl2"])
        for pc in (0, 1):
            it, rel, x = r[f"pcg{pc}"]
            assert it == r1[f"pcg{pc}"][0] and rel == r1[f"pcg{pc}"][1]
            assert np.array_equal(x, r1[f"pcg{pc}"][2])
    a.close()
    b.close()


def test_fp32_form_and_unlagged_step_are_reproducible(gpu_lib, w):
    import torch
    f = torch.float32
    c = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    c.set_dirichlet(0, value=w["T_inner"])
    c.set_spitzer_f32(_cuda(w["T"], f), w["kappa0"], _cuda(w["br"], f), _cuda(w["bt"], f),
                      _cuda(w["bp"], f))
    T = _cuda(w["T"])
    dt = 200.0 * c.dt_euler()
    res = []
    for _ in range(2):
        x = T.clone()
        it, rel, st = c.be_pcg_solve(T, x, dt, pc=gpu_lib.PC_JACOBI, rtol=1e-8)
        u = T.clone()
        c.rkl2_step(u, dt)
        res.append((it, rel, _host(x), _host(u)))
    assert res[0][:2] == res[1][:2]
    assert np.array_equal(res[0][2], res[1][2]) and np.array_equal(res[0][3], res[1][3])
    c.close()
    c = _ctx(gpu_lib, w)
    b = [_cuda(w[k]) for k in ("br", "bt", "bp")]
    outs = []
    for _ in range(2):
        u = T.clone()
        c.rkl2_step_nonlinear(u, dt, w["kappa0"], *b)
        outs.append(_host(u))
    assert np.array_equal(outs[0], outs[1])
    c.close()


def test_resistivity_solve_is_reproducible(gpu_lib, w):
    c = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], SHELL_BC)
    c.set_resistivity(1.0)
    E0 = _cuda(edge_potential(128, 128, 256))
    dt = 200.0 * c.resistivity_dt_euler()
    res = []
    for _ in range(2):
        x = E0.clone()
        it, rel, st = c.resistivity_be_pcg_solve(E0, x, dt, rtol=1e-8)
        assert st == 0
        res.append((it, rel, _host(x)))
    assert res[0][:2] == res[1][:2] and np.array_equal(res[0][2], res[1][2])
    c.close()
