"""The lagged-diffusivity march of the 128 x 128 x 256 shell over 10
successive steps (Sec. 1: kappa frozen at the start of every step; dt fixed
at 200 x the first step's dt_Euler; RKL2 stage count from each step's own
dt_Euler, Eq. rkl2_s; BE by Jacobi-PCG and by block-ILU0(8^3)-PCG to 1e-8,
Sec. 2), each method marching its own state on the GPU, against the
oracle's march of the same protocol stored by
tests/golden/make_shell128_march.py.  After every step: dt_E to 1e-12,
equal stage counts, PCG iteration counts within one, the state at the
stored cells to 1e-12 relative to max |u|, and the sum, 2-norm, min and max
of the whole state to 1e-12 relative."""
import json
import os

import numpy as np
import pytest

from workloads import make_workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "shell128_march.json")


@pytest.fixture(scope="module")
def march(gpu_lib):
    import torch
    with open(GOLDEN) as fh:
        g = json.load(fh)
    w = make_workload(g["workload"], with_velocity=False)
    ctx = gpu_lib.Context(gpu_lib.SPHERICAL, w["rf"], w["thf"], w["phf"], gpu_lib.SHELL_BC)
    ctx.set_dirichlet(0, value=w["T_inner"])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    b = tuple(dev(w[k]) for k in ("br", "bt", "bp"))
    yield g, w, ctx, dev(w["T"]), b
    ctx.close()


def _check_state(u, rec, idx, n, name):
    import torch
    torch.cuda.synchronize()
    vals = u[idx].cpu().numpy()
    scale = rec["max"]
    assert np.max(np.abs(vals - np.array(rec["values"]))) <= 1e-12 * scale, (name, n)
    uf = u.double()
    for key, got in (("sum", float(uf.sum())), ("norm2", float(torch.linalg.vector_norm(uf))),
                     ("min", float(uf.min())), ("max", float(uf.max()))):
        assert abs(got - rec[key]) <= 1e-12 * abs(rec[key]), (name, n, key, got, rec[key])


@pytest.mark.parametrize("name", ["rkl2", "jacobi", "ilu0"])
def test_march_matches_oracle(march, gpu_lib, name):
    import torch
    g, w, ctx, T, b = march
    idx = tuple(torch.tensor(c, device="cuda") for c in zip(*g["cells"]))
    dt = g["dt"]
    u = T.clone()
    x = torch.empty_like(u)
    for n, rec in enumerate(g["methods"][name]):
        ctx.set_spitzer(u, w["kappa0"], *b)
        assert ctx.dt_euler() == pytest.approx(rec["dt_euler"], rel=1e-12), (name, n)
        if name == "rkl2":
            assert ctx.rkl2_step(u, dt) == rec["work"], n
        else:
            x.copy_(u)
            pc = gpu_lib.PC_JACOBI if name == "jacobi" else gpu_lib.PC_BLOCK_ILU0
            it, rel, st = ctx.be_pcg_solve(u, x, dt, pc=pc, block=tuple(g["block"]),
                                           rtol=g["rtol"])
            assert st == 0 and rel <= g["rtol"] and abs(it - rec["work"]) <= 1, (n, it)
            u, x = x, u
        _check_state(u, rec, idx, n, name)
