"""rkl2_step_noalloc: the RKL2 super-step with its stage buffers in the
library's static device scratch (for callers that cannot allocate device
memory), called through the C ABI and checked against rkl2_step on the same
inputs (same kernels: bit for bit) and against the oracle."""
import numpy as np
import pytest

from oracle import operator as O
from oracle import rkl2 as orkl2
from tests.helpers import gpu_spitzer, oracle_spitzer, relmax, small_shell

pytestmark = pytest.mark.gpu

BC = (1, 0, 0, 0, 2, 2)  # Dirichlet r-inner, zero flux r-outer / theta, periodic phi
MAX_CELLS_FP64 = 4_194_304


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _stack(T, ncomp):
    """ncomp components: T and scaled / shifted copies of it."""
    return np.stack([T * (1.0 - 0.05 * m) + 1e4 * m for m in range(ncomp)])


def _run_pair(sts, w, ncomp, ratio, f32=False):
    """(noalloc result, rkl2_step result, s, free-memory drop of the noalloc
    call in bytes) on one fresh context."""
    import torch
    ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], BC, u_lo=w["T_inner"])
    if f32:
        f = lambda a: _dev(a).float()  # noqa: E731
        ctx.set_spitzer_f32(f(w["T"]), w["kappa0"], f(w["br"]), f(w["bt"]), f(w["bp"]))
    dt = ratio * ctx.dt_euler()
    u0 = _dev(_stack(w["T"], ncomp)) if ncomp > 1 else _dev(w["T"])
    ua = u0.clone()
    s_warm = ctx.rkl2_step_noalloc(ua, dt)  # warm-up: first launches of the stage kernels
    ua.copy_(u0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    s_a = ctx.rkl2_step_noalloc(ua, dt)
    torch.cuda.synchronize()
    drop = free0 - torch.cuda.mem_get_info()[0]
    ub = u0.clone()
    s_b = ctx.rkl2_step(ub, dt)
    torch.cuda.synchronize()
    ctx.close()
    assert s_a == s_b == s_warm
    return ua.cpu().numpy(), ub.cpu().numpy(), s_a, dt, drop


def test_noalloc_matches_rkl2_step_two_calls_second_smaller(gpu_lib):
    """Call 1: 40x48x72 with two components; call 2: a smaller 12x16x24 grid,
    one component, on another context of the same GPU (the scratch keeps call
    1's contents).  Both equal rkl2_step bit for bit, neither allocates, and
    call 2 matches the oracle's super-step to 1e-12."""
    sts = gpu_lib
    w1 = small_shell((40, 48, 72), seed=3)
    a1, b1, s1, _, drop1 = _run_pair(sts, w1, 2, 50.0)
    assert np.array_equal(a1, b1), relmax(a1, b1)
    # workspace of rkl2_step for this call: 3 x 276480 x 8 B = 6.6 MB
    assert drop1 < 1 << 20, drop1
    w2 = small_shell((12, 16, 24), seed=4)
    a2, b2, s2, dt2, drop2 = _run_pair(sts, w2, 1, 50.0)
    assert np.array_equal(a2, b2), relmax(a2, b2)
    assert drop2 < 1 << 20, drop2
    op = oracle_spitzer(w2["rf"], w2["thf"], w2["phf"], w2["T"], w2["br"], w2["bt"], w2["bp"],
                        w2["kappa0"], BC, u_lo=w2["T_inner"])
    ref = orkl2.rkl2_step(lambda v: O.apply_F(op, v), w2["T"], dt2, s2)
    assert relmax(a2, ref) <= 1e-12


def test_noalloc_fp32_form_matches_rkl2_step(gpu_lib):
    w = small_shell((24, 20, 40), seed=5)
    a, b, s, _, drop = _run_pair(gpu_lib, w, 1, 50.0, f32=True)
    assert np.array_equal(a, b) and drop < 1 << 20


def test_noalloc_limits(gpu_lib):
    """The largest accepted size runs and equals rkl2_step; one more component
    is rejected before anything is enqueued; s <= 0 needs a computed dt_E."""
    import torch
    sts = gpu_lib
    from workloads import shell_faces
    rf, thf, phf = shell_faces(128, 128, 256)  # 4,194,304 cells: the FP64 maximum
    ctx = sts.Context(sts.SPHERICAL, rf, thf, phf, sts.SHELL_BC)
    ctx.set_isotropic(1.0)
    n = 128 * 128 * 256
    assert n == MAX_CELLS_FP64
    g = torch.Generator(device="cpu").manual_seed(7)
    u0 = torch.rand(n, generator=g, dtype=torch.float64).reshape(128, 128, 256).cuda()
    with pytest.raises(sts.StsError) as e:
        ctx.rkl2_step_noalloc(u0.clone(), 1e-3)  # s = 0: dt_E not yet computed
    assert e.value.code == sts.STS_EINVAL and "sts_dt_euler" in str(e.value)
    dt = 30.0 * ctx.dt_euler()
    ua, ub = u0.clone(), u0.clone()
    s = ctx.rkl2_step_noalloc(ua, dt)
    assert ctx.rkl2_step(ub, dt) == s
    assert torch.equal(ua, ub)
    two = torch.stack([u0, u0])
    before = two.clone()
    with pytest.raises(sts.StsError) as e:
        ctx.rkl2_step_noalloc(two, dt)  # 2 x 4,194,304: above the scratch
    assert e.value.code == sts.STS_EINVAL and "scratch" in str(e.value)
    assert torch.equal(two, before)
    ctx.close()
