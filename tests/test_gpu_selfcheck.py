"""Diagnostics of the library on the GPU:

  * workgroup-order self-check: with STS_DEBUG_WG_REVERSE the stencil march,
    the PCG sweeps and the factor kernels take their work in reversed
    workgroup order (each workgroup still computes the same tiles and partial
    sums), so any dependence of a result on the order in which workgroups
    run -- a race through memory or a missing wait -- shows as a difference.
    F, an RKL2 step, Jacobi-, block-ILU0- and factor-PCG solves and the
    un-lagged RKL2 step must be bit for bit those of the normal order;
  * per-kernel timing (sts_set_profile / STS_PROFILE): every launch is
    bracketed by an event pair; the table counts the launches of a solve."""
import numpy as np
import pytest

from helpers import gpu_spitzer, small_shell

pytestmark = pytest.mark.gpu

BC = (1, 0, 0, 0, 2, 2)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _run_all(sts, w, ctx):
    """F, RKL2, three PCG solves and the un-lagged step on one context."""
    T = _cuda(w["T"])
    out = {"F": _host(ctx.apply_F(T))}
    dt = 120.0 * ctx.dt_euler()
    u = T.clone()
    out["s"] = ctx.rkl2_step(u, dt)
    out["rkl2"] = _host(u)
    for name, pc, blk in (("jacobi", sts.PC_JACOBI, (8, 8, 8)),
                          ("ilu0", sts.PC_BLOCK_ILU0, (8, 8, 8)),
                          ("ilu0_ragged", sts.PC_BLOCK_ILU0, (4, 5, 6)),
                          ("factor", sts.PC_FACTOR, (8, 8, 8))):
        x = T.clone()
        it, rel, st = ctx.be_pcg_solve(T, x, dt, pc=pc, block=blk, rtol=1e-10)
        out[name] = (it, rel, _host(x))
    b = [_cuda(w[k]) for k in ("br", "bt", "bp")]
    u = T.clone()
    out["s_nl"] = ctx.rkl2_step_nonlinear(u, dt, w["kappa0"], *b)
    out["nl"] = _host(u)
    return out


@pytest.mark.parametrize("shape", [(40, 36, 130), (64, 64, 128)])
def test_reversed_workgroup_order_is_bitwise_identical(gpu_lib, shape):
    sts = gpu_lib
    w = small_shell(shape, seed=2)
    res = []
    for flags in (0, sts.DEBUG_WG_REVERSE):
        ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                          w["kappa0"], BC, u_lo=w["T_inner"])
        ctx.set_debug(flags)
        # a seeded factor with off-diagonal entries (both runs use the same one)
        rng = np.random.default_rng(3)
        g = np.zeros((4,) + shape, np.float32)
        g[0] = 1e-3 * (1.0 + 0.1 * rng.random(shape))
        g[1:] = 1e-4 * rng.standard_normal((3,) + shape)
        ctx.set_pc_factor(_cuda(g))
        res.append(_run_all(sts, w, ctx))
        ctx.close()
    a, b = res
    for key in ("F", "rkl2", "nl"):
        assert np.array_equal(a[key], b[key]), key
    assert a["s"] == b["s"] and a["s_nl"] == b["s_nl"]
    for key in ("jacobi", "ilu0", "ilu0_ragged", "factor"):
        assert a[key][0] == b[key][0] and a[key][1] == b[key][1], key
        assert np.array_equal(a[key][2], b[key][2]), key


def test_reversed_order_cnn_and_resistivity(gpu_lib):
    """The same self-check for the CNN kernels (convolution, input and weight
    gradients, a training step) and the resistivity operator and its solve."""
    import torch
    sts = gpu_lib
    shape = (20, 12, 130)
    w = small_shell(shape, seed=6)
    rng = np.random.default_rng(7)
    n = int(np.prod(shape))
    x16 = torch.from_numpy(rng.standard_normal((n, 16)).astype(np.float32)).cuda().to(torch.bfloat16)
    d16 = torch.from_numpy(rng.standard_normal((n, 16)).astype(np.float32)).cuda().to(torch.bfloat16)
    wts = (0.05 * rng.standard_normal(15169)).astype(np.float32)
    res = []
    for flags in (0, sts.DEBUG_WG_REVERSE):
        ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                          w["kappa0"], BC, u_lo=w["T_inner"])
        ctx.set_debug(flags)
        net = sts.Cnn(ctx)
        net.set_weights(wts)
        out = {"conv": _host(net.conv(1, sts.CNN_RELU, x16).float()),
               "igrad": _host(net.conv(2, sts.CNN_INPUT_GRAD, d16, mask=x16).float()),
               "wgrad": _host(net.weight_grad(1, x16, d16))}
        T = _cuda(w["T"])
        dt = 30.0 * ctx.dt_euler()
        F0 = ctx.apply_F(T)
        net.set_norm(1.0 / float(torch.max(torch.abs(F0))), float(T.mean()), 1e-6, 1e-3)
        out["loss"] = net.train_step(F0, dt, T, T + 1.0, 1e-3)
        out["weights"] = net.get_weights()
        net.close()
        ctx.set_resistivity(0.3)
        ne = sum(ctx.resistivity_sizes())
        E = torch.from_numpy(rng.standard_normal(ne)).cuda() if flags == 0 else E0
        E0 = E
        out["rF"] = _host(ctx.apply_F_resistivity(E))
        xE = E.clone()
        it, rel, _ = ctx.resistivity_be_pcg_solve(E, xE, 50.0 * ctx.resistivity_dt_euler(),
                                                  rtol=1e-10)
        out["rsolve"] = (it, rel, _host(xE))
        res.append(out)
        ctx.close()
    a, b = res
    for key in ("conv", "igrad", "wgrad", "weights", "rF"):
        assert np.array_equal(a[key], b[key]), key
    assert a["loss"] == b["loss"]
    assert a["rsolve"][:2] == b["rsolve"][:2]
    assert np.array_equal(a["rsolve"][2], b["rsolve"][2])


def test_profile_counts_launches(gpu_lib):
    sts = gpu_lib
    w = small_shell((16, 20, 40), seed=3)
    ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], BC, u_lo=w["T_inner"])
    T = _cuda(w["T"])
    dt = 50.0 * ctx.dt_euler()
    ctx.set_profile(True)
    u = T.clone()
    s = ctx.rkl2_step(u, dt)
    x = T.clone()
    it, _, _ = ctx.be_pcg_solve(T, x, dt, pc=sts.PC_JACOBI, rtol=1e-9)
    tab = ctx.profile_summary()
    assert tab["stage_rk_first"][0] == 1 and tab["stage_rk"][0] == s - 1
    # iterations are enqueued in batches; kernels after convergence return at once
    assert tab["launch_pass_a"][0] >= it and tab["launch_pass_b_jacobi_fused"][0] >= it
    assert all(v[1] >= 0.0 for v in tab.values())
    assert tab["stage_rk"][2] > 0.0
    # reset: an empty table; profiling off: no records
    assert ctx.profile_summary() == {}
    ctx.set_profile(False)
    ctx.apply_F(T)
    assert ctx.profile_summary() == {}
    ctx.close()


@pytest.mark.parametrize("shape", [(40, 36, 130), (64, 64, 128)])
def test_separate_finalizers_match_fused(gpu_lib, shape):
    """The Jacobi and factor PCG with alpha, beta and the stopping test in
    kernels of their own sum the same partials in the same order as the
    in-sweep form: the same iterations, residual and solution bit for bit,
    converged or stopped at maxit (FP64 and the FP32 form)."""
    import torch
    sts = gpu_lib
    w = small_shell(shape, seed=5)
    res = []
    for flags in (0, sts.DEBUG_SEPARATE_FINALIZE):
        ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                          w["kappa0"], BC, u_lo=w["T_inner"])
        ctx.set_debug(flags)
        T = _cuda(w["T"])
        dt = 120.0 * ctx.dt_euler()
        out = []
        for maxit in (10000, 7):
            x = T.clone()
            it, rel, st = ctx.be_pcg_solve(T, x, dt, rtol=1e-10, maxit=maxit,
                                           allow_not_converged=True)
            out.append((it, rel, st, _host(x)))
        # the factored preconditioner's solve (a seeded factor)
        rng = np.random.default_rng(4)
        g = np.zeros((4,) + shape, np.float32)
        g[0] = 1e-3 * (1.0 + 0.1 * rng.random(shape))
        g[1:] = 1e-4 * rng.standard_normal((3,) + shape)
        ctx.set_pc_factor(_cuda(g))
        for maxit in (10000, 5):
            x = T.clone()
            it, rel, st = ctx.be_pcg_solve(T, x, dt, pc=sts.PC_FACTOR, rtol=1e-10, maxit=maxit,
                                           allow_not_converged=True)
            out.append((it, rel, st, _host(x)))
        # the FP32 form's inner Jacobi solve
        f = torch.float32
        ctx.set_spitzer_f32(T.to(f), w["kappa0"], *[_cuda(w[k]).to(f) for k in ("br", "bt", "bp")])
        x = T.clone()
        it, rel, st = ctx.be_pcg_solve(T, x, dt, rtol=1e-8)
        out.append((it, rel, st, _host(x)))
        res.append(out)
        ctx.close()
    for a, b in zip(*res):
        assert a[:3] == b[:3]
        assert np.array_equal(a[3], b[3])
    assert res[0][1][0] == 7 and res[0][1][2] != 0
    assert res[0][3][0] == 5 and res[0][3][2] != 0
