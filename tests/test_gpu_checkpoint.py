"""Checkpoint and resume on the GPU: a guess network and a factor network are
trained a few steps, saved with the fields of the run, trained further; the
same further training after restoring the checkpoint into fresh networks
gives bit for bit the same weights and losses (master parameters, Adam
moments, step count and scalings all restored).  cnn_set_state refuses
states it cannot hold."""
import numpy as np
import pytest

from helpers import gpu_spitzer, small_shell
from paper_1610_01265_amd import checkpoint
from workloads import flatten, he_normal

pytestmark = pytest.mark.gpu
BC = (1, 0, 0, 0, 2, 2)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_resume_is_exact(gpu_lib, tmp_path):
    import torch
    sts = gpu_lib
    shape = (12, 16, 66)
    w = small_shell(shape, seed=4)
    ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], BC, u_lo=w["T_inner"])
    T = _cuda(w["T"])
    dt = 40.0 * ctx.dt_euler()
    F0 = ctx.apply_F(T)
    xs = T.clone()
    ctx.be_pcg_solve(T, xs, dt, rtol=1e-10)
    z = _cuda(np.random.default_rng(2).choice([-1.0, 1.0], size=shape))

    def new_nets():
        g = sts.Cnn(ctx)
        g.set_weights(flatten(he_normal(4, 16, 0)))
        g.set_norm(1.0 / float(torch.max(torch.abs(F0))), float(T.mean()), 1e-6, 1e-3)
        g.set_adam(0.8, 0.95, 1e-7)
        p = sts.CnnPC(ctx)
        params = he_normal(4, 16, 1, out_ch=4)
        params[3][0] = params[3][0] * 0.1
        p.set_weights(flatten(params))
        p.set_norm(float(T.mean()), 1e-6)
        return g, p

    def train(g, p, steps):
        out = []
        for _ in range(steps):
            out.append(g.train_step(F0, dt, T, xs, 1e-3))
            out.append(p.train_step(T, dt, z, 2e-3))
        return out

    g, p = new_nets()
    train(g, p, 3)
    path = str(tmp_path / "ckpt.pt")
    checkpoint.save(path, fields={"T": T, "x": xs}, nets={"guess": g, "factor": p},
                    extra={"steps": 3})
    la = train(g, p, 2)
    wa = (g.get_weights(), p.get_weights())
    g.close()
    p.close()

    g2, p2 = new_nets()  # fresh networks, then the checkpoint
    fields, extra = checkpoint.load(path, nets={"guess": g2, "factor": p2})
    assert extra == {"steps": 3}
    assert torch.equal(fields["T"], T) and torch.equal(fields["x"], xs)
    lb = train(g2, p2, 2)
    assert la == lb
    assert np.array_equal(wa[0], g2.get_weights()) and np.array_equal(wa[1], p2.get_weights())

    # refusals: size, non-finite, negative second moment, a padding entry
    st = g2.get_state()
    n = st["buf"].size // 3
    for mutate in (lambda b, m: (b[:-1], m),
                   lambda b, m: (np.where(np.arange(b.size) == 5, np.nan, b), m),
                   lambda b, m: (np.where(np.arange(b.size) == 2 * n + 5, -1.0, b), m),
                   lambda b, m: (b, np.where(np.arange(8) == 0, -1.0, m))):
        b, m = mutate(st["buf"].copy(), st["meta"].copy())
        with pytest.raises(sts.StsError):
            g2.set_state({"buf": b.astype(np.float32), "meta": m})
    pad = st["buf"].copy()
    pad[16 * 16 * 27 - 1] = 1.0  # layer 0 has 2 input channels: (co 15, ci 15) is padding
    with pytest.raises(sts.StsError):
        g2.set_state({"buf": pad, "meta": st["meta"]})
    g2.close()
    p2.close()
    ctx.close()
