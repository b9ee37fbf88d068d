"""GPU parity of the learned-guess CNN kernels against the FP64 oracle
(oracle/cnn.py), through the C ABI.

Inputs and weights are bfloat16-representable, so both sides multiply the
same numbers; the kernels accumulate in FP32 (MFMA).  Tolerances:
  * FP32 outputs: |gpu - oracle| <= 1e-5 * sum |w||x| (the scale of FP32
    accumulation error over K <= 432 products);
  * bf16 outputs: additionally one bf16 rounding, 2^-8 |oracle|;
  * weight gradients: 1e-5 * sum |dout||act| per entry;
  * orchestration (cnn_forward, cnn_train_step) is compared bit for bit
    against the same kernels called one by one, and against the oracle's
    whole-network values within the effect of bf16 activation rounding.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn
from workloads import flatten, he_normal, shell_faces

pytestmark = pytest.mark.gpu

SHAPES = [(4, 8, 64), (5, 7, 70), (3, 5, 20), (2, 3, 3), (9, 12, 130)]
RB = ocnn.round_bf16


def _torch():
    import torch
    return torch


def _ctx(sts, shape):
    rf, thf, phf = shell_faces(*shape)
    return sts.Context(sts.SPHERICAL, rf, thf, phf)


def _params(seed, layers=4, bias_scale=0.05):
    rng = np.random.default_rng(1000 + seed)
    p = he_normal(layers, 16, seed)
    return [[RB(W), RB(bias_scale * rng.standard_normal(b.shape))] for W, b in p]


def _net(sts, shape, seed=0, layers=4):
    ctx = _ctx(sts, shape)
    net = sts.Cnn(ctx, layers)
    params = _params(seed, layers)
    net.set_weights(flatten(params))
    return ctx, net, params


def _dev16(x):
    """[C, n0, n1, n2] (bf16-representable) -> bf16 tensor [cells][16]."""
    torch = _torch()
    C = x.shape[0]
    a = np.zeros((x[0].size, 16), np.float32)
    a[:, :C] = x.reshape(C, -1).T
    return torch.from_numpy(a).to(torch.bfloat16).cuda()


def _host16(t, C, shape):
    torch = _torch()
    torch.cuda.synchronize()
    a = t.float().cpu().numpy().astype(np.float64)
    return a[:, :C].T.reshape((C,) + tuple(shape))


def _cuda(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch = _torch()
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _rand_act(rng, C, shape, relu=False):
    x = rng.standard_normal((C,) + tuple(shape))
    if relu:
        x = np.maximum(x, 0.0)
    return RB(x)


def _dims(l, layers=4):
    return (2 if l == 0 else 16), (1 if l == layers - 1 else 16)


# --------------------------------------------------------------------------- input packing
@pytest.mark.parametrize("shape", SHAPES[:3])
def test_pack_input_bit_exact(gpu_lib, shape):
    ctx, net, _ = _net(gpu_lib, shape)
    rng = np.random.default_rng(5)
    F = rng.standard_normal(shape) * 3e3
    T = 1e6 * (1 + 0.3 * rng.random(shape))
    dt, rs, tsh, tsc = 0.37, 2.5e-4, 1.1e6, 4e-6
    net.set_norm(rs, tsh, tsc, 1.0)
    x = net.pack_input(_cuda(F), dt, _cuda(T))
    got = x.float().cpu().numpy().astype(np.float64)
    ref = np.zeros_like(got)
    ref[:, 0] = RB((F * (dt * rs)).ravel())
    ref[:, 1] = RB(((T - tsh) * tsc).ravel())
    assert np.array_equal(got, ref)


# --------------------------------------------------------------------------- forward
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [0, 1, 3])
def test_conv_forward_f32(gpu_lib, shape, layer):
    ctx, net, params = _net(gpu_lib, shape, seed=layer)
    cin, cout = _dims(layer)
    rng = np.random.default_rng(10 + layer)
    x = _rand_act(rng, cin, shape, relu=layer > 0)
    W, b = params[layer]
    got = _host(net.conv(layer, gpu_lib.CNN_F32, _dev16(x)))
    ref = ocnn.conv3d(x, W, b)
    scale = ocnn.conv3d(np.abs(x), np.abs(W))
    g = got[:, :cout].T.reshape(ref.shape)
    assert np.all(np.abs(g - ref) <= 1e-5 * scale + 1e-30)
    assert np.all(got[:, cout:] == 0.0)


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_relu_bf16(gpu_lib, shape):
    ctx, net, params = _net(gpu_lib, shape, seed=1)
    rng = np.random.default_rng(21)
    x = _rand_act(rng, 16, shape, relu=True)
    W, b = params[1]
    got = _host16(net.conv(1, gpu_lib.CNN_RELU, _dev16(x)), 16, shape)
    z = ocnn.conv3d(x, W, b)
    ref = np.maximum(z, 0.0)
    scale = ocnn.conv3d(np.abs(x), np.abs(W))
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * scale + 1e-30)


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_output_layer(gpu_lib, shape):
    ctx, net, params = _net(gpu_lib, shape, seed=3)
    rng = np.random.default_rng(31)
    x = _rand_act(rng, 16, shape, relu=True)
    W, b = params[3]
    got = _host(net.conv(3, gpu_lib.CNN_LINEAR, _dev16(x))).reshape(shape)
    ref = ocnn.conv3d(x, W, b)[0]
    scale = ocnn.conv3d(np.abs(x), np.abs(W))[0]
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-30)


# --------------------------------------------------------------------------- gradients
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [1, 3])
def test_input_grad(gpu_lib, shape, layer):
    ctx, net, params = _net(gpu_lib, shape, seed=layer)
    cin, cout = _dims(layer)
    rng = np.random.default_rng(40 + layer)
    dy = _rand_act(rng, cout, shape)
    W, _ = params[layer]
    got = _host(net.conv(layer, gpu_lib.CNN_INPUT_GRAD_F32, _dev16(dy)))
    ref = ocnn.conv3d_input_grad(dy, W, cin)
    scale = ocnn.conv3d_input_grad(np.abs(dy), np.abs(W), cin)
    g = got[:, :cin].T.reshape(ref.shape)
    assert np.all(np.abs(g - ref) <= 1e-5 * scale + 1e-30)
    # masked bf16 form (the back-propagation step through a ReLU)
    mask = _rand_act(rng, cin, shape, relu=True)
    gm = _host16(net.conv(layer, gpu_lib.CNN_INPUT_GRAD, _dev16(dy), mask=_dev16(mask)), cin,
                 shape)
    refm = ref * (mask > 0)
    assert np.all(np.abs(gm - refm) <= 2.0 ** -8 * np.abs(refm) + 1e-5 * scale + 1e-30)
    assert np.all(gm[mask <= 0] == 0.0)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [0, 2, 3])
def test_weight_grad(gpu_lib, shape, layer):
    ctx, net, _ = _net(gpu_lib, shape)
    cin, cout = _dims(layer)
    rng = np.random.default_rng(50 + layer)
    act = _rand_act(rng, cin, shape, relu=layer > 0)
    dy = _rand_act(rng, cout, shape)
    got = _host(net.weight_grad(layer, _dev16(act), _dev16(dy)))
    gW = got[:16 * 16 * 27].reshape(16, 16, 3, 3, 3)
    gb = got[16 * 16 * 27:]
    refW = ocnn.conv3d_weight_grad(act, dy)
    scaleW = ocnn.conv3d_weight_grad(np.abs(act), np.abs(dy))
    assert np.all(np.abs(gW[:cout, :cin] - refW) <= 1e-5 * scaleW + 1e-30)
    assert np.all(gW[cout:] == 0.0) and np.all(gW[:, cin:] == 0.0)
    refb = dy.sum(axis=(1, 2, 3))
    scaleb = np.abs(dy).sum(axis=(1, 2, 3))
    assert np.all(np.abs(gb[:cout] - refb) <= 1e-5 * scaleb + 1e-30)
    assert np.all(gb[cout:] == 0.0)


# --------------------------------------------------------------------------- whole network
def _inputs(shape, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal(shape) * 2e4
    T = 1e6 * (1.2 + 0.2 * rng.standard_normal(shape))
    xs = T + 3e3 * rng.standard_normal(shape)
    return F, T, xs


def _chain_forward(sts, net, F, dt, T, layers=4):
    """The network evaluated kernel by kernel through the ABI."""
    acts = [net.pack_input(_cuda(F), dt, _cuda(T))]
    for l in range(layers - 1):
        acts.append(net.conv(l, sts.CNN_RELU, acts[-1]))
    pred = net.conv(layers - 1, sts.CNN_LINEAR, acts[-1])
    return acts, pred


@pytest.mark.parametrize("shape", [(6, 10, 72), (3, 5, 20)])
def test_forward_matches_chain_and_oracle(gpu_lib, shape):
    torch = _torch()
    ctx, net, params = _net(gpu_lib, shape, seed=7)
    F, T, _ = _inputs(shape, 7)
    dt, norm = 0.5, (1e-4, 1.2e6, 5e-6, 2e3)
    net.set_norm(*norm)
    x0 = _host(net.forward(_cuda(F), dt, _cuda(T)))
    acts, pred = _chain_forward(gpu_lib, net, F, dt, T)
    chain = _host(_cuda(T)) + norm[3] * _host(pred).reshape(shape)
    # same kernels in the same order; x0 = T + s * pred may be one fused multiply-add
    assert np.max(np.abs(x0 - chain) / np.abs(chain)) <= 4e-16
    # each layer against the oracle on the GPU's own input activation
    for l in range(3):
        a = _host16(acts[l], 16, shape)
        nxt = _host16(acts[l + 1], 16, shape)
        W, b = params[l]
        z = ocnn.conv3d(a[:_dims(l)[0]], W, b)
        scale = ocnn.conv3d(np.abs(a[:_dims(l)[0]]), np.abs(W))
        assert np.all(np.abs(nxt - np.maximum(z, 0)) <= 2.0 ** -8 * np.abs(z) + 1e-5 * scale + 1e-30)
    # whole network against the oracle (bf16-rounded activations on both sides;
    # rare ties decided differently by FP32 accumulation order move a value by
    # one bf16 step)
    xin = np.stack([RB((F * (dt * norm[0]))), RB((T - norm[1]) * norm[2])])
    y, _ = ocnn.forward(params, xin, act_round=RB)
    ref = T + norm[3] * y[0]
    d = np.abs(x0 - ref) / (norm[3] * np.max(np.abs(y)))
    assert np.max(d) < 2e-2 and np.median(d) < 1e-4
    torch.cuda.synchronize()


def _chain_grads(sts, net, F, dt, T, xs, norm):
    """Loss gradient of the network, kernel by kernel through the ABI:
    (padded gradient per layer as device tensors, activations, loss)."""
    torch = _torch()
    acts, pred = _chain_forward(sts, net, F, dt, T)
    n = T.size
    p = _host(pred)
    tgt = ((xs - T) * (1.0 / norm[3])).ravel()
    d = p - tgt
    g = np.zeros((n, 16), np.float32)
    g[:, 0] = (np.float32(2.0 / n) * d.astype(np.float32))
    gcur = torch.from_numpy(g).to(torch.bfloat16).cuda()
    grads = [None] * 4
    for l in range(3, -1, -1):
        grads[l] = net.weight_grad(l, acts[l], gcur)
        if l > 0:
            gcur = net.conv(l, sts.CNN_INPUT_GRAD, gcur, mask=acts[l])
    return grads, acts, float(np.mean(d * d))


def test_adam_step_matches_oracle(gpu_lib):
    """cnn_adam_step against the oracle's Adam (FP64) over four steps with
    varying gradients, beta1 = 0.5 != beta2 = 0.75 (a swap, a missing or
    mis-timed bias correction moves the weights by O(lr)).  Gradients are
    seeded FP32 values in the padded layout; padding entries are ignored."""
    sts = gpu_lib
    torch = _torch()
    ctx, net, params = _net(sts, (2, 3, 4), seed=5)
    b1, b2, eps, lr = 0.5, 0.75, 1e-8, 1e-3
    net.set_adam(b1, b2, eps)
    oparams = [[W.astype(np.float64).copy(), b.astype(np.float64).copy()] for W, b in params]
    st = ocnn.adam_init(oparams)
    rng = np.random.default_rng(42)
    P = sts.CNN_PADDED_PARAMS
    for t in range(4):
        gpad = rng.standard_normal((4, P)).astype(np.float32)
        grads = []
        for l in range(4):
            cin, cout = _dims(l)
            gW = gpad[l, :16 * 16 * 27].reshape(16, 16, 3, 3, 3)[:cout, :cin]
            grads.append([gW.astype(np.float64), gpad[l, 16 * 16 * 27:][:cout].astype(np.float64)])
        net.adam_step(torch.from_numpy(gpad.ravel()).cuda(), lr)
        st = ocnn.adam_step(oparams, grads, st, lr, beta1=b1, beta2=b2, eps=eps)
        w = net.get_weights().astype(np.float64)
        ref = flatten(oparams).astype(np.float64)
        # FP32 master weights and FP32 arithmetic: an ulp of the weight per step
        assert np.all(np.abs(w - ref) <= 2 * (t + 1) * np.spacing(np.abs(ref).astype(np.float32))
                      + 1e-4 * lr), t
    with pytest.raises(sts.StsError):
        net.set_adam(1.0, 0.5)


def test_train_steps_match_chain_and_adam_step(gpu_lib):
    """Three cnn_train_step calls (forward, loss, back-propagation, Adam with
    beta1 = 0.5, beta2 = 0.75) on different samples, against a second network
    driven by the kernels one by one and cnn_adam_step; the first step's
    gradients also against the oracle's back-propagation."""
    sts = gpu_lib
    shape = (5, 8, 66)
    ctx, net, params = _net(sts, shape, seed=11)
    ctx2 = _ctx(sts, shape)
    net2 = sts.Cnn(ctx2, 4)
    net2.set_weights(flatten(params))
    dt, norm = 0.5, (1e-4, 1.2e6, 5e-6, 2e3)
    lr = 1e-3
    for nn in (net, net2):
        nn.set_norm(*norm)
        nn.set_adam(0.5, 0.75)
    for t in range(3):
        F, T, xs = _inputs(shape, 11 + t)
        grads, acts, loss_ref = _chain_grads(sts, net2, F, dt, T, xs, norm)
        loss = net.train_step(_cuda(F), dt, _cuda(T), _cuda(xs), lr)
        assert loss == pytest.approx(loss_ref, rel=1e-6)
        _torch().cuda.synchronize()
        net2.adam_step(_torch().cat(grads), lr)
        w1, w2 = net.get_weights(), net2.get_weights()
        # FP32 on both sides; the loss gradient is formed on the host on one
        # side: a few ulps per step
        assert np.all(np.abs(w1 - w2) <= 4 * (t + 1) * np.spacing(np.abs(w2)) + 1e-4 * lr), t
        if t == 0:
            # the gradients against the oracle's back-propagation through the
            # same network (bf16 activation rounding on both sides)
            xin = np.stack([RB(F * (dt * norm[0])), RB((T - norm[1]) * norm[2])])
            y, cache = ocnn.forward(params, xin, act_round=RB)
            _, dy = ocnn.mse_loss(y, ((xs - T) / norm[3])[None])
            og = ocnn.backward(params, cache, dy)
            for l in range(4):
                cin, cout = _dims(l)
                gh = _host(grads[l])
                gW = gh[:16 * 16 * 27].reshape(16, 16, 3, 3, 3)[:cout, :cin]
                err = np.linalg.norm(gW - og[l][0]) / np.linalg.norm(og[l][0])
                assert err < 2e-2, (l, err)
    net2.close()
    ctx2.close()


def test_training_reduces_loss(gpu_lib):
    shape = (6, 12, 64)
    ctx, net, _ = _net(gpu_lib, shape, seed=2)
    F, T, xs = _inputs(shape, 3)
    # a learnable target: the increment is a fixed multiple of the rhs channel
    xs = T + 0.8 * 0.5 * F
    net.set_norm(1.0 / (0.5 * 2e4), 1.2e6, 5e-6, 0.8 * 0.5 * 2e4)
    Fd, Td, xsd = _cuda(F), _cuda(T), _cuda(xs)
    losses = [net.train_step(Fd, 0.5, Td, xsd, 3e-3) for _ in range(60)]
    assert losses[-1] < 0.2 * losses[0]
    assert np.all(np.isfinite(losses))


def test_deterministic(gpu_lib):
    shape = (5, 7, 70)
    out = []
    for _ in range(2):
        ctx, net, _ = _net(gpu_lib, shape, seed=4)
        F, T, xs = _inputs(shape, 4)
        net.set_norm(1e-4, 1.2e6, 5e-6, 2e3)
        for _ in range(3):
            net.train_step(_cuda(F), 0.5, _cuda(T), _cuda(xs), 1e-3, want_loss=False)
        out.append(net.get_weights())
    assert np.array_equal(out[0], out[1])


# --------------------------------------------------------------------------- guess + fallback
def _shell_ctx(sts, shape):
    from helpers import gpu_spitzer, small_shell
    w = small_shell(shape)
    ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], sts.SHELL_BC, u_lo=w["T_inner"])
    return w, ctx


def test_guess_fallback(gpu_lib):
    sts = gpu_lib
    shape = (6, 8, 16)
    w, ctx = _shell_ctx(sts, shape)
    dt = 50 * ctx.dt_euler()
    net = sts.Cnn(ctx)
    T = _cuda(w["T"])
    # zero network: x0 = T_prev exactly, equal residuals, the network's guess is kept
    x0, used, (rn, rp) = net.guess(T, dt)
    assert used and rn == rp and np.array_equal(_host(x0), w["T"])
    # a network far off: the residual test rejects it and x0 = T_prev
    bad = np.zeros(net.nparam, np.float32)
    bad[-1] = 1.0  # output bias
    net.set_weights(bad)
    net.set_norm(1.0, 0.0, 1.0, 1e9)
    x0, used, (rn, rp) = net.guess(T, dt)
    assert not used and rn > rp and np.array_equal(_host(x0), w["T"])
    # a guess that overflows FP64: non-finite, rejected
    bad = np.zeros(net.nparam, np.float32)
    bad[-1] = 3e38
    net.set_weights(bad)
    net.set_norm(1.0, 0.0, 1.0, 1e300)
    x0, used, (rn, rp) = net.guess(T, dt)
    assert not used and not np.isfinite(rn) and np.array_equal(_host(x0), w["T"])


def test_errors_and_weights_roundtrip(gpu_lib):
    sts = gpu_lib
    ctx = _ctx(sts, (3, 4, 8))
    with pytest.raises(sts.StsError):
        sts.Cnn(ctx, layers=1)
    with pytest.raises(sts.StsError):
        sts.Cnn(ctx, channels=8)
    net = sts.Cnn(ctx)
    assert net.nparam == 15169
    w = np.random.default_rng(0).standard_normal(net.nparam).astype(np.float32)
    net.set_weights(w)
    assert np.array_equal(net.get_weights(), w)
    with pytest.raises(sts.StsError):
        net.set_weights(w[:-1])
    bad = w.copy()
    bad[3] = np.nan
    with pytest.raises(sts.StsError):
        net.set_weights(bad)
    with pytest.raises(sts.StsError):
        net.set_norm(0.0, 0.0, 1.0, 1.0)
    x = _dev16(np.zeros((16, 3, 4, 8)))
    with pytest.raises(sts.StsError):
        net.conv(4, 0, x)
    with pytest.raises(sts.StsError):
        net.conv(0, 6, x)


def test_moments(gpu_lib):
    sts = gpu_lib
    shape = (5, 6, 40)
    ctx = _ctx(sts, shape)
    net = sts.Cnn(ctx)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(shape) * 5 + 2
    y = rng.standard_normal(shape)
    m, r = net.moments(_cuda(x), _cuda(y), 0.5)
    d = 0.5 * (x - y)
    assert m == pytest.approx(d.mean(), rel=1e-12)
    assert r == pytest.approx(np.sqrt(np.mean(d * d)), rel=1e-12)
    m, r = net.moments(_cuda(x))
    assert m == pytest.approx(x.mean(), rel=1e-12)
