"""Pins for the FP64 CNN oracle: the loop definition of the convolution with
its padding rules, exact central differences of the linear convolution, and
finite differences of the network loss."""
import numpy as np
import pytest

from oracle import cnn


def loop_conv(x, W, bias):
    C, n0, n1, n2 = x.shape
    out = np.zeros((W.shape[0], n0, n1, n2))
    for co in range(W.shape[0]):
        for i in range(n0):
            for j in range(n1):
                for k in range(n2):
                    s = bias[co]
                    for ci in range(C):
                        for a in (-1, 0, 1):
                            for b in (-1, 0, 1):
                                for c in (-1, 0, 1):
                                    ii, jj, kk = i + a, j + b, (k + c) % n2
                                    if 0 <= ii < n0 and 0 <= jj < n1:
                                        s += W[co, ci, a + 1, b + 1, c + 1] * x[ci, ii, jj, kk]
                    out[co, i, j, k] = s
    return out


def test_conv_matches_loop_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(cnn.conv3d(x, W, b), loop_conv(x, W, b), rtol=1e-13, atol=1e-12)


def test_padding_zero_in_r_theta_circular_in_phi():
    x = np.zeros((1, 3, 3, 4))
    x[0, 0, 0, 0] = 1.0
    W = np.ones((1, 1, 3, 3, 3))
    y = cnn.conv3d(x, W)
    assert y[0, 0, 0, 3] == 1.0   # phi wraps
    assert y[0, 2, 0, 0] == 0.0   # r does not
    assert y[0, 0, 2, 0] == 0.0   # theta does not


def test_input_and_weight_gradients_exact_central_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 3, 4, 5))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    dy = rng.standard_normal((2, 3, 4, 5))
    L = lambda x_, W_: np.sum(dy * cnn.conv3d(x_, W_))  # noqa: E731  (linear in each)
    gx = cnn.conv3d_input_grad(dy, W, 3)
    gW = cnn.conv3d_weight_grad(x, dy)
    h = 0.5
    for idx in [(0, 0, 0, 0), (1, 2, 3, 4), (2, 1, 0, 4), (0, 2, 3, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (L(x + e, W) - L(x - e, W)) / (2 * h)
        assert fd == pytest.approx(gx[idx], rel=1e-11, abs=1e-11)
    for idx in [(0, 0, 0, 0, 0), (1, 2, 2, 1, 0), (0, 1, 1, 1, 2), (1, 0, 2, 2, 2)]:
        e = np.zeros_like(W)
        e[idx] = h
        fd = (L(x, W + e) - L(x, W - e)) / (2 * h)
        assert fd == pytest.approx(gW[idx], rel=1e-11, abs=1e-11)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params(channels=4, layers=4, seed=3)
    for W, b in params:
        b += 0.1 * rng.standard_normal(b.shape)
    x = rng.standard_normal((2, 3, 4, 6))
    target = rng.standard_normal((1, 3, 4, 6))

    def loss():
        y, _ = cnn.forward(params, x)
        return cnn.mse_loss(y, target)[0]

    y, cache = cnn.forward(params, x)
    _, dy = cnn.mse_loss(y, target)
    grads = cnn.backward(params, cache, dy)
    h = 1e-6
    for l, q, idx in [(0, 0, (1, 0, 1, 1, 1)), (1, 0, (2, 3, 0, 2, 1)), (3, 0, (0, 2, 1, 0, 2)),
                      (2, 1, (1,)), (3, 1, (0,))]:
        p = params[l][q]
        old = p[idx]
        p[idx] = old + h
        lp = loss()
        p[idx] = old - h
        lm = loss()
        p[idx] = old
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(grads[l][q][idx], rel=1e-5, abs=1e-9)


def test_round_bf16():
    # bf16 spacing at 1 is 2^-7; 1 + 2^-8 and 1 + 3 2^-8 are ties -> even significand
    vals = np.array([1.0, 1.00390625, 1.01171875, -3.14159, 1e-3, 65504.0, 1.001953125])
    r = cnn.round_bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.015625 and r[6] == 1.0
    assert abs(r[3] + 3.140625) < 1e-12
    # representable values are fixed points
    assert np.array_equal(cnn.round_bf16(r), r)


def test_adam_moves_against_gradient():
    params = cnn.init_params(channels=2, layers=2, seed=0)
    g = [[np.ones_like(W), np.ones_like(b)] for W, b in params]
    st = cnn.adam_init(params)
    before = [W.copy() for W, _ in params]
    cnn.adam_step(params, g, st, lr=1e-2)
    for (W, _), W0 in zip(params, before):
        assert np.allclose(W - W0, -1e-2, rtol=1e-6)


def test_adam_matches_closed_form_sums_over_steps():
    """Adam after t steps with a varying gradient, against the unrolled moment
    sums m_t = (1-b1) sum_s b1^(t-s) g_s, v_t = (1-b2) sum_s b2^(t-s) g_s^2 and
    the bias corrections 1 - b^t of that t.  b1 != b2 (0.5 and 0.75), so
    swapping them, dropping a correction or using the wrong t fails."""
    b1, b2, lr, eps = 0.5, 0.75, 1e-2, 1e-8
    rng = np.random.default_rng(7)
    params = cnn.init_params(channels=2, layers=2, seed=1)
    st = cnn.adam_init(params)
    p0 = [[W.copy(), b.copy()] for W, b in params]
    gs = []
    for t in range(1, 6):
        g = [[rng.standard_normal(W.shape), rng.standard_normal(b.shape)] for W, b in params]
        gs.append(g)
        st = cnn.adam_step(params, g, st, lr, beta1=b1, beta2=b2, eps=eps)
        assert st[2] == t
        # replay the parameter trajectory in closed form
        for l in range(len(params)):
            for q in range(2):
                x = p0[l][q].copy()
                for tt in range(1, t + 1):
                    m = (1 - b1) * sum(b1 ** (tt - s) * gs[s - 1][l][q] for s in range(1, tt + 1))
                    v = (1 - b2) * sum(b2 ** (tt - s) * gs[s - 1][l][q] ** 2
                                       for s in range(1, tt + 1))
                    x = x - lr * (m / (1 - b1 ** tt)) / (np.sqrt(v / (1 - b2 ** tt)) + eps)
                assert np.max(np.abs(params[l][q] - x)) <= 1e-13
    # a constant gradient g gives steps of -lr g / (|g| + eps) at every t
    params = cnn.init_params(channels=2, layers=2, seed=2)
    st = cnn.adam_init(params)
    g = [[np.full_like(W, -0.3), np.full_like(b, 2.0)] for W, b in params]
    for _ in range(4):
        before = [[W.copy(), b.copy()] for W, b in params]
        st = cnn.adam_step(params, g, st, lr, beta1=b1, beta2=b2, eps=eps)
        for (W, b), (W0, bb0) in zip(params, before):
            assert np.allclose(W - W0, lr * 0.3 / (0.3 + eps), rtol=1e-12)
            assert np.allclose(b - bb0, -lr * 2.0 / (2.0 + eps), rtol=1e-12)
