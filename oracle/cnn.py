"""FP64 reference of the small 3D CNN that predicts the PCG initial guess
(oracle, test-only).

The network (a learned guess for the backward-Euler solve, beside the
paper's PCG of Sec. 2.2 / Fig. "pcg" whose x_0 it replaces):
    input  2 channels: the BE right-hand-side increment dt F(T_prev)
           (= (b - A T_prev) / V) and T_prev, each normalised by scalars;
    conv3x3x3(2 -> C) ReLU, conv(C -> C) ReLU, conv(C -> C) ReLU, conv(C -> 1);
    output the normalised increment; guess x_0 = T_prev + s_delta * output.
Convolutions use "same" padding: zero along axes 0 and 1 (r, theta), circular
along axis 2 (the periodic phi).  Arrays are [channels, n0, n1, n2].

Pinned by tests/test_oracle_cnn.py: a per-element loop convolution (the
definition), exact central differences of the (linear) convolution in its
input and its weights, and finite differences of the network loss.
"""
from __future__ import annotations

import numpy as np

OFFS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]  # tap t = 9a+3b+c+13


def _pad(x):
    """Zero-pad axes 1, 2 (r, theta) and wrap axis 3 (phi) of [C, n0, n1, n2]."""
    x = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    return np.concatenate([x[..., -1:], x, x[..., :1]], axis=-1)


def _shift(xp, off, shape):
    """View of the padded array at cell + off for every cell."""
    a, b, c = off
    n0, n1, n2 = shape
    return xp[:, 1 + a:1 + a + n0, 1 + b:1 + b + n1, 1 + c:1 + c + n2]


def conv3d(x, W, bias=None):
    """y[co] = bias[co] + sum_{ci, taps} W[co, ci, a+1, b+1, c+1] x[ci, cell + (a, b, c)]."""
    x = np.asarray(x, np.float64)
    W = np.asarray(W, np.float64)
    shape = x.shape[1:]
    xp = _pad(x)
    y = np.zeros((W.shape[0],) + shape)
    for (a, b, c) in OFFS:
        y += np.einsum("oi,ixyz->oxyz", W[:, :, a + 1, b + 1, c + 1], _shift(xp, (a, b, c), shape))
    if bias is not None:
        y += np.asarray(bias, np.float64)[:, None, None, None]
    return y


def conv3d_input_grad(dy, W, in_channels):
    """Adjoint of conv3d in x: dx[ci, cell] = sum_{co, taps} W[co, ci, tap] dy[co, cell - off]."""
    dy = np.asarray(dy, np.float64)
    shape = dy.shape[1:]
    dx = np.zeros((in_channels,) + shape)
    dyp = _pad(dy)
    for (a, b, c) in OFFS:
        dx += np.einsum("oi,oxyz->ixyz", W[:, :, a + 1, b + 1, c + 1],
                        _shift(dyp, (-a, -b, -c), shape))
    return dx


def conv3d_weight_grad(x, dy):
    """dW[co, ci, tap] = sum_cells dy[co, cell] x[ci, cell + off]."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    shape = x.shape[1:]
    xp = _pad(x)
    dW = np.zeros((dy.shape[0], x.shape[0], 3, 3, 3))
    for (a, b, c) in OFFS:
        dW[:, :, a + 1, b + 1, c + 1] = np.einsum("oxyz,ixyz->oi", dy, _shift(xp, (a, b, c), shape))
    return dW


def init_params(channels=16, layers=4, in_ch=2, out_ch=1, seed=0):
    """He-normal weights, zero biases (the network's initial state)."""
    rng = np.random.default_rng(seed)
    dims = [in_ch] + [channels] * (layers - 1) + [out_ch]
    params = []
    for l in range(layers):
        fan_in = dims[l] * 27
        W = rng.standard_normal((dims[l + 1], dims[l], 3, 3, 3)) * np.sqrt(2.0 / fan_in)
        params.append([W, np.zeros(dims[l + 1])])
    return params


def forward(params, x, act_round=None):
    """Returns (output, cache).  act_round (optional) rounds each stored
    activation (e.g. to bfloat16) where a reduced-precision implementation
    stores it."""
    acts = [x]
    pre = []
    h = x
    for l, (W, b) in enumerate(params):
        z = conv3d(h, W, b)
        pre.append(z)
        if l < len(params) - 1:
            h = np.maximum(z, 0.0)
            if act_round is not None:
                h = act_round(h)
            acts.append(h)
        else:
            h = z
    return h, (acts, pre)


def mse_loss(y, target):
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dy):
    """Gradients of a scalar loss with dL/d(output) = dy, for each (W, b)."""
    acts, pre = cache
    grads = [None] * len(params)
    g = dy
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = [conv3d_weight_grad(acts[l], g), g.sum(axis=(1, 2, 3))]
        if l > 0:
            g = conv3d_input_grad(g, W, W.shape[1]) * (pre[l - 1] > 0.0)
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; state = (m, v, t)."""
    m, v, t = state
    t += 1
    for l in range(len(params)):
        for q in range(2):
            m[l][q] = beta1 * m[l][q] + (1 - beta1) * grads[l][q]
            v[l][q] = beta2 * v[l][q] + (1 - beta2) * grads[l][q] ** 2
            mh = m[l][q] / (1 - beta1 ** t)
            vh = v[l][q] / (1 - beta2 ** t)
            params[l][q] = params[l][q] - lr * mh / (np.sqrt(vh) + eps)
    return (m, v, t)


def adam_init(params):
    m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    return (m, v, 0)


def round_bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
