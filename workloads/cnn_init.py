"""Seeded initial weights of the learned-guess CNN and the flat weight-vector
layout of the C ABI (cnn_set_weights).  Random draws and array layout only.

Network: `layers` 3x3x3 convolutions, 2 -> channels -> ... -> channels -> out_ch
(1 for the initial-guess network, 4 for the factor network).
Flat vector, per layer l: W[c_out][c_in][3][3][3] then bias[c_out].
"""
from __future__ import annotations

import numpy as np


def layer_dims(layers: int = 4, channels: int = 16, in_ch: int = 2, out_ch: int = 1):
    return [in_ch] + [channels] * (layers - 1) + [out_ch]


def he_normal(layers: int = 4, channels: int = 16, seed: int = 0, out_ch: int = 1):
    """[(W, b)] with W ~ N(0, 2 / fan_in), fan_in = 27 c_in, and zero biases."""
    rng = np.random.default_rng(seed)
    d = layer_dims(layers, channels, out_ch=out_ch)
    out = []
    for l in range(layers):
        W = rng.standard_normal((d[l + 1], d[l], 3, 3, 3)) * np.sqrt(2.0 / (27 * d[l]))
        out.append([W, np.zeros(d[l + 1])])
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in params]
                          ).astype(np.float32)


def unflatten(vec, layers: int = 4, channels: int = 16, out_ch: int = 1):
    d = layer_dims(layers, channels, out_ch=out_ch)
    vec = np.asarray(vec, np.float64)
    out, q = [], 0
    for l in range(layers):
        nw = d[l + 1] * d[l] * 27
        W = vec[q:q + nw].reshape(d[l + 1], d[l], 3, 3, 3)
        q += nw
        b = vec[q:q + d[l + 1]].copy()
        q += d[l + 1]
        out.append([W.copy(), b])
    if q != vec.size:
        raise ValueError(f"weight vector has {vec.size} values, expected {q}")
    return out
