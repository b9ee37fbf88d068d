"""GPU parity of the CNN kernels at the grid sizes the learned guess runs on,
where the kernels take their multi-plane paths: 64 x 64 x 256 (each
workgroup marches 2 r-planes through its LDS ring; 2048 weight-gradient work
items over 512 workgroups) and 128 x 128 x 256, the learned-guess workload
(8 r-planes per workgroup, so the ring advances 7 times; 2048 work items).

A whole-grid FP64 oracle convolution at these sizes takes minutes, so the
oracle (oracle/cnn.py, unchanged) runs on 3 x 3 x 3 windows: a convolution
output depends on the 3 x 3 x 3 neighbourhood of its cell, and a weight
gradient over cells whose output gradient vanishes elsewhere is the sum of
the windows' weight gradients.  Windows are gathered with the network's
padding (zero outside r / theta, periodic in phi), and the sampled cells
cover every boundary face, the first and last plane of every r-chunk and
seeded interior cells.  Tolerances as in test_gpu_cnn.py."""
import numpy as np
import pytest

from oracle import cnn as ocnn
from workloads import flatten, he_normal, shell_faces

pytestmark = pytest.mark.gpu

RB = ocnn.round_bf16
# (shape, r-planes per workgroup of the conv / weight-gradient march)
CASES = [((64, 64, 256), 2), ((128, 128, 256), 8)]


def _dev16(x):
    import torch
    C = x.shape[0]
    a = np.zeros((x[0].size, 16), np.float32)
    a[:, :C] = x.reshape(C, -1).T
    return torch.from_numpy(a).to(torch.bfloat16).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _net(sts, shape, seed):
    rf, thf, phf = shell_faces(*shape)
    ctx = sts.Context(sts.SPHERICAL, rf, thf, phf)
    net = sts.Cnn(ctx, 4)
    rng = np.random.default_rng(1000 + seed)
    params = [[RB(W), RB(0.05 * rng.standard_normal(b.shape))]
              for W, b in he_normal(4, 16, seed)]
    net.set_weights(flatten(params))
    return ctx, net, params


def _cells(shape, ci, n_random, seed):
    n0, n1, n2 = shape
    rng = np.random.default_rng(seed)
    out = set()
    for _ in range(n_random):
        out.add((int(rng.integers(n0)), int(rng.integers(n1)), int(rng.integers(n2))))
    for i0 in range(0, n0, ci):  # first and last plane of every r-chunk
        for i in (i0, min(i0 + ci - 1, n0 - 1)):
            out.add((i, int(rng.integers(n1)), int(rng.integers(n2))))
    for i in (0, n0 - 1):
        for j in (0, n1 // 2, n1 - 1):
            for k in (0, 63, 64, n2 - 1):
                out.add((i, j, k))
    for j in (0, 3, 4, n1 - 1):  # theta boundaries and tile-row edges
        for k in (0, n2 - 1):
            out.add((n0 // 2, j, k))
    return sorted(out)


def _window(x, cell):
    """x[:, i-1..i+1, j-1..j+1, k-1..k+1] with the network's padding."""
    i, j, k = cell
    n0, n1, n2 = x.shape[1:]
    w = np.zeros((x.shape[0], 3, 3, 3))
    for a in range(3):
        ii = i + a - 1
        if not 0 <= ii < n0:
            continue
        for b in range(3):
            jj = j + b - 1
            if not 0 <= jj < n1:
                continue
            for c in range(3):
                w[:, a, b, c] = x[:, ii, jj, (k + c - 1) % n2]
    return w


def _centre(y):
    return y[:, 1, 1, 1]


@pytest.mark.parametrize("shape,ci", CASES)
def test_conv_forward_and_input_grad_fullsize(gpu_lib, shape, ci):
    sts = gpu_lib
    ctx, net, params = _net(sts, shape, seed=1)
    rng = np.random.default_rng(60)
    x = RB(np.maximum(rng.standard_normal((16,) + shape), 0.0))
    W, b = params[1]
    got = _host(net.conv(1, sts.CNN_F32, _dev16(x)))
    dy = RB(rng.standard_normal((16,) + shape))
    gdx = _host(net.conv(1, sts.CNN_INPUT_GRAD_F32, _dev16(dy)))
    n0, n1, n2 = shape
    for cell in _cells(shape, ci, 150, 61):
        lin = (cell[0] * n1 + cell[1]) * n2 + cell[2]
        xw = _window(x, cell)
        ref = _centre(ocnn.conv3d(xw, W, b))
        scale = _centre(ocnn.conv3d(np.abs(xw), np.abs(W)))
        assert np.all(np.abs(got[lin, :16] - ref) <= 1e-5 * scale + 1e-30), cell
        dyw = _window(dy, cell)
        refg = _centre(ocnn.conv3d_input_grad(dyw, W, 16))
        scaleg = _centre(ocnn.conv3d_input_grad(np.abs(dyw), np.abs(W), 16))
        assert np.all(np.abs(gdx[lin, :16] - refg) <= 1e-5 * scaleg + 1e-30), cell


@pytest.mark.parametrize("shape,ci", CASES)
def test_weight_grad_fullsize(gpu_lib, shape, ci):
    """Output gradient non-zero on sampled cells only (seeded values), input
    activation random on the whole grid: every work item runs its full march,
    and the result is the sum of the sampled cells' window gradients."""
    sts = gpu_lib
    ctx, net, _ = _net(sts, shape, seed=2)
    rng = np.random.default_rng(70)
    act = RB(np.maximum(rng.standard_normal((16,) + shape), 0.0))
    cells = _cells(shape, ci, 400, 71)
    dy = np.zeros((16,) + shape)
    vals = RB(rng.standard_normal((len(cells), 16)))
    for c, v in zip(cells, vals):
        dy[(slice(None),) + c] = v
    got = _host(net.weight_grad(1, _dev16(act), _dev16(dy)))
    gW = got[:16 * 16 * 27].reshape(16, 16, 3, 3, 3)
    gb = got[16 * 16 * 27:]
    refW = np.zeros((16, 16, 3, 3, 3))
    scaleW = np.zeros_like(refW)
    for c, v in zip(cells, vals):
        aw = _window(act, c)
        dw = np.zeros((16, 3, 3, 3))
        dw[:, 1, 1, 1] = v
        refW += ocnn.conv3d_weight_grad(aw, dw)
        scaleW += ocnn.conv3d_weight_grad(np.abs(aw), np.abs(dw))
    assert np.all(np.abs(gW - refW) <= 1e-5 * scaleW + 1e-30)
    refb = vals.sum(axis=0)
    assert np.all(np.abs(gb - refb) <= 1e-5 * np.abs(vals).sum(axis=0) + 1e-30)
