"""GPU parity of the factored preconditioner M^-1 = G G^T and its network
(STS_PC_FACTOR, cnn_create_pc) against the oracle (oracle/learned_pc.py).

Factors given to both sides are seeded arrays of BF16-representable values
(the library stores the entries in BF16; the oracle reads the same values in
FP64), so the FP64 paths are compared at 1e-12: the
application z = G G^T r, PCG iterates at equal k (k <= 10), the training
objective and its gradient in the entries; the converged solve by iteration
count (within one) and the residual-test bound.  The network's
factor at known outputs (zero weights, last-layer biases b: o = b) against
the oracle's entry maps rounded to BF16 as the library rounds them; the network gradient against the
oracle's FP64 back-propagation with bf16-rounded activations (tolerance as
the initial-guess network's whole-network test)."""
import numpy as np
import pytest

from helpers import gpu_spitzer, oracle_spitzer, relmax, small_shell
from oracle import cnn as ocnn
from oracle import learned_pc as LP
from oracle import operator as O
from workloads import flatten

pytestmark = pytest.mark.gpu

BC = (1, 0, 0, 0, 2, 2)
RB = ocnn.round_bf16


def _cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _pair(sts, shape, seed=1):
    w = small_shell(shape, seed=seed)
    op = oracle_spitzer(w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                        w["kappa0"], BC, u_lo=w["T_inner"])
    ctx = gpu_spitzer(sts, w["rf"], w["thf"], w["phf"], w["T"], w["br"], w["bt"], w["bp"],
                      w["kappa0"], BC, u_lo=w["T_inner"])
    return w, op, ctx


def _factor32(op, dt, shape, seed, scale=0.3):
    """Seeded factor rounded to BF16 (stored as FP32): the values both sides use."""
    A19, _ = O.be_system(op, np.zeros(shape), dt)
    o = scale * np.random.default_rng(seed).standard_normal((4,) + tuple(shape))
    g = RB(LP.factor_entries(o, A19[0])).astype(np.float32)
    return g, g.astype(np.float64)


SHAPES = [(6, 10, 20), (5, 7, 9), (12, 16, 70)]


@pytest.mark.parametrize("shape", SHAPES)
def test_apply_factor_matches_oracle(gpu_lib, shape):
    w, op, ctx = _pair(gpu_lib, shape)
    dt = 60.0 * O.gershgorin_dt_euler(op)
    g32, g = _factor32(op, dt, shape, 3)
    ctx.set_pc_factor(_cuda(g32))
    r = np.random.default_rng(4).standard_normal(shape)
    z = _host(ctx.apply_pc_factor(_cuda(r)))
    assert relmax(z, LP.apply_Minv(g, r)) <= 1e-13


@pytest.mark.parametrize("shape", SHAPES[:2])
def test_pcg_factor_iterates_and_solution(gpu_lib, shape):
    w, op, ctx = _pair(gpu_lib, shape)
    dt = 100.0 * O.gershgorin_dt_euler(op)
    g32, g = _factor32(op, dt, shape, 5, scale=0.2)
    ctx.set_pc_factor(_cuda(g32))
    ks = (1, 3, 10)
    ref = LP.be_pcg_factor(op, w["T"], dt, g, rtol=1e-10, keep=ks)
    assert ref.converged
    for k, xk in zip(ks, ref.iterates):
        x = _cuda(w["T"])
        it, _, st = ctx.be_pcg_solve(_cuda(w["T"]), x, dt, pc=gpu_lib.PC_FACTOR, rtol=1e-30,
                                     maxit=k, allow_not_converged=True)
        assert it == k and st == gpu_lib.STS_NOT_CONVERGED
        assert relmax(_host(x), xk) <= 1e-12, k
    x = _cuda(w["T"])
    it, rel, st = ctx.be_pcg_solve(_cuda(w["T"]), x, dt, pc=gpu_lib.PC_FACTOR, rtol=1e-10)
    assert st == 0 and rel <= 1e-10 and abs(it - ref.iters) <= 1
    # Converged: with a random factor the two recurrences' rounding drifts
    # apart over the later iterations (measured up to 2.2e-10 of max |x|),
    # so the solutions are held to the bound that any two solutions meeting
    # the residual test obey, 2 rtol ||b|| / lambda_min(A), lambda_min(A) >=
    # min V (A = V - dt S, -S positive semi-definite).
    A19, b = O.be_system(op, w["T"], dt)
    xh = _host(x)
    assert np.linalg.norm(xh - ref.x) <= 2 * 1e-10 * np.linalg.norm(b) / np.min(op.V)
    assert relmax(xh, ref.x) <= 1e-9


@pytest.mark.parametrize("shape", SHAPES)
def test_objective_and_entry_gradient_match_oracle(gpu_lib, shape):
    w, op, ctx = _pair(gpu_lib, shape)
    dt = 50.0 * O.gershgorin_dt_euler(op)
    g32, g = _factor32(op, dt, shape, 6)
    ctx.set_pc_factor(_cuda(g32))
    z = np.random.default_rng(7).choice([-1.0, 1.0], size=shape)
    L, dg = ctx.pc_objective(dt, _cuda(z))
    A19, _ = O.be_system(op, w["T"], dt)
    Lr, dgr = LP.loss_and_grad(g, lambda v: O.apply19(A19, v), z)
    assert abs(L - Lr) <= 1e-12 * Lr
    assert relmax(_host(dg), dgr) <= 1e-12


def test_factor_checks(gpu_lib):
    sts = gpu_lib
    w, op, ctx = _pair(sts, (4, 6, 8))
    dt = 20.0 * O.gershgorin_dt_euler(op)
    x = _cuda(w["T"])
    with pytest.raises(sts.StsError) as e:  # no factor yet
        ctx.be_pcg_solve(_cuda(w["T"]), x, dt, pc=sts.PC_FACTOR)
    assert e.value.code == sts.STS_EINVAL
    g32, _ = _factor32(op, dt, (4, 6, 8), 8)
    bad = g32.copy()
    bad[0, 1, 2, 3] = 0.0
    with pytest.raises(sts.StsError):
        ctx.set_pc_factor(_cuda(bad))
    bad = g32.copy()
    bad[2, 1, 1, 1] = np.nan
    with pytest.raises(sts.StsError):
        ctx.set_pc_factor(_cuda(bad))
    # a positive FP32 diagonal entry below BF16's smallest value rounds to 0
    bad = g32.copy()
    bad[0, 2, 3, 4] = 1e-44
    with pytest.raises(sts.StsError):
        ctx.set_pc_factor(_cuda(bad))
    ctx.set_pc_factor(_cuda(g32))


def _pc_net(sts, ctx, params):
    net = sts.CnnPC(ctx)
    net.set_weights(flatten(params))
    return net


def _zero_params(last_bias):
    dims = [2, 16, 16, 16, 4]
    out = []
    for l in range(4):
        W = np.zeros((dims[l + 1], dims[l], 3, 3, 3))
        b = np.zeros(dims[l + 1]) if l < 3 else np.asarray(last_bias, np.float64)
        out.append([W, b])
    return out


def test_network_factor_at_known_outputs(gpu_lib):
    """Zero weights: o = last-layer bias.  b = 0 gives point Jacobi (up to the
    FP32 storage of the entries); b != 0 the oracle's entry maps."""
    sts = gpu_lib
    shape = (6, 10, 20)
    w, op, ctx = _pair(sts, shape)
    dt = 80.0 * O.gershgorin_dt_euler(op)
    T = _cuda(w["T"])
    net = _pc_net(sts, ctx, _zero_params([0.0, 0.0, 0.0, 0.0]))
    net.set_norm(1.2e6, 1e-5)
    assert net.factor(T, dt)
    A19, _ = O.be_system(op, w["T"], dt)
    r = np.random.default_rng(9).standard_normal(shape)
    z = _host(ctx.apply_pc_factor(_cuda(r)))
    # point Jacobi up to the BF16 storage of d = A_cc^-1/2 (applied twice)
    assert relmax(z, r / A19[0]) <= 2 * 2.0 ** -8
    assert relmax(z, LP.apply_Minv(RB(LP.factor_entries(np.zeros((4,) + shape), A19[0])), r)) \
        <= 1e-12
    net.close()
    b = [0.25, -0.125, 0.0625, 0.5]
    net = _pc_net(sts, ctx, _zero_params(b))
    net.set_norm(1.2e6, 1e-5)
    assert net.factor(T, dt)
    o = np.stack([np.full(shape, v) for v in b])
    g = RB(LP.factor_entries(o, A19[0]))  # the library's BF16 entries
    z = _host(ctx.apply_pc_factor(_cuda(r)))
    assert relmax(z, LP.apply_Minv(g, r)) <= 1e-12
    net.close()


def _oracle_features(op, T, dt, tsh, tsc):
    A19, _ = O.be_system(op, T, dt)
    dte = O.gershgorin_dt_euler(op)
    f0 = np.log(A19[0] / op.V) / np.log1p(dt / dte)
    return np.stack([RB(f0), RB((T - tsh) * tsc)]), A19


def test_network_gradient_matches_oracle(gpu_lib):
    """cnn_pc_grad against the oracle: features, network (bf16-rounded
    activations), entry maps, objective gradient and back-propagation in
    FP64; and cnn_pc_train_step equal to cnn_pc_grad + cnn_adam_step."""
    import torch
    sts = gpu_lib
    shape = (5, 8, 66)
    w, op, ctx = _pair(sts, shape)
    dt = 60.0 * O.gershgorin_dt_euler(op)
    rng = np.random.default_rng(11)
    params = []
    dims = [2, 16, 16, 16, 4]
    for l in range(4):
        W = RB(rng.standard_normal((dims[l + 1], dims[l], 3, 3, 3)) * np.sqrt(2.0 / (27 * dims[l]))
               * (0.3 if l == 3 else 1.0))
        params.append([W, RB(0.05 * rng.standard_normal(dims[l + 1]))])
    tsh, tsc = 1.2e6, 2e-6
    net = _pc_net(sts, ctx, params)
    net.set_norm(tsh, tsc)
    z = rng.choice([-1.0, 1.0], size=shape)
    T = _cuda(w["T"])
    L, grad = net.grad(T, dt, _cuda(z))
    got = _host(grad)
    # oracle
    x, A19 = _oracle_features(op, w["T"], dt, tsh, tsc)
    y, cache = ocnn.forward(params, x, act_round=RB)
    g = RB(LP.factor_entries(y, A19[0]))  # the library's BF16 entries
    Lr, dg = LP.loss_and_grad(g, lambda v: O.apply19(A19, v), z)
    do = LP.grad_outputs(dg, g, A19[0])
    grads = ocnn.backward(params, cache, do)
    assert abs(L - Lr) <= 2e-2 * Lr
    P = sts.CNN_PADDED_PARAMS
    for l in range(4):
        ci, co = dims[l], dims[l + 1]
        gW = got[l * P:l * P + 16 * 16 * 27].reshape(16, 16, 3, 3, 3)[:co, :ci]
        gb = got[l * P + 16 * 16 * 27:(l + 1) * P][:co]
        ref = np.concatenate([grads[l][0].ravel(), grads[l][1]])
        mine = np.concatenate([gW.ravel(), gb])
        d = np.abs(mine - ref) / np.max(np.abs(ref))
        assert np.max(d) < 5e-2 and np.median(d) < 1e-3, (l, np.max(d), np.median(d))
    # the train step is the gradient plus one Adam step
    net2 = _pc_net(sts, ctx, params)
    net2.set_norm(tsh, tsc)
    net2.set_adam(0.9, 0.999, 1e-8)
    net.set_adam(0.9, 0.999, 1e-8)
    net.set_weights(flatten(params))
    L1 = net.train_step(T, dt, _cuda(z), 1e-3)
    L2, g2 = net2.grad(T, dt, _cuda(z))
    net2.adam_step(g2, 1e-3)
    torch.cuda.synchronize()
    assert L1 == L2
    assert np.array_equal(net.get_weights(), net2.get_weights())
    net.close()
    net2.close()


def test_training_lowers_objective_and_iterations(gpu_lib, capsys):
    """A few hundred training steps on one operator: the objective falls
    and the learned factor takes fewer PCG iterations than point Jacobi."""
    import torch
    sts = gpu_lib
    from workloads import he_normal
    shape = (16, 16, 32)
    w, op, ctx = _pair(sts, shape)
    dt = 200.0 * O.gershgorin_dt_euler(op)
    params = he_normal(4, 16, 0, out_ch=4)
    params[3][0] = params[3][0] * 0.0  # start at point Jacobi
    net = _pc_net(sts, ctx, params)
    net.set_norm(float(np.mean(w["T"])), 1.0 / float(np.std(w["T"])))
    T = _cuda(w["T"])
    gen = np.random.default_rng(12)
    losses = []
    for step in range(300):
        z = _cuda(gen.choice([-1.0, 1.0], size=shape))
        losses.append(net.train_step(T, dt, z, 2e-3))
    assert np.mean(losses[-20:]) < 0.9 * np.mean(losses[:5])
    assert net.factor(T, dt)
    xa, xb = _cuda(w["T"]), _cuda(w["T"])
    ia, rel, st = ctx.be_pcg_solve(T, xa, dt, pc=sts.PC_FACTOR, rtol=1e-8)
    ib, _, _ = ctx.be_pcg_solve(T, xb, dt, pc=sts.PC_JACOBI, rtol=1e-8)
    assert st == 0 and rel <= 1e-8
    with capsys.disabled():
        print(f"\n[learned factor] objective {np.mean(losses[:5]):.4f} -> {np.mean(losses[-20:]):.4f}; "
              f"PCG iterations {ia} (factor) vs {ib} (Jacobi)")
    assert ia < ib
    torch.cuda.synchronize()
    net.close()
