"""The learned forms at the size they are specified for: the 128 x 128 x 256
shell, training on seeds 0-199 and testing on seeds 200-249, one backward-
Euler step per seed at dt = 200 dt_Euler, Jacobi-PCG to 1e-8 as the
baseline (Sec. 2.2, Fig. "pcg"; point Jacobi is PC1 of Sec. 2.3).

  * initial guess: the network trained on (rhs, T_prev) -> BE solutions of
    the plain solver (rtol 1e-10), then Jacobi-PCG from the zero, previous-
    step and network guesses (the network's guess falls back to T_prev when
    its residual is larger);
  * learned factor M^-1 = G G^T: the factor network trained on the
    objective ||G^T A G z - z||^2 / N with seeded probe vectors, then PCG with
    the factor from the previous-step and network guesses (Jacobi fallback
    if it does not reach the tolerance).

Every solve reaches rtol 1e-8; the test checks what each learned form gains
in iterations and prints iterations and times."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPE = (128, 128, 256)
RATIO = 200.0


@pytest.fixture(scope="module")
def full(gpu_lib, request):
    import torch
    from paper_1610_01265_amd import learned
    from workloads import flatten, he_normal
    train = learned.host_fields(SHAPE, range(0, 200), 16)
    test = learned.host_fields(SHAPE, range(200, 250), 16)
    prob = learned.Problem(SHAPE)
    net = gpu_lib.Cnn(prob.ctx)
    net.set_weights(flatten(he_normal(4, 16, 0)))
    pairs = learned.make_pairs(prob, train, RATIO, rtol=1e-10)
    learned.fit_norm(net, pairs)
    hist = learned.train(net, pairs, 4, 1e-3)
    del pairs
    torch.cuda.synchronize()
    guess = learned.summary(learned.evaluate(prob, net, test, RATIO, 1e-8))
    guess["loss_per_epoch"] = hist
    pc = gpu_lib.CnnPC(prob.ctx)
    params = he_normal(4, 16, 1, out_ch=4)
    params[3][0] = params[3][0] * 0.0  # the factor starts at point Jacobi
    pc.set_weights(flatten(params))
    learned.fit_factor_norm(pc, train)
    fhist = learned.train_factor(prob, pc, train, RATIO, epochs=2, lr=2e-3)
    del train
    factor = learned.factor_summary(learned.evaluate_factor(prob, pc, test, RATIO, 1e-8, net))
    factor["objective_per_epoch"] = fhist
    capman = request.config.pluginmanager.getplugin("capturemanager")
    with capman.global_and_fixture_disabled():
        print(f"\n[learned, 128x128x256, seeds 200-249] guess: {guess}\nfactor: {factor}",
              flush=True)
    yield guess, factor
    pc.close()
    net.close()
    prob.ctx.close()


def test_guess_at_full_size(full):
    guess, _ = full
    h = guess["loss_per_epoch"]
    assert all(np.isfinite(h)) and h[-1] < 0.5 * h[0]
    assert guess["network_kept"] >= 45
    it = guess["mean_iters"]
    assert it["network"] < it["previous"] < it["zero"]


def test_factor_at_full_size(full):
    _, factor = full
    h = factor["objective_per_epoch"]
    assert all(np.isfinite(h)) and h[-1] < h[0]
    assert factor["factor_kept"] == factor["cases"]
    it = factor["mean_iters"]
    assert it["factor_previous"] < it["jacobi_previous"]
    assert it["factor_network"] <= it["factor_previous"]
