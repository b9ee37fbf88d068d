"""Learned initial guess for the backward-Euler solve, end to end.

The paper's PCG (Sec. 2.2, Fig. "pcg") starts from x_0 = u^n.  This module
trains the library's CNN (sts_cnn) to predict a better x_0 and compares the
guesses:
  * training pairs: for each seed, the temperature T_prev of that seed, the
    Spitzer operator frozen at T_prev, dt = ratio * dt_E, F_prev = F(T_prev)
    and x_star, the BE solution from plain Jacobi-PCG at a tight tolerance;
  * scalings from the training set (cnn_moments): rhs_scale = 1 / rms(dt F),
    T_shift = mean T, T_scale = 1 / std T, delta_scale = rms(x_star - T);
  * training: cnn_train_step over the pairs in seeded random order;
  * evaluation: Jacobi-PCG to the target tolerance from x_0 = 0, from
    x_0 = T_prev and from cnn_guess (with its residual fallback).
Orchestration only: every arithmetic step runs in libsts; torch holds device
memory.  The seeded fields come from the workloads package.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from multiprocessing.pool import ThreadPool

import numpy as np
import torch

from . import _binding as B

KAPPA0 = 1e-15
T_INNER = 1.5e6


@dataclass
class Pair:
    seed: int
    T: torch.Tensor
    F: torch.Tensor
    dt: float
    x_star: torch.Tensor | None
    iters: int = 0


def _temperature(args):
    from workloads import shell_faces, temperature
    shape, seed = args
    rf, thf, phf = shell_faces(*shape)
    return seed, temperature(rf, thf, phf, seed)


def host_fields(shape, seeds, workers=8):
    """[(seed, T)] for each seed, generated on the host by a pool of threads
    of this process (numpy's generators and array passes release the
    interpreter lock, so the threads run in parallel).  No child process is
    ever started, whether or not this process holds the GPU."""
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 4:
        return [_temperature((shape, s)) for s in seeds]
    with ThreadPool(min(workers, len(seeds))) as pool:
        return pool.map(_temperature, [(shape, s) for s in seeds])


class Problem:
    """Grid, dipole field and one sts context on the current device."""

    def __init__(self, shape):
        from workloads import dipole_bhat, shell_faces
        self.shape = tuple(shape)
        rf, thf, phf = shell_faces(*shape)
        self.ctx = B.Context(B.SPHERICAL, rf, thf, phf, B.SHELL_BC)
        self.ctx.set_dirichlet(0, value=T_INNER)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        self.b = [dev(a) for a in dipole_bhat(rf, thf, phf)]

    def set_temperature(self, T: torch.Tensor) -> float:
        """Freeze the operator at T; returns dt_E."""
        self.ctx.set_spitzer(T, KAPPA0, *self.b)
        return self.ctx.dt_euler()


def make_pairs(prob: Problem, fields, ratio=200.0, rtol=1e-10, maxit=20000, solve=True):
    """Training pairs from host fields [(seed, T)] (host_fields)."""
    pairs = []
    for seed, T_host in fields:
        T = torch.from_numpy(T_host).cuda()
        dt = ratio * prob.set_temperature(T)
        F = prob.ctx.apply_F(T)
        xs, it = None, 0
        if solve:
            xs = T.clone()
            it, _, _ = prob.ctx.be_pcg_solve(T, xs, dt, B.PC_JACOBI, rtol=rtol, maxit=maxit)
        pairs.append(Pair(seed, T, F, dt, xs, it))
    torch.cuda.synchronize()
    return pairs


def fit_norm(net: B.Cnn, pairs):
    """The four scalings of the network from the training pairs."""
    ms = np.array([net.moments(p.F, None, p.dt) for p in pairs])
    mt = np.array([net.moments(p.T) for p in pairs])
    md = np.array([net.moments(p.x_star, p.T) for p in pairs])
    rhs_rms = np.sqrt(np.mean(ms[:, 1] ** 2))
    t_mean = np.mean(mt[:, 0])
    t_var = np.mean(mt[:, 1] ** 2) - t_mean ** 2
    d_rms = np.sqrt(np.mean(md[:, 1] ** 2))
    norm = (1.0 / rhs_rms, t_mean, 1.0 / np.sqrt(t_var), d_rms)
    net.set_norm(*norm)
    return norm


def train(net: B.Cnn, pairs, epochs=4, lr=1e-3, seed=0, log=None):
    """Adam over the pairs in seeded random order; returns the mean loss per epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        for q in order:
            p = pairs[q]
            tot += net.train_step(p.F, p.dt, p.T, p.x_star, lr)
        hist.append(tot / len(pairs))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.4g}")
    return hist


@dataclass
class GuessResult:
    seed: int
    iters: dict = field(default_factory=dict)    # guess name -> PCG iterations
    seconds: dict = field(default_factory=dict)  # guess name -> solve time (s)
    relres0: dict = field(default_factory=dict)  # guess name -> initial relative residual
    used_net: bool = True


def evaluate(prob: Problem, net: B.Cnn, fields, ratio=200.0, rtol=1e-8, maxit=20000):
    """Jacobi-PCG to rtol from the zero, previous-step and network guesses, on
    host fields [(seed, T)] (host_fields)."""
    out = []
    ctx = prob.ctx
    for seed, T_host in fields:
        T = torch.from_numpy(T_host).cuda()
        dt = ratio * prob.set_temperature(T)
        res = GuessResult(seed)
        t0 = time.perf_counter()
        g, used, (rn, rp) = net.guess(T, dt)
        t_guess = time.perf_counter() - t0
        res.used_net = used
        guesses = {"zero": torch.zeros_like(T), "previous": T.clone(), "network": g}
        for name, x in guesses.items():
            res.relres0[name] = ctx.be_residual(T, x, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, _, _ = ctx.be_pcg_solve(T, x, dt, B.PC_JACOBI, rtol=rtol, maxit=maxit)
            res.seconds[name] = time.perf_counter() - t0
            res.iters[name] = it
        res.seconds["network"] += t_guess
        out.append(res)
    return out


def summary(results):
    names = ("zero", "previous", "network")
    return {
        "mean_iters": {n: float(np.mean([r.iters[n] for r in results])) for n in names},
        "mean_seconds": {n: float(np.mean([r.seconds[n] for r in results])) for n in names},
        "median_relres0": {n: float(np.median([r.relres0[n] for r in results])) for n in names},
        "network_kept": int(sum(r.used_net for r in results)),
        "cases": len(results),
    }


# ---- the learned factor M^-1 = G G^T (STS_PC_FACTOR) ------------------------

def probes(shape, count=8, seed=0):
    """Seeded Rademacher probe vectors (+-1 per cell) on the device: the
    random input of the factor's training objective."""
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(rng.choice([-1.0, 1.0], size=tuple(shape))).cuda()
            for _ in range(count)]


def fit_factor_norm(net: B.CnnPC, fields):
    """Temperature scalings of the factor network's input from the training
    fields (host arrays)."""
    m = np.mean([np.mean(T) for _, T in fields])
    v = np.mean([np.mean(T * T) for _, T in fields]) - m * m
    net.set_norm(m, 1.0 / np.sqrt(v))
    return m, np.sqrt(v)


def train_factor(prob: Problem, net: B.CnnPC, fields, ratio=200.0, epochs=2, lr=2e-3, seed=0,
                 nprobe=8, log=None):
    """Adam on the factor objective: for every training field (seed, T) the
    operator is frozen at T, dt = ratio dt_E, and one step is taken with the
    next probe vector; fields in seeded random order.  Returns the mean
    objective per epoch."""
    rng = np.random.default_rng(seed)
    zs = probes(prob.shape, nprobe, seed)
    dev = [(s, torch.from_numpy(T).cuda()) for s, T in fields]
    hist, k = [], 0
    for ep in range(epochs):
        tot = 0.0
        for q in rng.permutation(len(dev)):
            _, T = dev[q]
            dt = ratio * prob.set_temperature(T)
            tot += net.train_step(T, dt, zs[k % nprobe], lr)
            k += 1
        hist.append(tot / len(dev))
        if log:
            log(f"factor epoch {ep}: mean objective {hist[-1]:.4g}")
    return hist


def solve_factor(ctx, u_n, x, dt, rtol=1e-8, maxit=20000):
    """PCG with the context's factor; the fallback is Jacobi-PCG, from the
    last iterate if the factor's solve did not reach rtol within maxit, from
    the initial guess after a breakdown.  Returns (iterations, used_factor)."""
    x0 = x.clone()
    try:
        it, _, st = ctx.be_pcg_solve(u_n, x, dt, B.PC_FACTOR, rtol=rtol, maxit=maxit,
                                     allow_not_converged=True)
    except B.StsError as e:
        if e.code != B.STS_BREAKDOWN:
            raise
        x.copy_(x0)
        it2, _, _ = ctx.be_pcg_solve(u_n, x, dt, B.PC_JACOBI, rtol=rtol, maxit=maxit)
        return it2, False
    if st == B.STS_OK:
        return it, True
    it2, _, _ = ctx.be_pcg_solve(u_n, x, dt, B.PC_JACOBI, rtol=rtol, maxit=maxit)
    return it + it2, False


def evaluate_factor(prob: Problem, net_pc: B.CnnPC, fields, ratio=200.0, rtol=1e-8,
                    net_guess: B.Cnn | None = None):
    """Per test field: Jacobi-PCG and factor-PCG from the previous-step guess
    and (with a guess network) from the network's guess: iterations and
    times (the factor's and the guess's set-up included)."""
    out = []
    ctx = prob.ctx
    for seed, T_host in fields:
        T = torch.from_numpy(T_host).cuda()
        dt = ratio * prob.set_temperature(T)
        res = GuessResult(seed)
        runs = [("jacobi_previous", B.PC_JACOBI, False), ("factor_previous", B.PC_FACTOR, False)]
        if net_guess is not None:
            runs += [("jacobi_network", B.PC_JACOBI, True), ("factor_network", B.PC_FACTOR, True)]
        for name, pc, use_guess in runs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if use_guess:
                x, _, _ = net_guess.guess(T, dt)
            else:
                x = T.clone()
            if pc == B.PC_FACTOR:
                used = net_pc.factor(T, dt)
                it, ok = solve_factor(ctx, T, x, dt, rtol)
                res.used_net = res.used_net and used and ok
            else:
                it, _, _ = ctx.be_pcg_solve(T, x, dt, pc, rtol=rtol)
            torch.cuda.synchronize()
            res.seconds[name] = time.perf_counter() - t0
            res.iters[name] = it
        out.append(res)
    return out


def factor_summary(results):
    names = list(results[0].iters)
    return {
        "mean_iters": {n: float(np.mean([r.iters[n] for r in results])) for n in names},
        "mean_seconds": {n: float(np.mean([r.seconds[n] for r in results])) for n in names},
        "factor_kept": int(sum(r.used_net for r in results)),
        "cases": len(results),
    }


def run(shape=(128, 128, 256), train_seeds=range(200), test_seeds=range(200, 250), ratio=200.0,
        epochs=4, lr=1e-3, init_seed=0, train_rtol=1e-10, rtol=1e-8, workers=8, log=print):
    """The whole learned-guess protocol; returns (summary, per-seed results, timings).
    The host fields are generated first, before this call touches the GPU."""
    from workloads import flatten, he_normal
    t = {}
    t0 = time.perf_counter()
    train_fields = host_fields(shape, train_seeds, workers)
    test_fields = host_fields(shape, test_seeds, workers)
    t["fields_s"] = time.perf_counter() - t0
    prob = Problem(shape)
    net = B.Cnn(prob.ctx)
    net.set_weights(flatten(he_normal(4, 16, init_seed)))
    t0 = time.perf_counter()
    pairs = make_pairs(prob, train_fields, ratio, train_rtol)
    del train_fields
    t["pairs_s"] = time.perf_counter() - t0
    fit_norm(net, pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, pairs, epochs, lr, seed=init_seed, log=log)
    torch.cuda.synchronize()
    t["train_s"] = time.perf_counter() - t0
    t["train_steps"] = epochs * len(pairs)
    del pairs
    results = evaluate(prob, net, test_fields, ratio, rtol)
    s = summary(results)
    s["loss_per_epoch"] = hist
    return s, results, t, net, prob


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned initial guess: train on seeded BE solves, "
                                             "compare Jacobi-PCG from zero / previous / network")
    ap.add_argument("--shape", type=int, nargs=3, default=(128, 128, 256))
    ap.add_argument("--train", type=int, nargs=2, default=(0, 200), help="seed range [a, b)")
    ap.add_argument("--test", type=int, nargs=2, default=(200, 250), help="seed range [a, b)")
    ap.add_argument("--ratio", type=float, default=200.0, help="dt / dt_Euler")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--workers", type=int, default=8)
    a = ap.parse_args(argv)
    s, results, t, net, prob = run(tuple(a.shape), range(*a.train), range(*a.test), a.ratio,
                                   a.epochs, a.lr, rtol=a.rtol, workers=a.workers,
                                   log=lambda m: print(m, flush=True))
    s.update(t)
    s["per_seed_iters"] = {r.seed: r.iters for r in results}
    print(json.dumps(s), flush=True)
    net.close()
    prob.ctx.close()


if __name__ == "__main__":
    main()
