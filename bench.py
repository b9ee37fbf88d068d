"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the synthetic shell input:
  * coefficient setup (lagged Spitzer diffusivity, face / edge weights,
    Gershgorin dt_Euler);
  * one RKL2 super-step at dt = f dt_Euler;
  * one BE step solved by Jacobi-PCG and one by block-ILU0(8^3)-PCG, each
    to the workload's relative residual;
  * the FP32 precision form: FP32 coefficient setup, RKL2 step, Jacobi-PCG
    (mixed-precision refinement to the same FP64 residual);
  * artificial viscosity on a 3-component velocity field: RKL2 step of all
    three components and one Jacobi-PCG BE solve per component;
  * the learned initial guess on its own grid (128 x 128 x 256, dt = 200
    dt_Euler): coefficient set-up, cnn_guess (network + residual fallback),
    Jacobi-PCG from that guess and from the previous-step guess, and one
    training step of the network;
  * the super-step variants of Sec. 6 on the temperature: RKL2 in 10
    sub-cycles, explicit Euler over a quarter step then RKL2, and RKL1 with
    one extra stage;
  * RKL2 with the diffusivity taken from every stage value (no lagging):
    one rkl2_step_nonlinear (its own set-up at u^n included);
  * resistive diffusion of the edge-staggered vector potential (Eq. mhd:a):
    one BE step by PC1-PCG at dt = f x its own explicit limit.
Inputs are resident in HBM before the timed region.  After the timed steps,
a march of 10 successive steps per method (RKL2, Jacobi-PCG, block-ILU0-PCG)
re-freezes kappa from each method's evolving state at every step and reports
per-step times, stage counts and iteration counts ("successive_steps").  Each phase is bracketed
by HIP events on the library's stream; phase times are medians over the timed
steps (means beside them).  `value` is the RKL2 throughput in cell-stage
updates per second; the BE solve times are reported beside it.  The host
fields of the learned guess's training set are generated in a process pool
before this process touches the GPU.

The roofline entry is for the RKL2 stage kernel (the fused stencil + stage
update): algorithmic bytes per launch (72 B/cell for stage 1, 88 B/cell for
stages 2..s) over the mean launch duration (median RKL2 phase time / s).  `traffic`
is the copy-calibrated HBM byte count per launch from the committed counter
summary of the same kernel, or null when the kernel's sources have changed
since those counters were taken.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_march_rkl2_stage_shell256_pmc.txt")
LEARNED_SHAPE = (128, 128, 256)  # grid of the learned-guess workload
LEARNED_RATIO = 200.0            # its dt / dt_Euler
STAGE_SOURCES = ["k_stencil.hip", "k_row.h", "k_common.h", "sts_internal.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="shell256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phases",
                    default="rkl2,jacobi,ilu0,fp32,visc,learned,variants,nonlinear,resist",
                    help="comma list of timed phases (profiling runs)")
    ap.add_argument("--march-steps", type=int, default=10,
                    help="successive steps per method in the march run after the timed steps "
                         "(0 skips it)")
    ap.add_argument("--learned-train-seeds", type=int, default=200,
                    help="training pairs (seeds 1..N) for the network before the timed steps")
    ap.add_argument("--learned-epochs", type=int, default=4)
    ap.add_argument("--pair-workers", type=int, default=8,
                    help="host processes generating the training fields before the GPU is "
                         "initialised (1: in this process)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="before the steps, run a plain device copy of 4 fields (known bytes) "
                         "that calibrates the HBM byte counters")
    return ap.parse_args()


def stage_source_hash():
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_1610_01265_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(ncell):
    """Copy-calibrated HBM bytes per stage launch from the counter summary,
    if it was taken on the current kernel sources and the same cell count."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != stage_source_hash():
            return None
        if int(kv.get("cells", -1)) != ncell:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(w, dt_factor, budget_s=12.0, max_steps=8, max_cells=1 << 22):
    """The oracle as it stands, timed on this host: RKL2 super-steps of the
    same workload, repeated until about budget_s seconds (the bounded sample).
    Grids above max_cells are sampled by their innermost r-planes (the slab
    keeps the Dirichlet inner boundary; its outer cut is zero-flux), so that
    one super-step stays within a few seconds."""
    from oracle import operator as O
    from oracle import rkl2 as orkl2
    T = w["T"]
    n12 = T.shape[1] * T.shape[2]
    nr = min(T.shape[0], max(1, max_cells // n12))
    sl = slice(0, nr)
    D = O.spitzer_tensor(T[sl], w["kappa0"], w["br"][sl], w["bt"][sl], w["bp"][sl])
    op = O.assemble("spherical", w["rf"][:nr + 1], w["thf"], w["phf"], D, O.SHELL_BC,
                    u_lo=w["T_inner"])
    dte = O.gershgorin_dt_euler(op)
    s = orkl2.stage_count(dt_factor)
    Ts = np.ascontiguousarray(T[sl])
    t = 0.0
    n = 0
    while n < max_steps and (n == 0 or t < budget_s):
        t0 = time.perf_counter()
        orkl2.rkl2_step(lambda v: O.apply_F(op, v), Ts, dt_factor * dte, s)
        t += time.perf_counter() - t0
        n += 1
    cells = Ts.size
    part = ("" if nr == T.shape[0] else
            f"the {nr} innermost r-planes ({nr}x{T.shape[1]}x{T.shape[2]} = {cells} cells) of ")
    return {"value": n * cells * s / t, "unit": "cell-stage updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} RKL2 super-step(s) (s={s}) of {part}{w['workload'].name} "
                      f"({T.size} cells), numpy FP64, one thread, {t:.1f} s"}


def progress(msg):
    """One line on stderr per stage of the run (stdout carries only the result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Timer:
    """Named HIP-event intervals on one stream."""

    def __init__(self, torch, stream):
        self.torch, self.stream, self.marks = torch, stream, []

    def mark(self, name):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        self.marks.append((name, ev))

    def intervals(self):
        out = {}
        for (a, ea), (_, eb) in zip(self.marks, self.marks[1:]):
            out[a] = out.get(a, 0.0) + ea.elapsed_time(eb)
        return out  # ms


def run_march(torch, sts, ctx, T, b, kappa0, wl, nsteps, stream):
    """The lagged protocol over nsteps successive steps: each method marches
    its own state from T, re-freezing kappa from that state at the start of
    every step; dt stays at f x the first step's dt_Euler and the RKL2 stage
    count follows each step's own dt_Euler.  Per-step times (set-up included)
    come from HIP events on the library's stream."""
    ctx.set_spitzer(T, kappa0, *b)
    dt = wl.dt_factor * ctx.dt_euler()
    ua, ub = torch.empty_like(T), torch.empty_like(T)
    out = {"steps": nsteps, "dt_over_first_dt_euler": wl.dt_factor}
    for name in ("rkl2", "jacobi", "ilu0"):
        ua.copy_(T)
        evs, work = [], []
        for _ in range(nsteps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.set_spitzer(ua, kappa0, *b)
            if name == "rkl2":
                work.append(ctx.rkl2_step(ua, dt))
            else:
                ub.copy_(ua)
                pc = sts.PC_JACOBI if name == "jacobi" else sts.PC_BLOCK_ILU0
                it, _, _ = ctx.be_pcg_solve(ua, ub, dt, pc=pc, block=wl.block, rtol=wl.rtol)
                work.append(it)
                ua, ub = ub, ua
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ms = [a.elapsed_time(z) for a, z in evs]
        out[name] = {"ms_per_step": ms, "mean_ms": sum(ms) / nsteps,
                     ("stages" if name == "rkl2" else "iters"): work}
    out["speedup_vs_fp64_jacobi_pcg"] = {
        k: out["jacobi"]["mean_ms"] / out[k]["mean_ms"] for k in ("rkl2", "ilu0")}
    return out


def nonlinear_entry(ph, info, ncell):
    """RKL2 with kappa from every stage value against the lagged protocol
    (coefficient set-up + RKL2 step).  Stage kernel bytes: 48 B/cell for stage
    1 (u, b read; F0, u_1 written), 64 B/cell for stages 2..s (u_{k-1}, b,
    u_{k-2}, u_0, F0 read; u_k written); its mean launch time is estimated as
    (phase - set-up) / s."""
    s = info.get("s_nl")
    if not s or "nl_rkl2" not in ph:
        return None
    t = ph["nl_rkl2"]
    lagged = ph.get("setup", 0.0) + ph.get("rkl2", 0.0)
    stage_us = max(t - ph.get("setup", 0.0), 0.0) / s * 1e3
    alg = (48 + 64 * (s - 1)) * ncell / s
    gbs = alg / (stage_us * 1e-6) / 1e9 if stage_us > 0 else None
    return {"ms": t, "stages": s, "lagged_setup_plus_rkl2_ms": lagged,
            "time_vs_lagged": t / lagged if lagged > 0 else None,
            "stage_kernel": {"mean_launch_us_est": stage_us, "alg_bytes_per_launch": alg,
                             "achieved_GBs": gbs,
                             "frac_hbm": gbs / HBM_PEAK_GBS if gbs else None}}


RES_ETA = 1.0  # c^2 eta / 4 pi in code units (it cancels in dt / dt_Euler)


def resist_entry(ph, info, ctxr):
    """BE + PC1 of the resistive term: time, iterations, and per iteration the
    HBM bytes the five sweeps move at minimum (RES_BYTES_PER_EDGE per edge)
    over the mean iteration time."""
    it = info.get("it_resist")
    if not it or ctxr is None:
        return None
    ne = sum(ctxr.resistivity_sizes())
    t = ph["resist_be"]
    per_it = t / it * 1e3  # us (set-up included)
    gbs = RES_BYTES_PER_EDGE * ne / (per_it * 1e-6) / 1e9
    return {"ms": t, "iterations": it, "edges": ne, "us_per_iteration": per_it,
            "alg_bytes_per_edge_iteration": RES_BYTES_PER_EDGE, "achieved_GBs": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS}


# p = z + beta p (r, 1/diag, p_old in, p out: 32 B), face fluxes (p in, w C p
# out: 16 B), C^T + matvec (fluxes, p in, y out: 24 B), pass B (x, p, r, y,
# 1/diag in; x, r out: 56 B) -- per edge, faces counted as one per edge.
RES_BYTES_PER_EDGE = 128


def median(xs):
    xs = sorted(xs)
    n = len(xs)
    return 0.5 * (xs[(n - 1) // 2] + xs[n // 2]) if n else 0.0


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; how the path would shard "
                                   "across GPUs is described, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1610_01265_amd as sts
    from paper_1610_01265_amd import learned
    from workloads import WORKLOADS, edge_potential, flatten, he_normal, make_workload

    wl = WORKLOADS[args.workload]
    phases = args.phases.split(",")
    # host fields of the learned guess (training seeds 1..N and the evaluated
    # seed 0), generated before anything here touches the GPU
    lfields = None
    if "learned" in phases:
        progress("generating the learned guess's host fields")
        lfields = learned.host_fields(LEARNED_SHAPE, range(0, 1 + args.learned_train_seeds),
                                      args.pair_workers)
    progress("generating the workload's host fields")
    w = make_workload(wl, with_velocity=True)
    torch.cuda.set_device(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T, br, bt, bp = dev(w["T"]), dev(w["br"]), dev(w["bt"]), dev(w["bp"])
    f32 = torch.float32
    T32, br32, bt32, bp32 = T.to(f32), br.to(f32), bt.to(f32), bp.to(f32)
    v0 = dev(np.stack(w["v"]))
    nu = w["nu"]

    def shell_ctx(u_lo):
        c = sts.Context(sts.SPHERICAL, w["rf"], w["thf"], w["phf"], sts.SHELL_BC)
        c.set_dirichlet(0, value=u_lo)
        return c

    ctx, ctx32, ctxv = shell_ctx(w["T_inner"]), shell_ctx(w["T_inner"]), shell_ctx(0.0)
    u = torch.empty_like(T)
    x = torch.empty_like(T)
    v = torch.empty_like(v0)
    xv = torch.empty_like(T)
    ncell = T.numel()
    stream = torch.cuda.current_stream()

    ctxr = None
    if "resist" in phases:
        # tables are constant for a grid: set once, outside the timed steps
        ctxr = shell_ctx(0.0)
        ctxr.set_resistivity(RES_ETA)
        E0 = dev(edge_potential(wl.nr, wl.nth, wl.nph))
        Ex = torch.empty_like(E0)

    net = None
    held = None
    lprob = None
    learned_info = {}
    if "learned" in phases:
        progress("training the guess network (untimed)")
        # network trained (untimed) on seeds 1..N of its own grid; the timed
        # steps guess for seed 0 (not a training pair) and train on a held pair
        lprob = learned.Problem(LEARNED_SHAPE)
        net = sts.Cnn(lprob.ctx)
        net.set_weights(flatten(he_normal(4, 16, 0)))
        t0 = time.perf_counter()
        pairs = learned.make_pairs(lprob, lfields[1:], LEARNED_RATIO, rtol=1e-10)
        learned.fit_norm(net, pairs)
        hist = learned.train(net, pairs, args.learned_epochs, 1e-3)
        torch.cuda.synchronize()
        learned_info = {"grid": list(LEARNED_SHAPE), "dt_over_dt_euler": LEARNED_RATIO,
                        "train_pairs": len(pairs), "epochs": args.learned_epochs,
                        "loss_per_epoch": hist, "pretrain_s": time.perf_counter() - t0}
        held = pairs[0]
        del pairs
        TL = dev(lfields[0][1])
        xl = torch.empty_like(TL)
        lfields = None

    if args.copy_calib:
        src = torch.empty(4 * ncell, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(rec):
        tm = Timer(torch, stream)
        info = {}
        tm.mark("setup")
        ctx.set_spitzer(T, w["kappa0"], br, bt, bp)
        dt = wl.dt_factor * ctx.dt_euler()
        tm.mark("rkl2")
        if "rkl2" in phases:
            u.copy_(T)
            info["s"] = ctx.rkl2_step(u, dt)
        tm.mark("jacobi")
        if "jacobi" in phases:
            x.copy_(T)
            info["it_jac"], _, _ = ctx.be_pcg_solve(T, x, dt, pc=sts.PC_JACOBI, rtol=wl.rtol)
        tm.mark("ilu0")
        if "ilu0" in phases:
            x.copy_(T)
            info["it_ilu"], _, _ = ctx.be_pcg_solve(T, x, dt, pc=sts.PC_BLOCK_ILU0,
                                                    block=wl.block, rtol=wl.rtol)
        tm.mark("fp32_setup")
        if "fp32" in phases:
            ctx32.set_spitzer_f32(T32, w["kappa0"], br32, bt32, bp32)
            dt32 = wl.dt_factor * ctx32.dt_euler()
        tm.mark("fp32_rkl2")
        if "fp32" in phases:
            u.copy_(T)
            ctx32.rkl2_step(u, dt32)
        tm.mark("fp32_jacobi")
        if "fp32" in phases:
            x.copy_(T)
            info["it_jac32"], _, _ = ctx32.be_pcg_solve(T, x, dt32, pc=sts.PC_JACOBI,
                                                        rtol=wl.rtol)
        tm.mark("visc_rkl2")
        if "visc" in phases:
            ctxv.set_isotropic(nu)
            dtv = wl.dt_factor * ctxv.dt_euler()
            v.copy_(v0)
            info["s_visc"] = ctxv.rkl2_step(v, dtv)
        tm.mark("visc_jacobi")
        if "visc" in phases:
            its = []
            for m in range(3):
                xv.copy_(v0[m])
                it, _, _ = ctxv.be_pcg_solve(v0[m], xv, dtv, pc=sts.PC_JACOBI, rtol=wl.rtol)
                its.append(it)
            info["it_visc"] = its
        tm.mark("learned_setup")
        if "learned" in phases:
            dtl = LEARNED_RATIO * lprob.set_temperature(TL)
        tm.mark("learned_guess")
        if "learned" in phases:
            _, used, rel = net.guess(TL, dtl, xl)
            info["guess_used_net"], info["guess_relres"] = used, rel
        tm.mark("learned_jacobi")
        if "learned" in phases:
            info["it_learned"], _, _ = lprob.ctx.be_pcg_solve(TL, xl, dtl, pc=sts.PC_JACOBI,
                                                              rtol=wl.rtol)
        tm.mark("learned_prev_jacobi")
        if "learned" in phases:
            xl.copy_(TL)
            info["it_learned_prev"], _, _ = lprob.ctx.be_pcg_solve(TL, xl, dtl,
                                                                   pc=sts.PC_JACOBI,
                                                                   rtol=wl.rtol)
        tm.mark("learned_train")
        if "learned" in phases:
            net.train_step(held.F, held.dt, held.T, held.x_star, 1e-4, want_loss=False)
        tm.mark("var_subcycle10")
        if "variants" in phases:
            u.copy_(T)
            info["n_sub10"] = ctx.rkl_step(u, dt, nsub=10)
        tm.mark("var_euler_quarter")
        if "variants" in phases:
            u.copy_(T)
            info["n_euler"] = ctx.rkl_step(u, dt, euler_fraction=0.25)
        tm.mark("var_rkl1_extra1")
        if "variants" in phases:
            u.copy_(T)
            info["n_rkl1"] = ctx.rkl_step(u, dt, scheme=1, extra=1)
        tm.mark("nl_rkl2")
        if "nonlinear" in phases:
            u.copy_(T)
            info["s_nl"] = ctx.rkl2_step_nonlinear(u, dt, w["kappa0"], br, bt, bp)
        tm.mark("resist_be")
        if "resist" in phases:
            dtr = wl.dt_factor * ctxr.resistivity_dt_euler()
            Ex.copy_(E0)
            info["it_resist"], _, _ = ctxr.resistivity_be_pcg_solve(E0, Ex, dtr, rtol=wl.rtol)
        tm.mark("end")
        if rec is not None:
            rec.append((tm, info))

    progress(f"inputs ready; {args.warmup} warm-up steps")
    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    progress(f"{args.steps} timed steps")
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress("timed steps done")
    march = None
    if args.march_steps > 0:
        progress("successive-step march")
        march = run_march(torch, sts, ctx, T, (br, bt, bp), w["kappa0"], wl, args.march_steps,
                          stream)
    per = {}
    for tm, _ in recs:
        for k, val in tm.intervals().items():
            per.setdefault(k, []).append(val)
    ph = {k: median(vals) for k, vals in per.items()}
    ph_mean = {k: sum(vals) / len(vals) for k, vals in per.items()}
    info = recs[-1][1]
    sec = {k: val / 1e3 for k, val in ph.items()}
    s = info.get("s", 0)
    t_rk = sec["rkl2"]
    value = ncell * s / t_rk if s else 0.0
    alg_bytes = (72 + 88 * (s - 1)) * ncell if s else 0
    achieved = alg_bytes / t_rk / 1e9 if s else 0.0
    traffic = read_traffic(ncell) if s else None
    t_jac = sec["jacobi"]
    t_learn = sec["learned_guess"] + sec["learned_jacobi"]

    def ratio(a, b):
        return a / b if (a > 0 and b > 0) else None

    def pcg_hbm(iters, bpc, seconds, cells=ncell):
        """Algorithmic bytes of the iterations over the whole solve time
        (set-up included, so a lower bound on the sweeps' own rate)."""
        if not iters or seconds <= 0:
            return None
        gbs = iters * bpc * cells / seconds / 1e9
        return {"alg_bytes_per_cell_iteration": bpc, "achieved_GBs": gbs,
                "frac_hbm": gbs / HBM_PEAK_GBS}

    out = {
        "metric": "RKL2 stage cell-updates/s + BE-PCG s/solve at 1e-8 res; % HBM peak",
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: spherical shell {wl.nr}x{wl.nth}x{wl.nph} "
                               f"({ncell} cells), Spitzer conduction, tilted dipole b, "
                               f"dt = {wl.dt_factor:g} dt_Euler, rtol {wl.rtol:g}; viscosity "
                               f"on 3 velocity components; learned guess (4-layer CNN) on "
                               f"{'x'.join(map(str, LEARNED_SHAPE))}",
                   "rkl2_stages": s, "ilu_block": list(wl.block)},
        "timing": "phase times: median over the timed steps (HIP events on the library's "
                  "stream), after the warm-up steps",
        "phase_ms": ph,
        "phase_ms_mean": ph_mean,
        "be_pcg_s_per_solve": {"jacobi": t_jac, "block_ilu0_8x8x8": sec["ilu0"],
                               "fp32_form_jacobi": sec["fp32_jacobi"],
                               "viscosity_jacobi_per_component": sec["visc_jacobi"] / 3,
                               "learned_grid_jacobi_from_previous": sec["learned_prev_jacobi"],
                               "learned_grid_jacobi_from_guess_incl_guess": t_learn},
        "be_pcg_iters": {"jacobi": info.get("it_jac"), "block_ilu0_8x8x8": info.get("it_ilu"),
                         "fp32_form_jacobi_inner": info.get("it_jac32"),
                         "viscosity_jacobi": info.get("it_visc"),
                         "learned_grid_jacobi_from_previous": info.get("it_learned_prev"),
                         "learned_grid_jacobi_from_guess": info.get("it_learned")},
        "be_pcg_hbm": {"jacobi": pcg_hbm(info.get("it_jac"), 144, t_jac),
                       "block_ilu0_8x8x8": pcg_hbm(info.get("it_ilu"), 216, sec["ilu0"]),
                       "viscosity_jacobi": pcg_hbm(sum(info.get("it_visc") or []), 96,
                                                   sec["visc_jacobi"])},
        "speedup_vs_fp64_jacobi_pcg": {
            "block_ilu0_8x8x8": ratio(t_jac, sec["ilu0"]),
            "fp32_form_jacobi": ratio(t_jac, sec["fp32_jacobi"]),
            "rkl2_step": ratio(t_jac, t_rk),
            "fp32_form_rkl2_step": ratio(t_jac, sec["fp32_rkl2"]),
            "learned_guess_jacobi_on_its_grid": ratio(sec["learned_prev_jacobi"], t_learn)},
        "successive_steps": march,
        "super_step_variants": {
            "rkl2_10_subcycles": {"ms": ph.get("var_subcycle10"),
                                  "operator_applications": info.get("n_sub10")},
            "euler_quarter_then_rkl2": {"ms": ph.get("var_euler_quarter"),
                                        "operator_applications": info.get("n_euler")},
            "rkl1_one_extra_stage": {"ms": ph.get("var_rkl1_extra1"),
                                     "operator_applications": info.get("n_rkl1")}},
        "nonlinear_kappa_rkl2": nonlinear_entry(ph, info, ncell),
        "resistivity_be_pc1": resist_entry(ph, info, ctxr),
        "learned": dict(learned_info, guess_used_net=info.get("guess_used_net"),
                        guess_relres_net_prev=info.get("guess_relres"),
                        train_step_ms=ph.get("learned_train")),
        "roofline": {"kernel": "k_march (fused 19-point stencil + RKL2 stage update)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes / s if s else None,
                     "mean_launch_us": t_rk / s * 1e6 if s else None},
    }
    if not args.no_cpu_baseline:
        progress("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(w, wl.dt_factor)
    print(json.dumps(out), flush=True)
    if net is not None:
        net.close()
    for c in (ctx, ctx32, ctxv) + ((ctxr,) if ctxr is not None else ()) + (
            (lprob.ctx,) if lprob is not None else ()):
        c.close()


if __name__ == "__main__":
    main()
