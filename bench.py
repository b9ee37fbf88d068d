"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the synthetic shell input:
  coefficient setup (lagged Spitzer diffusivity, face / edge weights,
  Gershgorin dt_Euler), one RKL2 super-step at dt = f dt_Euler, one BE step
  solved by Jacobi-PCG and one by block-ILU0(8^3)-PCG, each to the workload's
  relative residual; then the FP32 precision form of the RKL2 step and of the
  Jacobi-PCG solve (mixed-precision refinement to the same FP64 residual).
Inputs are resident in HBM before the timed region.  Each phase is bracketed
by HIP events on the library's stream.  `value` is the RKL2 throughput in
cell-stage updates per second over the RKL2 phases; the BE solve times are
reported beside it.  The roofline entry is for the RKL2 stage kernel (88
algorithmic bytes per cell per stage).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="shell128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phases", default="rkl2,jacobi,ilu0,fp32",
                    help="comma list of timed phases (profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="before the steps, run a plain device copy of 4 fields (known bytes) "
                         "that calibrates the HBM byte counters")
    return ap.parse_args()


def cpu_baseline(w, dt_factor):
    """The oracle as it stands, timed on this host: one RKL2 super-step of the
    same workload (the bounded sample: one step of s stages)."""
    from oracle import operator as O
    from oracle import rkl2 as orkl2
    D = O.spitzer_tensor(w["T"], w["kappa0"], w["br"], w["bt"], w["bp"])
    op = O.assemble("spherical", w["rf"], w["thf"], w["phf"], D, O.SHELL_BC, u_lo=w["T_inner"])
    dte = O.gershgorin_dt_euler(op)
    s = orkl2.stage_count(dt_factor)
    t0 = time.perf_counter()
    orkl2.rkl2_step(lambda v: O.apply_F(op, v), w["T"], dt_factor * dte, s)
    t = time.perf_counter() - t0
    cells = w["T"].size
    return {"value": cells * s / t, "unit": "cell-stage updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one RKL2 super-step (s={s}) of {w['workload'].name} "
                      f"({cells} cells), numpy FP64, single thread, {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a "
                                   "design (DESIGN.md), not an implemented path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1610_01265_amd as sts
    from workloads import make_workload, WORKLOADS

    wl = WORKLOADS[args.workload]
    w = make_workload(wl, with_velocity=False)
    torch.cuda.set_device(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T, br, bt, bp = dev(w["T"]), dev(w["br"]), dev(w["bt"]), dev(w["bp"])
    f32 = torch.float32
    T32, br32, bt32, bp32 = T.to(f32), br.to(f32), bt.to(f32), bp.to(f32)
    ctx = sts.Context(sts.SPHERICAL, w["rf"], w["thf"], w["phf"], sts.SHELL_BC)
    ctx.set_dirichlet(0, value=w["T_inner"])
    ctx32 = sts.Context(sts.SPHERICAL, w["rf"], w["thf"], w["phf"], sts.SHELL_BC)
    ctx32.set_dirichlet(0, value=w["T_inner"])
    u = torch.empty_like(T)
    x = torch.empty_like(T)
    ncell = T.numel()
    phases = args.phases.split(",")
    stream = torch.cuda.current_stream()

    if args.copy_calib:
        src = torch.empty(4 * ncell, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(rec):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
        ev[0].record(stream)
        ctx.set_spitzer(T, w["kappa0"], br, bt, bp)
        dte = ctx.dt_euler()
        dt = wl.dt_factor * dte
        ev[1].record(stream)
        s = 0
        if "rkl2" in phases:
            u.copy_(T)
            s = ctx.rkl2_step(u, dt)
        ev[2].record(stream)
        itj = iti = 0
        if "jacobi" in phases:
            x.copy_(T)
            itj, _, _ = ctx.be_pcg_solve(T, x, dt, pc=sts.PC_JACOBI, rtol=wl.rtol)
        ev[3].record(stream)
        if "ilu0" in phases:
            x.copy_(T)
            iti, _, _ = ctx.be_pcg_solve(T, x, dt, pc=sts.PC_BLOCK_ILU0, block=wl.block,
                                         rtol=wl.rtol)
        ev[4].record(stream)
        it32 = 0
        if "fp32" in phases:
            # precision form: FP32 coefficient set-up, RKL2 step, Jacobi-PCG solve
            ctx32.set_spitzer_f32(T32, w["kappa0"], br32, bt32, bp32)
            dt32 = wl.dt_factor * ctx32.dt_euler()
            ev[5].record(stream)
            u.copy_(T)
            ctx32.rkl2_step(u, dt32)
            ev[6].record(stream)
            x.copy_(T)
            it32, _, _ = ctx32.be_pcg_solve(T, x, dt32, pc=sts.PC_JACOBI, rtol=wl.rtol)
        else:
            ev[5].record(stream)
            ev[6].record(stream)
        ev[7].record(stream)
        if rec is not None:
            rec.append((ev, s, itj, iti, it32))

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(7)] for r in recs])  # ms
    s = recs[-1][1]
    t_setup, t_rk, t_jac, t_ilu, t_set32, t_rk32, t_jac32 = ph.mean(axis=0) / 1e3
    cell_updates = ncell * s
    value = cell_updates / t_rk if t_rk > 0 else 0.0
    # algorithmic bytes of one RKL2 super-step: stage 1 reads u0 + 6 coefficient
    # arrays and writes F0, u1 (72 B/cell); stages 2..s read u_{k-1}, u_{k-2}, u0,
    # F0 + 6 coefficients and write u_k (88 B/cell)
    alg_bytes = (72 + 88 * (s - 1)) * ncell if s else 0
    achieved = alg_bytes / t_rk / 1e9 if t_rk > 0 else 0.0
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
                               f"dt = {wl.dt_factor:g} dt_Euler, rtol {wl.rtol:g}",
                   "rkl2_stages": s, "ilu_block": list(wl.block)},
        "phase_ms": {"setup": t_setup * 1e3, "rkl2_step": t_rk * 1e3,
                     "be_pcg_jacobi": t_jac * 1e3, "be_pcg_ilu0": t_ilu * 1e3,
                     "fp32_setup": t_set32 * 1e3, "fp32_rkl2_step": t_rk32 * 1e3,
                     "fp32_be_pcg_jacobi": t_jac32 * 1e3},
        "be_pcg_s_per_solve": {"jacobi": t_jac, "block_ilu0_8x8x8": t_ilu,
                               "fp32_form_jacobi": t_jac32},
        "be_pcg_iters": {"jacobi": recs[-1][2], "block_ilu0_8x8x8": recs[-1][3],
                         "fp32_form_jacobi_inner": recs[-1][4]},
        "speedup_vs_fp64_jacobi_pcg": {
            "block_ilu0_8x8x8": t_jac / t_ilu if t_ilu > 0 else None,
            "fp32_form_jacobi": t_jac / t_jac32 if t_jac32 > 0 else None,
            "rkl2_step": t_jac / t_rk if t_rk > 0 else None,
            "fp32_form_rkl2_step": t_jac / t_rk32 if t_rk32 > 0 else None},
        "roofline": {"kernel": "k_stage<OP_SPITZER> (fused 19-point stencil + RKL2 stage)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_cell_stage": 88},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, wl.dt_factor)
    print(json.dumps(out), flush=True)
    ctx.close()
    ctx32.close()


if __name__ == "__main__":
    main()
