"""Writes shell128_march.json: the oracle's lagged-diffusivity march of the
128 x 128 x 256 shell (10 successive steps per method), for the GPU test of
the same march (tests/test_gpu_shell128_march.py).

Protocol (Sec. 1 lagged diffusivity, Sec. 2 backward Euler + PCG, Sec. 3
RKL2): starting from the seed-0 temperature, each method marches its own
state; at the start of every step the diffusivity is frozen from that state,
dt stays at 200 x the first step's dt_Euler (Appendix B), RKL2 takes the
minimal stable stage count of Eq. rkl2_s for the step's own dt_Euler, and BE
solves to a relative residual of 1e-8 with point-Jacobi (PC1) or block
ILU0 on 8^3 blocks (PC2, Appendix A), starting from the step's initial state.

Stored per method and step: the stage count or PCG iteration count, dt_E of
the step, the state at fixed sampled cells, and the sum, 2-norm, min and max
of the whole state.  Only the oracle and the seeded input generators run
here; the run takes about half an hour on one CPU core.

    python tests/golden/make_shell128_march.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import operator as O  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from oracle import rkl2 as orkl2  # noqa: E402
from workloads import make_workload  # noqa: E402

NSTEPS = 10
OUT = os.path.join(HERE, "shell128_march.json")


def sample_cells(shape, n_random=48, seed=11):
    """Fixed cells: seeded interior picks plus every boundary face and corner."""
    n0, n1, n2 = shape
    rng = np.random.default_rng(seed)
    cells = {tuple(int(v) for v in (rng.integers(n0), rng.integers(n1), rng.integers(n2)))
             for _ in range(n_random)}
    for i in (0, 1, n0 // 2, n0 - 2, n0 - 1):
        for j in (0, n1 // 3, n1 - 1):
            for k in (0, n2 // 2, n2 - 1):
                cells.add((i, j, k))
    return sorted(cells)


def main():
    w = make_workload("shell128", with_velocity=False)
    wl = w["workload"]
    cells = sample_cells(w["T"].shape)
    idx = tuple(np.array(c) for c in zip(*cells))

    def op_at(u):
        D = O.spitzer_tensor(u, w["kappa0"], w["br"], w["bt"], w["bp"])
        return O.assemble("spherical", w["rf"], w["thf"], w["phf"], D, O.SHELL_BC,
                          u_lo=w["T_inner"])

    dt = wl.dt_factor * O.gershgorin_dt_euler(op_at(w["T"]))
    out = {"workload": wl.name, "shape": list(w["T"].shape), "dt_factor": wl.dt_factor,
           "dt": dt, "rtol": wl.rtol, "block": [8, 8, 8], "steps": NSTEPS,
           "cells": [list(c) for c in cells], "methods": {}}
    for name in ("rkl2", "jacobi", "ilu0"):
        u = w["T"].copy()
        rec = []
        for n in range(NSTEPS):
            t0 = time.perf_counter()
            op = op_at(u)
            dte = O.gershgorin_dt_euler(op)
            if name == "rkl2":
                s = orkl2.stage_count(dt / dte)
                u = orkl2.rkl2_step(lambda v: O.apply_F(op, v), u, dt, s)
                work = s
            else:
                r = opcg.be_pcg(op, u, dt, name, rtol=wl.rtol, block=(8, 8, 8))
                assert r.converged, (name, n)
                u, work = r.x, r.iters
            rec.append({"dt_euler": dte, "work": int(work), "values": u[idx].tolist(),
                        "sum": float(u.sum()), "norm2": float(np.sqrt(np.sum(u * u))),
                        "min": float(u.min()), "max": float(u.max())})
            print(f"{name} step {n}: work {work}, {time.perf_counter() - t0:.1f} s", flush=True)
        out["methods"][name] = rec
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
