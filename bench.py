"""Throughput benchmark of the FVLBM time step on one MI355X.

Headline workload: lid-driven cavity, Re = 1000, U = 0.1, 20,000 jittered
triangles from a 100 x 100 tanh-clustered grid (growth 1.08, seed 0),
four-stage RK, FP32 storage, dt from CFL 0.5.  One step = one full RK step
(four RHS evaluations) over all cells; the metric is M cell-updates/s.

Prints one JSON line.  Extra objects:
  roofline      the RK stage kernel against the HBM peak (algorithmic bytes per
                launch / average launch duration, HIP events on the solver's stream)
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload
  streaming     the same kernel on an 8.4M-triangle mesh that does not fit the
                on-chip caches (honest HBM fraction), Euler and RK4
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
# algorithmic bytes per cell (see the design notes): state read/write + compact mesh
MESH_BYTES = {3: 60, 4: 72}           # per RHS evaluation
STATE_BYTES = {"euler": 18, "rk4": 99}  # x bytes per stored value, per cell-update


def alg_bytes_per_update(nf: int, scheme: str, sbytes: int) -> float:
    n_rhs = 4 if scheme == "rk4" else 1
    return STATE_BYTES[scheme] * sbytes + n_rhs * MESH_BYTES[nf]


def timed_run(F, solver, steps: int, warmup: int, stream):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    solver.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3


def cpu_baseline(mesh_raw, tau, scheme, target_s=12.0):
    from oracle import oracle as O
    o = O.Oracle(mesh_raw, tau=tau, cfl=0.5, u_ref=0.1, scheme=scheme)
    o.init()
    t0 = time.perf_counter(); o.step(1); t1 = time.perf_counter()
    per = max(t1 - t0, 1e-4)
    n = max(2, int(target_s / per))
    t0 = time.perf_counter(); o.step(n); t1 = time.perf_counter()
    return dict(value=mesh_raw.n_cells * n / (t1 - t0) / 1e6, unit="M cell-updates/s", cores=1,
                kind="oracle", sample=f"{n} {scheme} steps of the same {mesh_raw.n_cells}-cell mesh (FP64, 1 thread)")


def streaming(F, mg, stream, schemes=("euler", "rk4"), n=2048, steps=None):
    out = {}
    m = mg.streaming_cavity(n=n)
    mesh = F.Mesh(m, reorder=F.REORDER_RCM)
    nf = mesh.info()["nf"]
    for scheme in schemes:
        k = steps or (20 if scheme == "euler" else 5)
        s = F.Solver(mesh, F.make_params(tau=3e-5, scheme=scheme, storage="fp32dev"))
        el = timed_run(F, s, k, 2, stream)
        n_launch = k * (4 if scheme == "rk4" else 1)
        t_launch = el / n_launch
        alg = alg_bytes_per_update(nf, scheme, 4) / (4 if scheme == "rk4" else 1) * m.n_cells
        out[scheme] = dict(cells=m.n_cells, steps=k, M_cell_updates_per_s=m.n_cells * k / el / 1e6,
                           launch_ms=t_launch * 1e3, achieved_GBs=alg / t_launch / 1e9,
                           frac=alg / t_launch / 1e9 / HBM_PEAK_GBS)
        s.close()
    mesh.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="fp32dev")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-streaming", action="store_true")
    ap.add_argument("--block", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this library has no multi-GPU path; "
              "see the design notes for how the step would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1812_00390_amd import fvlbm as F
    from paper_1812_00390_amd import meshgen as mg

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    U, Re = 0.1, 1000.0
    tau = 3 * U * 1.0 / Re
    m = mg.cavity(n=100, ratio=1.08, jitter=0.2, seed=0, lid_u=U)
    mesh = F.Mesh(m, reorder=F.REORDER_RCM)
    nf = mesh.info()["nf"]
    s = F.Solver(mesh, F.make_params(tau=tau, cfl=0.5, u_ref=U, scheme="rk4", storage=args.storage))
    if args.block:
        s.set_schedule(args.block, True)
    el = timed_run(F, s, args.steps, args.warmup, stream)
    n = m.n_cells
    value = n * args.steps / el / 1e6
    sbytes = 2 if args.storage == "fp16dev" else 4
    t_launch = el / (4 * args.steps)
    alg_launch = alg_bytes_per_update(nf, "rk4", sbytes) / 4 * n
    rho, u, st = s.macros()
    rec = {
        "metric": "M cell-updates/s (D2Q9, FP32)",
        "value": round(value, 3),
        "unit": "M cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage != "fp16dev" else "f32 (fp16 storage)",
        "data": "synthetic",
        "config": {"workload": "lid-driven cavity Re=1000, 20000 jittered triangles (100x100 tanh 1.08, seed 0), "
                               "RK4, CFL 0.5", "cells": n, "scheme": "rk4", "storage": args.storage,
                   "dt": s.dt, "schedule": list(s.get_schedule())},
        "roofline": {"bound": "hbm", "achieved": round(alg_launch / t_launch / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg_launch / t_launch / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_stage<3,FP32> (one RK stage)",
                     "alg_bytes_per_launch": alg_launch, "launch_us": t_launch * 1e6},
        "check": {"max_u": float(np.abs(u).max()), "mass": st["mass"]},
    }
    if not args.no_streaming:
        rec["streaming"] = streaming(F, mg, stream)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(m, tau, "rk4")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
