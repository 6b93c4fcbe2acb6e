"""Throughput benchmark of the FVLBM time step on one MI355X.

Headline workload (the largest single-GPU FP32 configuration): flow past a
circular cylinder, Re = 100, u_inf = 0.1, body-fitted O-grid of 256 radial x
384 circumferential quadrilaterals (98,304 cells, first cell 0.005 D, far
field at 30 D), four-stage RK, dt from CFL 0.5, FP32 storage of the
deviations from the free-stream equilibrium.  One step = one full RK step
(four RHS evaluations) over all cells; the metric is M cell-updates/s.

Prints one JSON line.  Besides the contract fields:
  roofline      the RK stage kernel against the HBM peak: algorithmic bytes per
                launch (see the design notes) / average launch duration, timed
                with HIP events on the solver's stream over the timed region
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload, on
                one host thread and on all the job's host threads (its OpenMP
                build, bitwise the same results), with the host CPU's model
  cavity20k     the lid-driven cavity, Re 1000, 20,000 jittered triangles
                (100 x 100 tanh grid, growth 1.08, seed 0), four-stage RK:
                the paper's cavity class, small enough to sit in the on-chip
                caches (a latency-bound launch)
  streaming     the same kernel on 8.4M triangles (larger than the on-chip
                caches): the honest HBM fraction, Euler and four-stage RK
  batched       64 seeded instances (2k-200k cells) advanced together by the
                batched, graph-replayed, autotuned path with FP16-deviation
                storage, each instance's error against its stored FP64 oracle
                run, next to the same instances run one at a time (FP16 and
                FP32 deviations) and batched with FP32 deviations
  precision     each storage mode's velocity error against stored FP64 oracle runs
  served        Poisson-arrival serving at a reduced size (the serving module
                runs the full sweep): p50/p99 latency and aggregate throughput
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
# Algorithmic bytes per cell-update: the state a step must read and write plus
# one read of a compact mesh description per RHS evaluation (60 B per
# triangle, 72 B per quadrilateral).
MESH_BYTES = {3: 60, 4: 72}
STATE_VALUES = {"euler": 18, "rk4": 99}   # stored values moved per cell-update
# bytes per stored value: the 16-bit block-scaled format adds one exponent byte per nine values
STORE_BYTES = {"fp32": 4.0, "fp32dev": 4.0, "fp16dev": 2.0, "i16dev": 19.0 / 9.0}
# FP16 deviations also carry each cell's mass and momentum rounding residual
# (three FP16 values), read and rewritten once per step by its last stage
CARRY_BYTES = {"fp16dev": 12.0}


def alg_bytes_per_update(nf: int, scheme: str, storage: str) -> float:
    n_rhs = 4 if scheme == "rk4" else 1
    return state_bytes_per_update(scheme, storage) + n_rhs * MESH_BYTES[nf]


def state_bytes_per_update(scheme: str, storage: str) -> float:
    """The state part of the algorithmic bytes alone (18 s or 99 s B per cell-update)."""
    return STATE_VALUES[scheme] * STORE_BYTES[storage] + CARRY_BYTES.get(storage, 0.0)


def measured_traffic(workload, schedule, leg=None):
    """HBM bytes per launch of the stage kernel from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain copy of
    known size), or None when the kernel sources changed since they were taken
    or the timed schedule is not one they were taken with.  leg: the scheme and
    storage, where one workload's record covers several."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_tile_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    key = "%d,%d,%d" % (schedule["block"], int(schedule["xcd_remap"]), int(schedule["persistent"]))
    if leg:
        key = leg + ":" + key
    ent = rec["per_schedule"].get(key)
    return ent["bytes_per_launch"] if ent else None


def events_time(stream, fn):
    import torch
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inst, label, scheme="rk4", target_s=10.0):
    """The FP64 oracle on the host: one thread, then its OpenMP build on every
    thread this job has (OMP_NUM_THREADS, else the visible cores)."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    out = {}
    for key, th in (("one", 1), ("all", threads)):
        o = O.Oracle(inst.mesh, tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme=scheme, threads=th)
        o.init(u0=inst.u0)
        t0 = time.perf_counter(); o.step(1); t1 = time.perf_counter()
        n = max(2, int(target_s / max(t1 - t0, 1e-4)))
        t0 = time.perf_counter(); o.step(n); t1 = time.perf_counter()
        out[key] = (inst.n_cells * n / (t1 - t0) / 1e6, n, o.threads)
        del o
    v_all, n_all, th_all = out["all"]
    v_one, n_one, _ = out["one"]
    return dict(value=round(v_all, 4), unit="M cell-updates/s", cores=th_all, kind="oracle",
                single_thread_value=round(v_one, 4), cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                sample=f"{label}: {n_all} four-stage RK steps on {th_all} threads (OpenMP build over cells) "
                       f"and {n_one} on one thread, FP64, {inst.n_cells} cells")


def make_solver(F, inst, scheme, storage, reorder=None):
    mesh = F.Mesh(inst.mesh, reorder=inst.order if reorder is None else reorder)
    s = F.Solver(mesh, F.make_params(tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme=scheme,
                                     storage=storage, u_dev=inst.u0),
                 u=np.tile(np.asarray(inst.u0, float), (inst.n_cells, 1)))
    return mesh, s


STREAMING_LEGS = (("euler", "fp32dev", 20), ("rk4", "fp32dev", 5), ("euler", "fp16dev", 20), ("rk4", "fp16dev", 5),
                  ("rk4", "i16dev", 5))


def streaming(F, W, stream, schedule=None, legs=None):
    out = {}
    m = W.streaming()
    mesh = F.Mesh(m, reorder=F.REORDER_BISECT)
    nf = mesh.info()["nf"]
    for scheme, storage, k in STREAMING_LEGS:
        leg = f"{scheme}_{storage}"
        if legs and leg not in legs:
            continue
        s = F.Solver(mesh, F.make_params(tau=3e-5, scheme=scheme, storage=storage))
        if schedule:
            s.set_schedule(*schedule)
            s.step(2)
        else:
            s.autotune(k)
        s.step(k)                                      # warm (graphs built, caches in steady state)
        el = sorted(events_time(stream, lambda: s.step(k)) for _ in range(3))[1]   # median of three runs
        n_launch = k * (4 if scheme == "rk4" else 1)
        t_launch = el / n_launch
        alg = alg_bytes_per_update(nf, scheme, storage) / (4 if scheme == "rk4" else 1) * m.n_cells
        state = state_bytes_per_update(scheme, storage) / (4 if scheme == "rk4" else 1) * m.n_cells
        sched = s.get_schedule()
        out[leg] = dict(cells=m.n_cells, steps=k, M_cell_updates_per_s=round(m.n_cells * k / el / 1e6, 1),
                        M_rhs_evals_per_s=round(m.n_cells * k * (4 if scheme == "rk4" else 1) / el / 1e6, 1),
                        state_only_frac=round(state / t_launch / 1e9 / HBM_PEAK_GBS, 4),
                        launch_ms=round(t_launch * 1e3, 4), achieved_GBs=round(alg / t_launch / 1e9, 1),
                        frac=round(alg / t_launch / 1e9 / HBM_PEAK_GBS, 4), alg_bytes_per_launch=alg,
                        traffic=measured_traffic("streaming8m", sched, leg), schedule=sched)
        s.close()
    mesh.close()
    return out


def precision(F):
    """Max |u - u_oracle| / U of each storage mode against the stored FP64 oracle runs
    (written by tests/golden/make_oracle_refs.py from the oracle alone)."""
    from paper_1812_00390_amd import meshgen as mg
    gold = os.path.join(ROOT, "tests", "golden")
    out = {}
    runs = [("cavity 20k tri, RK4, 2000 steps", "oracle_cavity100_rk4_2000.npz",
             lambda: mg.cavity(n=100, ratio=1.08, jitter=0.2, seed=0, lid_u=0.1), {}, None),
            ("cylinder 98k quads, RK4, 100 steps", "oracle_cylinder256_rk4_100.npz",
             lambda: mg.cylinder(nr=256, nt=384), dict(u_ref=0.2, u_dev=(0.1, 0.0)), (0.1, 0.0)),
            ("cylinder 98k quads, RK4, 20000 steps", "oracle_cylinder256_rk4_20000.npz",
             lambda: mg.cylinder(nr=256, nt=384), dict(u_ref=0.2, u_dev=(0.1, 0.0)), (0.1, 0.0))]
    for label, fname, make, extra, u0 in runs:
        path = os.path.join(gold, fname)
        if not os.path.exists(path):
            continue
        ref = np.load(path)
        m = make()
        mesh = F.Mesh(m)
        errs = {}
        for storage in ("fp32", "fp32dev", "fp16dev", "i16dev"):
            kw = dict(u=np.tile(np.asarray(u0, float), (m.n_cells, 1))) if u0 else {}
            s = F.Solver(mesh, F.make_params(tau=float(ref["tau"]), dt=float(ref["dt"]), scheme="rk4",
                                             storage=storage, **extra), **kw)
            s.step(int(ref["steps"]))
            _, u, _ = s.macros()
            errs[storage] = float(f"{np.abs(u[ref['idx']] - ref['u']).max() / 0.1:.3g}")
            s.close()
        mesh.close()
        out[label] = errs
    return {"metric": "max |u - u_oracle| / U at sampled cells", "runs": out}


def served(F, W):
    """The served workload at a reduced size: the 64 batched instances (2k-200k
    cells, cavities and cylinders) as requests of 1000 four-stage RK steps
    each, FP32-deviation storage, advanced in chunks of 250 steps by the
    continuous-batching server (preparation on worker threads); first all at
    once (saturated), then as a Poisson stream at 0.75 x that capacity.  Every
    result's error against its stored FP64 oracle run.  The full served sweep
    (5k-500k cells, 200 requests x 5 rates, residual 1e-6 or 20,000 steps) is
    run by the serving module itself."""
    from paper_1812_00390_amd.serve import GpuBackend, Request, Server, summarize
    insts = W.batched()
    gold = os.path.join(ROOT, "tests", "golden", "oracle_batched64_rk4_1000.npz")
    ref = np.load(gold) if os.path.exists(gold) else None
    steps, chunk, budget = 1000, 250, 2 ** 31
    out = {"config": dict(requests=len(insts), cells=sum(i.n_cells for i in insts), steps_per_request=steps,
                          chunk=chunk, storage="fp32dev", scheme="rk4", slots=64, prep_workers=4, loads=[0.75],
                          hbm_budget_gb=2.0, seed=2)}

    def errors(res):
        if ref is None:
            return None
        e = [float(np.abs(r.u[ref[f"idx_{r.rid}"]] - ref[f"u_{r.rid}"]).max() / 0.1) for r in sorted(res, key=lambda r: r.rid)]
        return dict(max=float(f"{max(e):.3g}"), per_request=[float(f"{x:.3g}") for x in e])

    schedule = None
    rng = np.random.default_rng(2)
    for label, rate in (("saturated", None), ("load_0.75", 0.75)):
        if rate is None:
            arrivals = np.zeros(len(insts))
        else:
            arrivals = np.cumsum(rng.exponential(1.0 / (rate * out["capacity_req_per_s"]), len(insts)))
        reqs = [Request(k, inst, tol=0.0, budget=steps, arrival=float(a)) for k, (inst, a) in enumerate(zip(insts, arrivals))]
        be = GpuBackend(chunk=chunk, storage="fp32dev", schedule=schedule)
        srv = Server(be, int(2 * 2 ** 30), 64, chunk, keep_fields=ref is not None, prep_workers=4)
        res = srv.run(reqs)
        schedule = be.schedule
        rec = summarize(res, srv.wall, srv.cell_updates)
        rec.update(**be.graph_counts(), chunks=srv.chunks, host_s=round(srv.host_s, 2), oracle_error=errors(res))
        if rate is None:
            out["capacity_req_per_s"] = round(len(res) / srv.wall, 3)
        else:
            rec["rate_req_per_s"] = round(rate * out["capacity_req_per_s"], 3)
        out[label] = rec
    out["schedule"] = schedule
    return out


def batched(F, W, stream, steps=1000, single_steps=100):
    """The batched workload: 64 instances in shared, graph-replayed launches,
    FP16-deviation storage, autotuned; each instance's error against its stored
    FP64 oracle run after the same 1000 steps; then the batching gain at equal
    storage (batched FP32 deviations, and FP16 and FP32 deviations one
    instance at a time on the plain single-instance path)."""
    insts = W.batched()
    total = sum(i.n_cells for i in insts)
    gold = os.path.join(ROOT, "tests", "golden", "oracle_batched64_rk4_1000.npz")
    ref = np.load(gold) if os.path.exists(gold) and steps == 1000 else None
    rec = dict(instances=len(insts), cells=total, steps=steps, storage="fp16dev", scheme="rk4")
    for storage in ("fp16dev", "fp32dev"):
        pairs = [make_solver(F, i, "rk4", storage) for i in insts]
        b = F.Batch([s for _, s in pairs])
        tune_ms = b.autotune(32)
        el = events_time(stream, lambda: b.step(steps))
        if storage == "fp16dev":
            rec.update(M_cell_updates_per_s=round(total * steps / el / 1e6, 1), ms_per_step=round(el * 1e3 / steps, 4),
                       tuned_ms_per_step=round(tune_ms, 4), schedule=b.get_schedule())
            if ref is not None:
                errs = []
                for k, (_, s) in enumerate(pairs):
                    _, u, _ = s.macros()
                    errs.append(float(np.abs(u[ref[f"idx_{k}"]] - ref[f"u_{k}"]).max() / 0.1))
                rec["oracle_error"] = dict(metric="max |u - u_oracle| / U at 200 sampled cells, per instance",
                                           max=float(f"{max(errs):.3g}"),
                                           per_instance=[float(f"{e:.3g}") for e in errs])
        else:
            rec["batched_fp32dev_M_cell_updates_per_s"] = round(total * steps / el / 1e6, 1)
        b.close()
        for mesh, s in pairs:
            s.close(); mesh.close()
    # the plain single-instance path on the same instances, one after another
    for storage in ("fp16dev", "fp32dev"):
        t = 0.0
        for inst in insts:
            mesh, s = make_solver(F, inst, "rk4", storage)
            s.step(8)
            s.prepare(single_steps)
            t += events_time(stream, lambda: s.step(single_steps))
            s.close(); mesh.close()
        rec[f"single_{storage}_M_cell_updates_per_s"] = round(total * single_steps / t / 1e6, 1)
    rec["speedup_vs_single_fp32dev"] = round(rec["M_cell_updates_per_s"] / rec["single_fp32dev_M_cell_updates_per_s"], 2)
    rec["batching_gain_fp16dev"] = round(rec["M_cell_updates_per_s"] / rec["single_fp16dev_M_cell_updates_per_s"], 2)
    rec["batching_gain_fp32dev"] = round(rec["batched_fp32dev_M_cell_updates_per_s"] /
                                         rec["single_fp32dev_M_cell_updates_per_s"], 2)
    return rec


ORDERS = {"bisect": 3, "hilbert": 2}
ORDER_NAMES = {v: k for k, v in ORDERS.items()}


def single_workload(F, stream, inst, label, traffic_key, args, schedule, order=None):
    """One solver stepped `args.steps` four-stage RK steps (graphs instantiated
    beforehand), timed with HIP events on its stream.  order: the mesh's cell
    order (tiles are runs of consecutive cells; default: the instance's)."""
    order = order or ORDER_NAMES[inst.order]
    mesh, s = make_solver(F, inst, "rk4", args.storage, reorder=ORDERS[order])
    nf = mesh.info()["nf"]
    if schedule:
        s.set_schedule(*schedule)
    elif not args.no_autotune:
        s.autotune(64)
    s.step(args.warmup)
    s.prepare(args.steps)
    el = events_time(stream, lambda: s.step(args.steps))
    n = inst.n_cells
    t_launch = el / (4 * args.steps)
    alg_launch = alg_bytes_per_update(nf, "rk4", args.storage) / 4 * n
    rho, u, st = s.macros()
    sched = s.get_schedule()
    state_launch = state_bytes_per_update("rk4", args.storage) / 4 * n
    out = dict(value=round(n * args.steps / el / 1e6, 3), ms_per_step=round(el * 1e3 / args.steps, 5),
               M_rhs_evals_per_s=round(4 * n * args.steps / el / 1e6, 3),
               config={"workload": label, "cells": n, "scheme": "rk4", "storage": args.storage, "dt": s.dt,
                       "cell_order": order, "schedule": sched},
               roofline={"bound": "hbm", "achieved": round(alg_launch / t_launch / 1e9, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg_launch / t_launch / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic(traffic_key, sched, order) if args.storage == "fp32dev" else None,
                         "kernel": f"k_tile<{nf},...> (one RK stage)",
                         "alg_bytes_per_launch": alg_launch, "launch_us": round(t_launch * 1e6, 3),
                         "state_only_frac": round(state_launch / t_launch / 1e9 / HBM_PEAK_GBS, 4)},
               check={"max_u": float(np.abs(u).max()), "mass": st["mass"]})
    s.close(); mesh.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="fp32dev")
    ap.add_argument("--only", choices=["all", "headline", "cavity20k", "streaming", "batched", "precision", "served",
                                       "copy"], default="all")
    ap.add_argument("--schedule", default="", help="force a launch schedule 'block,xcd,persistent' instead of tuning")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--legs", default="", help="streaming legs to run, e.g. 'rk4_fp32dev' (default: all)")
    ap.add_argument("--reorder", choices=sorted(ORDERS), default=None,
                    help="cell order of the headline mesh (default: the workload's, Hilbert for the cylinder O-grid)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no multi-GPU path; "
              "the design notes describe how the step would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1812_00390_amd import fvlbm as F
    from paper_1812_00390_amd import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    schedule = None
    if args.schedule:
        b, x, p = (int(v) for v in args.schedule.split(","))
        schedule = (b, bool(x), int(p))
    rec = {}
    if args.only in ("all", "headline"):
        inst = W.cylinder98k()
        label = ("flow past a circular cylinder Re=100 u_inf=0.1, O-grid 256x384 quads (98304 cells, "
                 "first cell 0.005 D, far field 30 D), four-stage RK, CFL 0.5, deviations from the free stream")
        h = single_workload(F, stream, inst, label, "cylinder98k", args, schedule, args.reorder)
        rec.update({
            "metric": "M cell-updates/s (D2Q9, FP32)",
            "value": h["value"],
            "unit": "M cell-updates/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": h["ms_per_step"],
            "M_rhs_evals_per_s": h["M_rhs_evals_per_s"],
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32" if args.storage in ("fp32", "fp32dev") else f"f32 compute, {args.storage} storage",
            "data": "synthetic",
            "config": h["config"],
            "roofline": h["roofline"],
            "check": h["check"],
        })
        if not args.no_cpu_baseline:
            rec["cpu_baseline"] = cpu_baseline(inst, "the same 98,304-quad cylinder")
    if args.only in ("all", "cavity20k"):
        label = ("lid-driven cavity Re=1000 U=0.1, 20000 jittered triangles (100x100 tanh growth 1.08, seed 0), "
                 "four-stage RK, CFL 0.5")
        c = single_workload(F, stream, W.cavity20k(), label, "cavity20k", args, schedule)
        c["M_cell_updates_per_s"] = c.pop("value")
        rec["cavity20k"] = c
    if args.only == "copy":
        # calibration of the HBM byte counters: a plain device copy of a known size
        n = 1 << 28                       # 1 GiB of FP32 each way
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        el = events_time(stream, lambda: [dst.copy_(src) for _ in range(5)])
        rec["copy"] = dict(bytes_each_way=4 * n, launches=5, GBs=round(2 * 4 * n * 5 / el / 1e9, 1))
    if args.only in ("all", "streaming"):
        rec["streaming"] = streaming(F, W, stream, schedule, [x for x in args.legs.split(",") if x])
    if args.only in ("all", "batched"):
        rec["batched"] = batched(F, W, stream)
    if args.only in ("all", "precision"):
        rec["precision"] = precision(F)
    if args.only in ("all", "served"):
        rec["served"] = served(F, W)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
