"""Serving loop: continuous batching of flow-solve requests on one GPU.

A request is a seeded workload instance (its mesh and parameters, the
client's payload), a residual tolerance (velocity residual of Eq. 32 over the
residual lag, which is the chunk) and a step budget.  The server

  * admits queued requests in arrival order while a slot is free and the
    request's device footprint (mesh arrays + solver state) fits the HBM
    budget; a request larger than the whole budget is rejected;
  * prepares admitted requests (device mesh: topology, cell order, FP64
    geometry; solver state, Step 0) on worker threads and a side stream while
    the GPU advances the requests already running;
  * keeps running meshes and states resident and advances every running
    request together, `chunk` steps at a time, through one batched,
    graph-replayed launch sequence (their work overlaps on the device);
  * after each chunk reads every member's residual with one sync, completes
    members that converged or reached their budget, copies their fields out
    and frees their slot and bytes; prepared requests join at that boundary;
  * reports latency = completion - arrival (p50/p99) and the aggregate
    cell-updates/s.

A member's arithmetic does not depend on the other members or on the launch
schedule, so a result is the same alone and in any mix (bitwise).

Every step of the method runs in the HIP library; this module only decides
what to launch when.  The device work sits behind a small backend interface
so the admission and bookkeeping logic also runs against a host stand-in.
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import dataclasses
import json
import math
import sys
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    inst: object                 # workloads.Instance
    tol: float = 1e-6
    budget: int = 20000
    arrival: float = 0.0         # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    n_cells: int
    steps: int
    residual: float
    converged: bool
    arrival: float
    admitted: float
    completed: float
    rho: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None
    kind: str = ""

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class GpuBackend:
    """Device work through the C ABI.  Running requests share one compute
    stream (a non-blocking torch stream, so the preparing threads' copies on
    other streams do not wait for it); requests are prepared on a side stream
    and handed to the compute stream when they join."""

    def __init__(self, scheme: str = "rk4", storage: str = "fp32dev", chunk: int = 1000, autotune: bool = True,
                 schedule: Optional[dict] = None, tune_members: int = 8):
        import torch
        from . import fvlbm as F
        self.F = F
        self.torch = torch
        self.scheme, self.storage, self.chunk, self.autotune = scheme, storage, chunk, autotune
        self.schedule = schedule          # tuned once, on the first batch of tune_members or more, then reused
        self.tune_members = tune_members
        self.compute = torch.cuda.Stream()
        self.prep = torch.cuda.Stream()
        self._batch = None
        self._members = None
        self.batch_builds = 0           # batches created
        self.member_changes = 0         # membership changes applied to the running batch in place
        self.graphs_built = self.graphs_repointed = 0   # of closed batches (see graph_counts)
        # host seconds of the main thread: batch (re)builds, enqueueing chunks (the first
        # chunk of a new batch also instantiates its graphs), releasing finished requests
        self.t_build = self.t_enqueue = self.t_free = 0.0

    def timings(self) -> dict:
        return dict(build_s=round(self.t_build, 2), enqueue_s=round(self.t_enqueue, 2), free_s=round(self.t_free, 2))

    def graph_counts(self) -> dict:
        """Batch graphs instantiated, and re-pointed in place by membership changes."""
        built, rep = self.graphs_built, self.graphs_repointed
        if self._batch is not None:
            c = self._batch.graph_counts()
            built, rep = built + c["built"], rep + c["repointed"]
        return dict(batch_builds=self.batch_builds, member_changes=self.member_changes, graphs_built=built,
                    graphs_repointed=rep)

    def prepare(self, inst):
        """Device mesh and solver (Step 0) for a request, on the side stream; tile tables for
        the serving schedule are built here too.  Runs on a worker thread."""
        F, torch = self.F, self.torch
        torch.cuda.set_device(0)
        mesh = F.Mesh(inst.mesh, reorder=inst.order, stream=self.prep)
        p = F.make_params(tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme=self.scheme, storage=self.storage,
                          u_dev=inst.u0, residual_lag=self.chunk)
        s = F.Solver(mesh, p, u=np.tile(np.asarray(inst.u0, float), (inst.n_cells, 1)), stream=self.prep)
        if self.schedule is not None:
            try:
                s.set_schedule(self.schedule["block"], self.schedule["xcd_remap"], 0)
            except F.FvlbmError:
                pass                      # this mesh's tiles do not fit that size: the batch falls back
        s.set_stream(self.compute)
        return (mesh, s)

    def footprint(self, inst) -> int:
        """Device bytes a request will hold (mesh arrays + solver state), before creating it."""
        n = inst.n_cells
        nf = 4 if np.diff(inst.mesh.cell_ptr).max() == 4 else 3
        np_ = (n + 511) // 512 * 512
        copy = {"fp16dev": 18, "i16dev": 19}.get(self.storage, 36) * np_
        carry = 6 * np_ if self.storage == "fp16dev" else 0
        nbuf = 3 if self.scheme == "rk4" else 2
        mesh = np_ * (nf * 16 + 16) + n * 12 + np_ * 8
        state = nbuf * copy + carry + 9 * np_ * 4 + 4 * n * 8 + 9 * n * 8
        return int(mesh + state)

    def _batch_for(self, handles: List):
        """The running batch with these members.  A membership change keeps the batch, its
        schedule and its instantiated graphs (re-pointed in place); a new batch is made only
        when there is none, or the new members' tiles do not fit the batch's tile size."""
        F = self.F
        members = [h[1] for h in handles]
        if self._members is not None and len(self._members) == len(members) and \
                all(a is b for a, b in zip(self._members, members)):
            return self._batch
        t0 = time.perf_counter()
        if self._batch is not None:
            try:
                self._batch.set_members(members)
                self.member_changes += 1
            except F.FvlbmError:
                self._batch.close()
                self._batch = None
        if self._batch is None:
            self._batch = F.Batch(members)
            self.batch_builds += 1
            if self.schedule is not None:
                try:
                    self._batch.set_schedule(self.schedule["block"], self.schedule["xcd_remap"],
                                             self.schedule["persistent"])
                except F.FvlbmError:
                    pass                 # this mix's tiles do not fit that schedule: keep the default
        self._members = members
        if self.schedule is None and self.autotune and len(members) >= self.tune_members:
            self._batch.autotune(16)
            self.schedule = self._batch.get_schedule()
        self.t_build += time.perf_counter() - t0
        return self._batch

    def advance(self, handles: List, steps: int):
        """Enqueue `steps` steps of every running request (does not wait)."""
        b = self._batch_for(handles)
        t0 = time.perf_counter()
        b.step(steps)
        self.t_enqueue += time.perf_counter() - t0

    def residuals(self, handles: List) -> List[float]:
        """Residual of every running request (-1 while none), one sync."""
        res, _ = self._batch_for(handles).residuals()
        return list(res)

    def fields(self, handle):
        rho, u, _ = handle[1].macros()
        return rho, u

    def free(self, handle):
        """Release a request's solver and mesh.  While the running batch still holds the
        solver, the library frees it when the batch next changes members or is closed.
        A batch whose members have all finished is kept, graphs and all, for the next
        requests (it is not stepped until then)."""
        t0 = time.perf_counter()
        handle[1].close()
        handle[0].close()
        self.t_free += time.perf_counter() - t0

    def close(self):
        """Destroy the running batch (and with it the solvers of finished requests it holds)."""
        if self._batch is not None:
            counts = self._batch.graph_counts()
            self.graphs_built += counts["built"]
            self.graphs_repointed += counts["repointed"]
            self._batch.close()
        self._batch = None
        self._members = None


class Server:
    """prep_workers: threads preparing admitted requests while the GPU runs (0: prepare
    inline at admission, as the host stand-in tests do)."""

    def __init__(self, backend, hbm_budget: int, max_slots: int = 64, chunk: int = 1000, keep_fields: bool = False,
                 prep_workers: int = 0, progress=None):
        self.backend = backend
        self.hbm_budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.keep_fields = keep_fields
        self.prep_workers = int(prep_workers)
        self.progress = progress
        self.used = 0
        self.queue: collections.deque = collections.deque()
        self.preparing: Dict[int, dict] = {}
        self.active: Dict[int, dict] = {}
        self.results: List[Result] = []
        self.rejected: List[int] = []
        self.cell_updates = 0
        self.chunks = 0
        self.host_s = 0.0                # main-thread host time outside the device waits
        self._pool = cf.ThreadPoolExecutor(max_workers=self.prep_workers) if self.prep_workers > 0 else None

    # ---------------------------------------------------------------- admission
    def _admit(self, now: float):
        while self.queue and len(self.active) + len(self.preparing) < self.max_slots:
            req = self.queue[0]
            need = self.backend.footprint(req.inst)
            if need > self.hbm_budget:
                self.queue.popleft()
                self.rejected.append(req.rid)
                continue
            if self.used + need > self.hbm_budget:
                break                                   # wait for bytes to free up (FIFO)
            self.queue.popleft()
            self.used += need
            rec = dict(req=req, bytes=need, admitted=now, steps=0)
            if self._pool is None:
                rec["h"] = self.backend.prepare(req.inst)
                self.active[req.rid] = rec
            else:
                rec["fut"] = self._pool.submit(self.backend.prepare, req.inst)
                self.preparing[req.rid] = rec

    def _join_prepared(self, block: bool = False):
        """Prepared requests join the running set (at a chunk boundary)."""
        if not self.preparing:
            return
        if block:
            cf.wait([r["fut"] for r in self.preparing.values()], return_when=cf.FIRST_COMPLETED)
        for rid in sorted(self.preparing):
            rec = self.preparing[rid]
            if rec["fut"].done():
                rec["h"] = rec.pop("fut").result()
                del self.preparing[rid]
                self.active[rid] = rec

    def cancel(self, rid: int) -> bool:
        """Drop a queued or running request; frees its slot and bytes."""
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                return True
        rec = self.preparing.pop(rid, None)
        if rec is not None:
            self.backend.free(rec.pop("fut").result())
            self.used -= rec["bytes"]
            return True
        a = self.active.pop(rid, None)
        if a is None:
            return False
        self.backend.free(a["h"])
        self.used -= a["bytes"]
        return True

    # ---------------------------------------------------------------- loop
    def run(self, requests: List[Request], clock=time.perf_counter) -> List[Result]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = clock()
        try:
            while pending or self.queue or self.preparing or self.active:
                h0 = clock()
                now = h0 - t0
                while pending and pending[0].arrival <= now:
                    self.queue.append(pending.popleft())
                self._admit(now)
                self._join_prepared(block=not self.active and bool(self.preparing))
                if not self.active:
                    if pending and not self.preparing:      # idle until the next arrival
                        wait = pending[0].arrival - (clock() - t0)
                        if wait > 0:
                            time.sleep(min(wait, 0.05))
                        continue
                    if self.preparing or pending or self.queue:
                        continue
                    break
                ids = sorted(self.active)
                handles = [self.active[i]["h"] for i in ids]
                self.backend.advance(handles, self.chunk)
                h1 = clock()
                res = self.backend.residuals(handles)        # waits for the chunk
                h2 = clock()
                self.chunks += 1
                done = []
                for i, r in zip(ids, res):
                    a = self.active[i]
                    a["steps"] += self.chunk
                    self.cell_updates += a["req"].inst.n_cells * self.chunk
                    if (0 <= r < a["req"].tol) or a["steps"] >= a["req"].budget:
                        done.append((i, r))
                now = clock() - t0
                for i, r in done:
                    a = self.active.pop(i)
                    rho = u = None
                    if self.keep_fields:
                        rho, u = self.backend.fields(a["h"])
                    self.backend.free(a["h"])
                    self.used -= a["bytes"]
                    q = a["req"]
                    self.results.append(Result(q.rid, q.inst.n_cells, a["steps"], r, 0 <= r < q.tol,
                                               q.arrival, a["admitted"], now, rho, u,
                                               getattr(q.inst, "kind", "")))
                    if self.progress:
                        self.progress(self.results[-1], self)
                self.host_s += (h1 - h0) + (clock() - h2)
        finally:
            if self._pool is not None:
                self._pool.shutdown(wait=True)
            if hasattr(self.backend, "close"):
                self.backend.close()
        self.wall = clock() - t0
        return self.results


def summarize(results: List[Result], wall: float, cell_updates: int) -> dict:
    lat = np.array([r.latency for r in results]) if results else np.zeros(1)
    by_kind = collections.Counter(r.kind for r in results if r.converged)
    return dict(requests=len(results), p50_latency_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_s=round(float(np.percentile(lat, 99)), 4),
                mean_latency_s=round(float(lat.mean()), 4),
                M_cell_updates_per_s=round(cell_updates / max(wall, 1e-9) / 1e6, 1),
                converged=int(sum(r.converged for r in results)), converged_by_kind=dict(by_kind),
                wall_s=round(wall, 2))


KINDS = ("couette", "cavity", "cylinder", "two_cylinders")


def make_requests(n: int, rate: float, seed: int, lo: float, hi: float, tol: float, budget: int,
                  kinds=KINDS) -> List[Request]:
    """Poisson arrivals at `rate` per second; the kind drawn uniformly from `kinds`
    (two-cylinder meshes have their fixed size), cells log-uniform in [lo, hi]."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        cells = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        inst = W.served_instance(rng, cells, kinds=kinds)
        out.append(Request(k, inst, tol, budget, t))
    return out


def main():
    ap = argparse.ArgumentParser(description="served FVLBM workload: Poisson arrivals, continuous batching")
    ap.add_argument("--requests", type=int, default=200, help="requests per arrival rate")
    ap.add_argument("--loads", default="0.25,0.5,0.75,1.0,1.25", help="arrival rates as fractions of the capacity")
    ap.add_argument("--min-cells", type=float, default=5e3)
    ap.add_argument("--max-cells", type=float, default=5e5)
    ap.add_argument("--budget", type=int, default=20000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--chunk", type=int, default=1000, help="steps per chunk, also the residual lag K")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--calib", type=int, default=48, help="requests of the saturated run (all there at t = 0)")
    ap.add_argument("--hbm-budget-gb", type=float, default=4.0, help="artificial admission budget")
    ap.add_argument("--seed", type=int, default=2)
    # FP32 deviations: the 16-bit formats keep a rounding noise in the non-conserved moments that
    # the collision relaxes at dt/tau per step; where tau >> dt (the viscous Couette requests) it
    # holds the residual of Eq. 32 above 1e-6 (2e-4 block-scaled, 3e-3 FP16 on a 5k-cell channel)
    ap.add_argument("--storage", default="fp32dev", choices=["fp32dev", "fp16dev", "i16dev"])
    ap.add_argument("--prep-workers", type=int, default=4)
    ap.add_argument("--capacity", type=float, default=0.0,
                    help="requests/s of a previous capacity run (skips the capacity run)")
    ap.add_argument("--schedule", default="", help="'block,xcd,persistent' of a previous run (with --capacity)")
    ap.add_argument("--single", type=int, default=12,
                    help="calibration requests also run alone on the single-instance FP32 path (0: none)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    out = {"config": dict(vars(args), kinds=list(KINDS), residual_lag=args.chunk)}
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))

    def progress(r, srv):
        if len(srv.results) % 10 == 0:
            log(f"  {len(srv.results)} done, last {r.kind} {r.n_cells} cells {r.steps} steps "
                f"latency {r.latency:.2f} s, {len(srv.active)} running, {len(srv.queue)} queued")

    budget = int(args.hbm_budget_gb * 2 ** 30)
    # the load runs' requests (sizes and kinds do not depend on the rate: the arrival gaps
    # are drawn from the same generator, only scaled); their mean work sets the capacity
    probe = make_requests(args.requests, 1.0, args.seed, args.min_cells, args.max_cells, args.tol, args.budget)
    mean_work = float(np.mean([q.inst.n_cells for q in probe])) * args.budget
    out["load_requests"] = dict(mean_cells=round(mean_work / args.budget, 1),
                                kinds=dict(collections.Counter(q.inst.kind for q in probe)))
    del probe
    if args.capacity > 0:
        capacity = args.capacity
        b, x, p = (int(v) for v in args.schedule.split(","))
        schedule = dict(block=b, xcd_remap=bool(x), persistent=bool(p))
        out["capacity_req_per_s"] = capacity
    else:
        # capacity: a saturated stream (every request there at t = 0) drawn like the load runs
        backend = GpuBackend(chunk=args.chunk, storage=args.storage)
        calib = make_requests(args.calib, 1e9, args.seed + 100, args.min_cells, args.max_cells, args.tol, args.budget)
        log(f"capacity run: {len(calib)} requests")
        srv = Server(backend, budget, args.slots, args.chunk, prep_workers=args.prep_workers, progress=progress)
        srv.run(calib)
        cap_cells = srv.cell_updates / srv.wall
        # requests/s the saturated rate sustains for the load runs' mean request (its
        # cell count times the step budget; the few that converge early take less)
        capacity = cap_cells / mean_work
        schedule = backend.schedule
        out["capacity_req_per_s"] = round(capacity, 4)
        out["saturated"] = summarize(srv.results, srv.wall, srv.cell_updates)
        out["saturated"].update(**backend.graph_counts(), chunks=srv.chunks, host_s=round(srv.host_s, 2),
                                **backend.timings())
        out["saturated_M_cell_updates_per_s"] = round(cap_cells / 1e6, 1)
        if args.single > 0:
            # the plain single-instance FP32 path on the first calibration requests, one at a time
            from . import fvlbm as F
            stream = torch.cuda.current_stream()
            cells = steps_done = 0
            t = 0.0
            for q in calib[:args.single]:
                inst = q.inst
                mesh = F.Mesh(inst.mesh, reorder=inst.order)
                s = F.Solver(mesh, F.make_params(tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme="rk4", storage="fp32dev",
                                                 u_dev=inst.u0), u=np.tile(np.asarray(inst.u0, float), (inst.n_cells, 1)))
                s.step(8)
                s.prepare(args.chunk)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.step(args.chunk)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
                cells += inst.n_cells * args.chunk
                s.close(); mesh.close()
            out["single_fp32dev_M_cell_updates_per_s"] = round(cells / t / 1e6, 1)
            out["single_sample"] = f"the first {min(args.single, len(calib))} calibration requests, {args.chunk} steps each"
    out["schedule"] = schedule
    for load in [float(x) for x in args.loads.split(",")]:
        reqs = make_requests(args.requests, load * capacity, args.seed, args.min_cells, args.max_cells,
                             args.tol, args.budget)
        log(f"load {load}: {len(reqs)} requests at {load * capacity:.3f}/s")
        be = GpuBackend(chunk=args.chunk, storage=args.storage, schedule=schedule)
        srv = Server(be, budget, args.slots, args.chunk, prep_workers=args.prep_workers, progress=progress)
        res = srv.run(reqs)
        s = summarize(res, srv.wall, srv.cell_updates)
        s.update(rate_req_per_s=round(load * capacity, 4), rejected=len(srv.rejected), chunks=srv.chunks,
                 **be.graph_counts(), host_s=round(srv.host_s, 2), **be.timings())
        out[f"load_{load}"] = s
        log(json.dumps(s))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
