"""Serving form: continuous batching of RVE toughness requests on one GPU.

Requests (one RVE each: grid, microstructure, contrasts) arrive over time.
The server keeps pools of batched handles, one pool per compatible problem
class (grid, voxel size, l, k, load direction, precision, split), each with
its own HIP stream and its fields resident in HBM.  Every scheduler tick:

  1. admission: waiting requests, oldest first, take a free slot of a pool
     of their class, or open a new pool if its workspace
     (rve_query_workspace for its slot count) fits the HBM budget beside
     the pools already open; otherwise they wait (an admission stall);
  2. all pools with occupied slots advance them in one rve_run_budget call
     each, concurrently on their streams: the pool's slots take
     dissipation-controlled steps (Eq. 16) at their own pace until they
     have committed steps_per_tick steps per occupied slot together (a fast
     request takes more steps than a slow one), and a step still in flight
     at the end of the call stays on the device for the next tick
     (RVE_RUN_KEEP); a step that fails is halved inside the library, and a
     step that still fails leaves the slot's state as it was and ends the
     request;
  3. a slot whose RVE has reached the fracture point yields G_eff
     (Eq. 32-33), records its latency and is released for the next request;
     pools left empty are closed when memory is needed.

All solver work runs in libmirve; this module only schedules.
"""
import concurrent.futures as cf
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import mirve


@dataclasses.dataclass
class Request:
    rid: int
    workload: object                  # workloads.Workload
    arrival: float = 0.0              # seconds after the start of the stream
    max_steps: int = 400


@dataclasses.dataclass
class Result:
    rid: int
    G_eff: Optional[float]
    steps: int
    status: int                       # 0, or the RVE_E* code that stopped it
    arrival: float
    admitted: float
    finished: float
    n_greenop: int = 0

    @property
    def latency(self):
        return self.finished - self.arrival


def problem_class(w, precision, split):
    return (tuple(w.n), float(w.h), float(w.ell), float(w.k),
            tuple(np.round(np.asarray(w.f, dtype=float), 15)), int(precision), int(split))


class Pool:
    """One batched handle (B slots of one problem class) on its own stream."""

    def __init__(self, key, w0, slots, precision, split, tol):
        import torch
        self.key = key
        self.stream = torch.cuda.Stream()
        cfg = mirve.make_config(w0.n, h=w0.h, ell=w0.ell, k=w0.k, f=w0.f, precision=precision,
                                batch=slots, split=split, **tol)
        cfg.max_materials = 4096
        self.rve = mirve.Rve(cfg, stream=self.stream)
        self.B = slots
        self.nbytes = self.rve.nbytes
        self.req: List[Optional[Request]] = [None] * slots
        self.admitted = [0.0] * slots
        self.steps = [0] * slots
        self.greens = [0] * slots

    def free_slot(self):
        for i, r in enumerate(self.req):
            if r is None:
                return i
        return None

    def occupied(self):
        return sum(r is not None for r in self.req)

    def admit(self, req, now):
        i = self.free_slot()
        self.rve.set_workload(req.workload, slot=i)
        self.req[i] = req
        self.admitted[i] = now
        self.steps[i] = 0
        self.greens[i] = 0
        return i

    def step(self, steps_per_tick):
        dt = [float(r.workload.dtau) if r is not None else 0.0 for r in self.req]
        caps = [r.max_steps - s if r is not None else 0 for r, s in zip(self.req, self.steps)]
        return self.rve.rve_run_budget(dt, steps_per_tick * self.occupied(), stop_at_fracture=True,
                                       keep=True, max_steps=caps)

    def close(self):
        self.rve.close()


class Server:
    """Continuous-batching request loop.

    budget_bytes bounds the sum of the pools' workspaces (default: 80 % of
    the free device memory at start).  slots_per_pool is the slot count of
    a new pool (fewer if the budget only fits fewer).
    """

    def __init__(self, precision=mirve.RVE_PREC_MIXED, split=mirve.RVE_SPLIT_NONE,
                 budget_bytes=None, slots_per_pool=16, tol=None, clock=time.perf_counter,
                 steps_per_tick=1):
        import torch
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.precision = precision
        self.split = split
        self.budget = int(budget_bytes)
        self.slots_per_pool = int(slots_per_pool)
        self.steps_per_tick = max(1, int(steps_per_tick))
        self.tol = dict(tol or {})
        self.pools: Dict[tuple, List[Pool]] = {}
        self.waiting: List[Request] = []
        self.results: Dict[int, Result] = {}
        self.clock = clock
        self.t0 = clock()
        self.stalls = 0
        self.peak_bytes = 0
        self.ticks = 0
        self._ex = cf.ThreadPoolExecutor(max_workers=32)

    # -- bookkeeping ---------------------------------------------------------
    def now(self):
        return self.clock() - self.t0

    def used_bytes(self):
        return sum(p.nbytes for ps in self.pools.values() for p in ps)

    def all_pools(self):
        return [p for ps in self.pools.values() for p in ps]

    def submit(self, req):
        self.waiting.append(req)

    def pending(self):
        return len(self.waiting) + sum(p.occupied() for p in self.all_pools())

    def footprint(self, w, slots):
        cfg = mirve.make_config(w.n, h=w.h, ell=w.ell, k=w.k, f=w.f, precision=self.precision,
                                batch=slots, split=self.split, **self.tol)
        return mirve.rve_query_workspace(cfg)

    # -- admission -----------------------------------------------------------
    def _open_pool(self, key, w):
        """A new pool of the class of w within the budget (closing empty pools
        of other classes if that makes room), or None."""
        slots = self.slots_per_pool
        while slots >= 1:
            need = self.footprint(w, slots)
            if self.used_bytes() + need > self.budget:
                for k2, ps in list(self.pools.items()):
                    for p in list(ps):
                        if p.occupied() == 0 and self.used_bytes() + need > self.budget:
                            p.close()
                            ps.remove(p)
                    if not ps:
                        del self.pools[k2]
            if self.used_bytes() + need <= self.budget:
                pool = Pool(key, w, slots, self.precision, self.split, self.tol)
                self.pools.setdefault(key, []).append(pool)
                self.peak_bytes = max(self.peak_bytes, self.used_bytes())
                return pool
            slots //= 2
        return None

    def _admit(self):
        still = []
        for req in self.waiting:
            key = problem_class(req.workload, self.precision, self.split)
            pool = None
            for p in self.pools.get(key, []):
                if p.free_slot() is not None:
                    pool = p
                    break
            if pool is None:
                pool = self._open_pool(key, req.workload)
            if pool is None and self.used_bytes() == 0:
                # not even a one-slot pool fits the budget: refuse
                now = self.now()
                self.results[req.rid] = Result(req.rid, None, 0, mirve.RVE_ENOSPC, req.arrival,
                                               now, now)
                continue
            if pool is None:
                still.append(req)
                continue
            pool.admit(req, self.now())
        if still:
            self.stalls += 1
        self.waiting = still

    # -- one tick ------------------------------------------------------------
    def tick(self):
        self._admit()
        active = [p for p in self.all_pools() if p.occupied()]
        if not active:
            return []
        outs = list(self._ex.map(lambda p: p.step(self.steps_per_tick), active))
        self.ticks += 1
        done = []
        for p, (infos, status) in zip(active, outs):
            for i, req in enumerate(p.req):
                if req is None:
                    continue
                st = status[i]
                p.steps[i] += infos[i]["n_steps"]
                p.greens[i] += infos[i]["n_greenop"] * int(np.prod(req.workload.n))
                finished = st != 0 or infos[i]["fractured"] or p.steps[i] >= req.max_steps
                if not finished:
                    continue
                G = None
                if st == 0 and infos[i]["fractured"]:
                    G = p.rve.rve_effective_toughness(i)
                elif st == 0:
                    st = mirve.RVE_ENOTDONE
                res = Result(req.rid, G, p.steps[i], st, req.arrival, p.admitted[i], self.now(),
                             p.greens[i])
                self.results[req.rid] = res
                done.append(res)
                p.req[i] = None
                p.rve.rve_release_slot(i)
        return done

    def run(self, requests, realtime=True, on_result=None):
        """Serve requests (sorted by arrival).  With realtime, a request is
        submitted once the clock passes its arrival time; otherwise all are
        submitted at once.  on_result(result) is called as results come."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        k = 0
        self.t0 = self.clock()
        while k < len(reqs) or self.pending():
            now = self.now()
            while k < len(reqs) and (not realtime or reqs[k].arrival <= now):
                self.submit(reqs[k])
                k += 1
            if not self.pending():
                time.sleep(max(0.0, min(0.01, reqs[k].arrival - now)))
                continue
            for res in self.tick():
                if on_result:
                    on_result(res)
        return [self.results[r.rid] for r in requests]

    def close(self):
        for p in self.all_pools():
            p.close()
        self.pools.clear()
        self._ex.shutdown(wait=True)


def summarize(results, wall):
    lat = np.array([r.latency for r in results])
    ok = [r for r in results if r.G_eff is not None]
    return {"requests": len(results), "solved": len(ok), "wall_s": round(wall, 3),
            "solves_per_s": round(len(ok) / wall, 3) if wall > 0 else None,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
            "voxel_iter_per_s": round(sum(r.n_greenop for r in results) / wall, 1) if wall > 0 else None}


def serve_sequential(requests, precision=mirve.RVE_PREC_FP64, split=mirve.RVE_SPLIT_NONE,
                     tol=None, clock=time.perf_counter, on_result=None, chunk=10, on_chunk=None):
    """The plain form: one RVE at a time, first come first served, each in a
    handle of its own (batch 1).  Latency includes the wait behind earlier
    requests; arrivals are honoured (the GPU idles until the next one)."""
    import torch
    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = clock()
    out = {}
    for req in reqs:
        now = clock() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        start = clock() - t0
        w = req.workload
        r = mirve.from_workload(w, precision=precision, split=split, **dict(tol or {}))
        # chunks of `chunk` steps (the same steps as one call; the caller can
        # report progress between them)
        steps = greens = 0
        st, fractured = 0, False
        while steps < req.max_steps and st == 0 and not fractured:
            todo = min(chunk, req.max_steps - steps)
            infos, status = r.rve_run_slots([w.dtau], [todo], stop_at_fracture=True)
            st = status[0]
            steps += infos[0]["n_steps"]
            greens += infos[0]["n_greenop"] * int(np.prod(w.n))
            fractured = bool(infos[0]["fractured"])
            if on_chunk:
                on_chunk(req.rid, steps)
        fractured = fractured and st == 0
        G = r.rve_effective_toughness() if fractured else None
        if st == 0 and not fractured:
            st = mirve.RVE_ENOTDONE
        r.close()
        torch.cuda.synchronize()
        out[req.rid] = Result(req.rid, G, steps, st, req.arrival, start, clock() - t0, greens)
        if on_result:
            on_result(out[req.rid])
    return [out[r.rid] for r in requests]
