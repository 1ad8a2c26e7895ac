"""Continuous-batching request loop over libvie.

A request is one solve: (unit cell, wavelength, incidence angles,
polarisation) -> absorptance per domain, R and T.  Requests arrive over time
(a trace with arrival times, or `submit` from a client).  While others run, a
request is admitted as soon as a worker slot is free and its device footprint
fits the HBM budget:
- each request owns one library context; its Z, block factors and Krylov
  basis stay resident in its workspace until it finishes;
- each worker owns one HIP stream, so admitted requests run concurrently on
  the device;
- the footprint is the exact `vie_workspace_bytes` of the request's mesh, so
  the sum over admitted requests never exceeds the budget.

Admission policy:
- first come, first served, with skip-ahead: when the oldest waiting request
  does not fit, younger ones that fit are admitted;
- once the oldest has waited longer than `max_skip_s`, nothing is admitted
  ahead of it, so large requests are not starved.

The scheduler is independent of the device (`Server` takes a backend), which
lets the CPU tests drive it with a fake backend.  `VieBackend` is the real
one.  Everything a request computes runs in libvie's kernels; this module only
orders and dispatches.

    python -m paper_1809_05334_amd.serve --rates 2,5,10 --requests 40 --precision mixed
"""
from __future__ import annotations

import argparse
import json
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    rid: int
    ok: bool = True
    error: str = ""
    N: int = 0
    footprint: int = 0
    A: list = field(default_factory=list)
    R: float = 0.0
    T: float = 0.0
    iters: int = 0
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    worker: int = -1

    @property
    def latency(self):
        return self.t_done - self.t_arrival


class _Job:
    __slots__ = ("req", "prep", "footprint", "t_arrival", "t_admit", "result")

    def __init__(self, req, prep, footprint, t_arrival):
        self.req, self.prep, self.footprint, self.t_arrival = req, prep, footprint, t_arrival
        self.t_admit = 0.0
        self.result = None


class Server:
    """Admission, dispatch and bookkeeping; the backend does the solving.

    backend.prepare(req) -> (prep, footprint_bytes)   (host work, any thread)
    backend.make_worker(i) -> worker state (e.g. a HIP stream)
    backend.run(prep, worker_state) -> dict(N, A, R, T, iters)
    backend.release(prep)
    """

    def __init__(self, backend, slots=4, hbm_budget=200e9, max_skip_s=2.0, clock=time.perf_counter):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.backend, self.slots, self.budget = backend, slots, float(hbm_budget)
        self.max_skip_s = max_skip_s
        self.clock = clock
        self._cv = threading.Condition()
        self._pending = deque()          # prepared jobs waiting for admission, arrival order
        self._free = list(range(slots))  # idle worker ids
        self._inbox = [deque() for _ in range(slots)]
        self._used = 0.0
        self._running = 0
        self._stop = False
        self.done = []
        self.peak_used = 0.0
        self.peak_running = 0
        self.admit_order = []
        self._workers = []

    # ------------------------------------------------------------ workers
    def _worker(self, wid):
        state = self.backend.make_worker(wid)
        while True:
            with self._cv:
                while not self._inbox[wid] and not self._stop:
                    self._cv.wait()
                if not self._inbox[wid]:
                    return
                job = self._inbox[wid].popleft()
            res = Result(rid=job.req["rid"], footprint=job.footprint, t_arrival=job.t_arrival, t_admit=job.t_admit,
                         worker=wid)
            try:
                out = self.backend.run(job.prep, state)
                res.N, res.A, res.R, res.T, res.iters = out["N"], list(out["A"]), out["R"], out["T"], out["iters"]
            except Exception as e:  # a failed request must not take the server down
                res.ok, res.error = False, f"{type(e).__name__}: {e}"
            finally:
                self.backend.release(job.prep)
            res.t_done = self.clock()
            with self._cv:
                self._used -= job.footprint
                self._running -= 1
                self._free.append(wid)
                self.done.append(res)
                self._cv.notify_all()

    def start(self):
        for i in range(self.slots):
            th = threading.Thread(target=self._worker, args=(i,), daemon=True)
            th.start()
            self._workers.append(th)

    def stop(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for th in self._workers:
            th.join()

    # ------------------------------------------------------------ admission
    def _admit_locked(self, now):
        """Admit what fits; called with the lock held."""
        admitted = False
        head_blocked = False
        i = 0
        while i < len(self._pending) and self._free:
            job = self._pending[i]
            if self._used + job.footprint <= self.budget:
                del self._pending[i]
                wid = self._free.pop(0)
                job.t_admit = now
                self._used += job.footprint
                self._running += 1
                self.peak_used = max(self.peak_used, self._used)
                self.peak_running = max(self.peak_running, self._running)
                self.admit_order.append(job.req["rid"])
                self._inbox[wid].append(job)
                admitted = True
                continue
            # the head does not fit: skip ahead only while it has not waited too long
            if i == 0:
                head_blocked = now - job.t_arrival > self.max_skip_s
            if head_blocked:
                break
            i += 1
        if admitted:
            self._cv.notify_all()

    def _enqueue(self, req, t_arrival):
        prep, fp = self.backend.prepare(req)
        job = _Job(req, prep, fp, t_arrival)
        with self._cv:
            if fp > self.budget:
                self.backend.release(prep)
                self.done.append(Result(rid=req["rid"], ok=False, error="footprint exceeds the HBM budget",
                                        footprint=fp, t_arrival=t_arrival, t_done=self.clock()))
                return
            self._pending.append(job)
            self._admit_locked(self.clock())

    def run_trace(self, requests, time_scale=1.0, progress_s=0.0):
        """Replay requests at their `arrival` times (s, scaled); returns the
        results in request order once all have finished.  progress_s > 0:
        a line on stderr every progress_s seconds."""
        import sys
        reqs = sorted(requests, key=lambda r: r["arrival"])
        self.start()
        t0 = self.clock()
        t_prog = t0
        k = 0
        try:
            while True:
                now = self.clock()
                if progress_s > 0 and now - t_prog >= progress_s:
                    t_prog = now
                    print(f"serve: {len(self.done)}/{len(reqs)} done, {self._running} running, "
                          f"{len(self._pending)} waiting at {now - t0:.0f} s", file=sys.stderr, flush=True)
                while k < len(reqs) and t0 + reqs[k]["arrival"] * time_scale <= now:
                    self._enqueue(reqs[k], t0 + reqs[k]["arrival"] * time_scale)
                    k += 1
                with self._cv:
                    self._admit_locked(self.clock())
                    if k == len(reqs) and not self._pending and self._running == 0:
                        break
                    nxt = t0 + reqs[k]["arrival"] * time_scale if k < len(reqs) else None
                    wait = 0.05 if nxt is None else max(0.0, min(0.05, nxt - self.clock()))
                    if wait > 0:
                        self._cv.wait(timeout=wait)
        finally:
            self.stop()
        self.t_start, self.t_end = t0, self.clock()
        return sorted(self.done, key=lambda r: r.rid)


def summarize(results, t_span):
    ok = [r for r in results if r.ok]
    lat = np.array([r.latency for r in ok]) * 1e3 if ok else np.zeros(1)
    return {"requests": len(results), "ok": len(ok), "solves_per_s": len(ok) / t_span if t_span > 0 else 0.0,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean())},
            "N": {"min": int(min(r.N for r in ok)) if ok else 0, "max": int(max(r.N for r in ok)) if ok else 0}}


# ---------------------------------------------------------------- libvie backend
class VieBackend:
    """Runs each request through libvie on its own context."""

    def __init__(self, device=0, precision=None, restart=100, tol=1e-8, max_iter=3000, sym=False):
        import torch

        from . import vie
        from . import workloads as W
        self.torch, self.vie, self.W = torch, vie, W
        self.device = device
        self.precision = vie.VIE_MIXED_FP32 if precision is None else precision
        self.restart, self.tol, self.max_iter = restart, tol, max_iter
        self.sym = sym   # one lattice sum per unordered far pair (admission counts its staging copy)
        # prepared contexts wait on one shared stream (they issue no device
        # work before `run` moves them to a worker's stream)
        self.prep_stream = torch.cuda.Stream(device=device)

    def make_worker(self, wid):
        return self.torch.cuda.Stream(device=self.device)

    def prepare(self, req):
        # a request names a cell of the workload generator, or brings its own
        # mesh (and then may bring its own per-tetrahedron permittivities)
        mesh = req["mesh"] if "mesh" in req else self.W.cell_mesh(req["cell"])
        s = self.vie.Solver(self.device, stream=self.prep_stream)
        s.upload_mesh(mesh)
        if self.sym:
            s.set_option(self.vie.VIE_OPT_SYM_FILL, 1)
        fp = s.workspace_bytes(self.precision, self.restart)
        return {"solver": s, "mesh": mesh, "req": req}, fp

    def run(self, prep, stream):
        s, mesh, req = prep["solver"], prep["mesh"], prep["req"]
        s.set_stream(stream)
        s.bind(self.precision, self.restart)
        eps = req["eps"] if "eps" in req else self.W.osc_eps(mesh, req["lambda"])
        s.fill(req["lambda"], req["theta"], req["phi"], eps)
        s.factor()
        info = s.solve(req["pol"], tol=self.tol, max_iter=self.max_iter, restart=self.restart)
        A, R, T = s.absorption()
        return {"N": s.num_unknowns(), "A": A.tolist(), "R": R, "T": T, "iters": info["iters"]}

    def release(self, prep):
        s = prep.get("solver")
        if s is not None:
            big = s.ws is not None and s.ws.numel() >= (1 << 30)
            s.close()   # waits for the context's stream, then drops the workspace
            prep["solver"] = None
            if big:
                # hand a large workspace back to the device at once: kept in
                # torch's cache it would hold memory that neither the next
                # request (of another size) nor the HIP runtime (queues,
                # scratch) could use
                self.torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="2,5,10")
    ap.add_argument("--requests", type=int, default=40)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--sym-fill", action="store_true", help="one lattice sum per unordered far pair")
    ap.add_argument("--out", default="", help="write each request's result to this JSON file (per rate)")
    args = ap.parse_args()
    from . import vie
    from . import workloads as W
    prec = vie.VIE_MIXED_FP32 if args.precision == "mixed" else vie.VIE_FP64
    per = {}
    for rate in [float(r) for r in args.rates.split(",")]:
        trace = W.serve_trace(rate, args.requests, seed=args.seed)
        be = VieBackend(precision=prec, tol=args.tol, sym=args.sym_fill)
        srv = Server(be, slots=args.slots, hbm_budget=args.budget_gb * 1e9)
        res = srv.run_trace(trace, progress_s=30.0)
        out = summarize(res, srv.t_end - srv.t_start)
        out.update({"rate_req_s": rate, "precision": args.precision, "slots": args.slots,
                    "budget_gb": args.budget_gb, "peak_gb": srv.peak_used / 1e9, "peak_running": srv.peak_running,
                    "sym_fill": args.sym_fill, "failed": [r.error for r in res if not r.ok][:3]})
        print(json.dumps(out), flush=True)
        per[str(rate)] = [{"rid": r.rid, "ok": r.ok, "N": r.N, "A": r.A, "R": r.R, "T": r.T, "iters": r.iters,
                           "latency_s": r.latency} for r in res]
        if args.out:
            with open(args.out, "w") as f:
                json.dump(per, f)


if __name__ == "__main__":
    main()
