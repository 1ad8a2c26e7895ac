"""Batched solves of many independent unit cells of uneven size.

Fused mode (default): cells are grouped into waves (in request order, up to
`max_cells` per wave, each wave's workspaces within its share of the HBM
budget).  A wave is one `vie.Batch`: the library fills every cell of the
wave with one launch per fill kernel and colour pair, factors all their
diagonal blocks in one panel loop, and runs GMRES with every cell's Arnoldi
step in one launch sequence replayed as a captured HIP graph; the fused
matvec's rows per wave come from the autotuner, run once per N bucket
(< 4k, 4-8k, > 8k unknowns) on a cell of that bucket.  `slots`
workers run waves concurrently, each on its own stream, so one wave's host
work (mesh topology, lattice-sum table fits) overlaps another's device work;
a host thread prepares the next cells' meshes ahead of the workers.

Streams mode: the serving scheduler with every arrival at 0, one context and
stream per running cell (the per-cell path the fused mode is compared with).

Results come back in request order.  Throughput is cells/s over the batch.

    python -m paper_1809_05334_amd.batch --cells 256 --slots 2 --precision mixed
"""
from __future__ import annotations

import argparse
import json
import queue
import threading
import time

import numpy as np

from .serve import Result, Server, VieBackend, summarize


def cell_requests(n_cells=256, seed=0, n_lo=2000, n_hi=15000):
    from . import workloads as W
    cells = W.batch_cells(n_cells, seed=seed, n_lo=n_lo, n_hi=n_hi)
    return [{"rid": i, "arrival": 0.0, "cell": c, "lambda": c["lambda"], "theta": c["theta"], "phi": c["phi"],
             "pol": c["pol"]} for i, c in enumerate(cells)]


def _prepare(req, vie, W, device, precision, restart, sym):
    mesh = req["mesh"] if "mesh" in req else W.cell_mesh(req["cell"])
    s = vie.Solver(device, stream=_DummyStream.get(device))
    s.upload_mesh(mesh)
    if sym:   # one lattice sum per unordered far pair (a staging copy of Z's far part)
        s.set_option(vie.VIE_OPT_SYM_FILL, 1)
    eps = req["eps"] if "eps" in req else W.osc_eps(mesh, req["lambda"])
    return {"req": req, "solver": s, "mesh": mesh, "eps": eps, "bytes": s.workspace_bytes(precision, restart)}


class _DummyStream:
    """One shared stream for contexts before they join a wave (the batch
    moves them to its own stream when it binds them)."""
    _s = {}

    @classmethod
    def get(cls, device):
        import torch
        if device not in cls._s:
            cls._s[device] = torch.cuda.Stream(device=device)
        return cls._s[device]


def run_fused(requests, precision, slots=2, budget_gb=200.0, tol=1e-8, restart=100, max_cells=32, graph=True,
              device=0, max_iter=3000, sym=True):
    """Fused batch: returns (results in request order, seconds, stats)."""
    import torch

    from . import vie
    from . import workloads as W
    t0 = time.perf_counter()
    share = budget_gb * 1e9 / max(1, slots)
    prepq = queue.Queue(maxsize=4 * max_cells)
    results = {}
    stats = {"waves": 0, "cells_per_wave": [], "peak_gb": 0.0, "fill_s": 0.0, "factor_s": 0.0, "solve_s": 0.0,
             "fill_wall_s": 0.0}
    lock = threading.Lock()
    used = [0.0]

    def producer():
        for r in requests:
            prepq.put(_prepare(r, vie, W, device, precision, restart, sym))
        for _ in range(slots):
            prepq.put(None)

    wave_lock = threading.Lock()
    pending = []
    tuned = {}   # N bucket -> matvec rows per wave picked by the autotuner

    def bucket(n):
        return 0 if n < 4000 else (1 if n < 8000 else 2)

    def next_wave():
        """Take the next wave from the prepared cells (request order)."""
        with wave_lock:
            wave, nbytes = [], 0
            while len(wave) < max_cells:
                if pending:
                    p = pending.pop(0)
                else:
                    p = prepq.get()
                    if p is None:
                        prepq.put(None)   # leave the end mark for the other workers
                        break
                if wave and nbytes + p["bytes"] > share:
                    pending.insert(0, p)
                    break
                wave.append(p)
                nbytes += p["bytes"]
            return wave, nbytes

    def worker(wid):
        stream = torch.cuda.Stream(device=device)
        while True:
            wave, nbytes = next_wave()
            if not wave:
                return
            with lock:
                used[0] += nbytes
                stats["peak_gb"] = max(stats["peak_gb"], used[0] / 1e9)
                stats["waves"] += 1
                stats["cells_per_wave"].append(len(wave))
            try:
                for p in wave:
                    p["solver"].set_stream(stream)
                    p["solver"].bind(precision, restart)
                b = vie.Batch([p["solver"] for p in wave], device=device, stream=stream, graph=graph)
                tf = time.perf_counter()
                b.fill([p["req"]["lambda"] for p in wave], [p["req"]["theta"] for p in wave],
                       [p["req"]["phi"] for p in wave], [p["eps"] for p in wave])
                tf = time.perf_counter() - tf
                b.factor()
                # launch shapes per N bucket: the autotuner times the matvec
                # variants on one cell of the bucket (first wave holding it)
                for p in wave:
                    k = bucket(p["solver"].num_unknowns())
                    with lock:
                        pick = tuned.get(k)
                    if pick is None:
                        pick = p["solver"].autotune(reps=2)["matvec_rows"]
                        with lock:
                            tuned[k] = pick
                            stats.setdefault("matvec_rows_by_bucket", {})[str(k)] = pick
                    p["solver"].set_option(vie.VIE_OPT_MATVEC_ROWS, pick)
                infos = b.solve([p["req"]["pol"] for p in wave], tol=tol, max_iter=max_iter, restart=restart,
                                allow_noconv=True)
                t_done = time.perf_counter()
                with lock:   # device time of the wave's stages (HIP events), and the fill's wall time
                    stats["fill_s"] += infos[0]["t_fill_ms"] / 1e3
                    stats["factor_s"] += infos[0]["t_factor_ms"] / 1e3
                    stats["solve_s"] += infos[0]["t_solve_ms"] / 1e3
                    stats["fill_wall_s"] += tf
                for p, inf in zip(wave, infos):
                    s = p["solver"]
                    A, R, T = s.absorption()
                    res = Result(rid=p["req"]["rid"], N=s.num_unknowns(), A=list(A), R=R, T=T, iters=inf["iters"],
                                 footprint=p["bytes"], t_arrival=t0, t_admit=t0, t_done=t_done, worker=wid)
                    if not inf["converged"]:
                        res.ok, res.error = False, "GMRES did not converge"
                    with lock:
                        results[res.rid] = res
                b.close()
            except Exception as e:  # the wave's cells fail, the batch goes on
                for p in wave:
                    with lock:
                        results[p["req"]["rid"]] = Result(rid=p["req"]["rid"], ok=False,
                                                          error=f"{type(e).__name__}: {e}")
            finally:
                for p in wave:
                    p["solver"].close()
                torch.cuda.empty_cache()   # the wave's workspaces back to the device (see serve.VieBackend.release)
                with lock:
                    used[0] -= nbytes

    prod = threading.Thread(target=producer, daemon=True)
    prod.start()
    ws = [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(slots)]
    for w in ws:
        w.start()
    for w in ws:
        w.join()
    prod.join()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return [results[r["rid"]] for r in requests], dt, stats


def run_batch(requests, precision, slots=2, budget_gb=200.0, tol=1e-8, restart=100, mode="fused", max_cells=32,
              graph=True, sym=True):
    """Solve the requests as one batch; returns (results in request order,
    seconds, stats).  mode: 'fused' (vie.Batch waves) or 'streams' (one
    context and stream per running cell)."""
    if mode == "fused":
        return run_fused(requests, precision, slots=slots, budget_gb=budget_gb, tol=tol, restart=restart,
                         max_cells=max_cells, graph=graph, sym=sym)
    be = VieBackend(precision=precision, tol=tol, restart=restart)
    srv = Server(be, slots=slots, hbm_budget=budget_gb * 1e9, max_skip_s=1e9)
    t0 = time.perf_counter()
    res = srv.run_trace(requests)
    dt = time.perf_counter() - t0
    return res, dt, {"peak_gb": srv.peak_used / 1e9, "peak_running": srv.peak_running}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--max-cells", type=int, default=32)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--mode", choices=["fused", "streams"], default="fused")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-sym-fill", action="store_true")
    ap.add_argument("--precision", choices=["mixed", "fp64", "both"], default="both")
    args = ap.parse_args()
    from . import vie
    reqs = cell_requests(args.cells)
    out = {}
    runs = {"mixed": vie.VIE_MIXED_FP32, "fp64": vie.VIE_FP64}
    sel = list(runs) if args.precision == "both" else [args.precision]
    results = {}
    for name in sel:
        res, dt, st = run_batch(reqs, runs[name], args.slots, args.budget_gb, args.tol, mode=args.mode,
                                max_cells=args.max_cells, graph=not args.no_graph, sym=not args.no_sym_fill)
        results[name] = res
        s = summarize(res, dt)
        ok = [r for r in res if r.ok]
        out[name] = {"mode": args.mode, "cells": len(res), "ok": s["ok"], "seconds": dt, "cells_per_s": s["ok"] / dt,
                     "N": s["N"], "iters_mean": float(np.mean([r.iters for r in ok])) if ok else 0.0,
                     "failed": [r.error for r in res if not r.ok][:3], **{k: v for k, v in st.items()
                                                                         if k != "cells_per_wave"}}
        print(f"{name}: {json.dumps(out[name])}", flush=True)
    if len(results) == 2:
        dA = max(max(np.max(np.abs(np.array(a.A) - np.array(b.A))), abs(a.R - b.R), abs(a.T - b.T))
                 for a, b in zip(results["mixed"], results["fp64"]) if a.ok and b.ok)
        out["dA_mixed_vs_fp64"] = float(dA)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
