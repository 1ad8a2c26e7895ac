"""Batched solves of many independent unit cells of uneven size.

All cells are queued at once; the serving scheduler admits them in waves
under the HBM budget, one context and one stream per running cell.  Results
come back in cell order.  Throughput is cells/s over the whole batch.

    python -m paper_1809_05334_amd.batch --cells 256 --slots 8 --precision mixed
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from .serve import Server, VieBackend, summarize


def cell_requests(n_cells=256, seed=0, n_lo=2000, n_hi=15000):
    from . import workloads as W
    cells = W.batch_cells(n_cells, seed=seed, n_lo=n_lo, n_hi=n_hi)
    return [{"rid": i, "arrival": 0.0, "cell": c, "lambda": c["lambda"], "theta": c["theta"], "phi": c["phi"],
             "pol": c["pol"]} for i, c in enumerate(cells)]


def run_batch(requests, precision, slots=8, budget_gb=200.0, tol=1e-8, restart=100):
    be = VieBackend(precision=precision, tol=tol, restart=restart)
    srv = Server(be, slots=slots, hbm_budget=budget_gb * 1e9, max_skip_s=1e9)
    t0 = time.perf_counter()
    res = srv.run_trace(requests)
    dt = time.perf_counter() - t0
    return res, dt, srv


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", choices=["mixed", "fp64", "both"], default="both")
    args = ap.parse_args()
    from . import vie
    reqs = cell_requests(args.cells)
    out = {}
    runs = {"mixed": vie.VIE_MIXED_FP32, "fp64": vie.VIE_FP64}
    sel = list(runs) if args.precision == "both" else [args.precision]
    results = {}
    for name in sel:
        res, dt, srv = run_batch(reqs, runs[name], args.slots, args.budget_gb, args.tol)
        results[name] = res
        s = summarize(res, dt)
        out[name] = {"cells": len(res), "ok": s["ok"], "seconds": dt, "cells_per_s": s["ok"] / dt,
                     "N": s["N"], "peak_gb": srv.peak_used / 1e9, "peak_running": srv.peak_running,
                     "iters_mean": float(np.mean([r.iters for r in res if r.ok]))}
        print(f"{name}: {json.dumps(out[name])}", flush=True)
    if len(results) == 2:
        dA = max(max(np.max(np.abs(np.array(a.A) - np.array(b.A))), abs(a.R - b.R), abs(a.T - b.T))
                 for a, b in zip(results["mixed"], results["fp64"]) if a.ok and b.ok)
        out["dA_mixed_vs_fp64"] = float(dA)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
