"""The structured-grid operator (VIE_GRID_FP64) against the dense operators on
the plasmonic cell meshed as a uniform Kuhn grid.

Cell: the bench cell's stack (active 80 nm, spacer 40 nm, Drude-Ag sphere
r = 20 nm centred in the spacer), a = b = `--a`, every brick `--h` on a side
(16 x 16 x 24 bricks, N = 74,240 at a = 80 nm, h = 5 nm).  Per operator: the
fill time, the time of one product Z x (`--reps` back to back), the
workspace, and a paired TE + TM solve (GMRES(`--restart`), tol `--tol`): the
grid operator with the forms in `--grid-precond` (identity, M = I, and/or
jacobi, M = diag(Z); it stores no diagonal blocks), the dense ones with the
block-diagonal preconditioner (Sec. 2.3) and the forms in `--dense-extra`.
Absorptances are compared with the FP64 dense solve; the summary line takes
the first grid form.

One JSON line per operator, then one with the grid operator's speedups.

    python -m paper_1809_05334_amd.grid_study --a 80 --h 5
"""
import argparse
import json
import sys
import time

import numpy as np

from . import workloads as W


def run(vie, mesh, prec, precond, args, eps):
    torch = __import__("torch")
    s = vie.Solver()
    N = s.upload_mesh(mesh)
    ws = s.bind(prec, args.restart)
    s.set_option(vie.VIE_OPT_PRECOND, {"block": 0, "identity": 1, "jacobi": 2}[precond])
    t0 = time.perf_counter()
    s.fill(args.lam, args.theta, args.phi, eps)
    torch.cuda.synchronize()
    t_fill_wall = time.perf_counter() - t0
    fs = s.fill_stats()
    mv = s.bench_matvec(args.reps)
    out = {"operator": {vie.VIE_GRID_FP64: "grid", vie.VIE_MIXED_FP32: "mixed", vie.VIE_FP64: "fp64"}[prec],
           "precond": precond, "N": N, "workspace_gb": ws / 1e9, "fill_ms": fs["t_fill_ms"],
           "fill_wall_ms": 1e3 * t_fill_wall, "matvec_ms": mv}
    print(f"  {out['operator']}: fill {fs['t_fill_ms']:.1f} ms, matvec {mv:.3f} ms", file=sys.stderr, flush=True)
    if args.solve:
        t_factor = 0.0
        if precond == "block":
            s.factor()
            t_factor = s.factor_stats()["t_factor_ms"]
        infos = s.solve_pair(tol=args.tol, max_iter=args.max_iter, allow_noconv=True)
        out.update({"factor_ms": t_factor, "iters": [i["iters"] for i in infos],
                    "converged": [bool(i["converged"]) for i in infos], "solve_ms": infos[0]["t_solve_ms"],
                    "A": [list(s.absorption(pol=p, want_rt=False)) for p in (0, 1)]})
        print(f"    solve {out['solve_ms']:.0f} ms, iterations {out['iters']}", file=sys.stderr, flush=True)
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--a", type=float, default=80.0)
    ap.add_argument("--h", type=float, default=5.0)
    ap.add_argument("--lam", type=float, default=600.0)
    ap.add_argument("--theta", type=float, default=0.35)
    ap.add_argument("--phi", type=float, default=0.6)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--operators", default="grid,mixed,fp64")
    ap.add_argument("--solve", action="store_true")
    ap.add_argument("--grid-precond", default="identity", help="comma list of identity, jacobi")
    ap.add_argument("--dense-extra", default="", help="comma list of jacobi, identity (besides block)")
    args = ap.parse_args()

    from . import vie

    mesh = W.osc_cell_mesh(args.a, 80.0, 40.0, 20.0, args.h, args.h)
    eps = W.osc_eps(mesh, args.lam)
    code = {"grid": vie.VIE_GRID_FP64, "mixed": vie.VIE_MIXED_FP32, "fp64": vie.VIE_FP64}
    rows = []
    for name in args.operators.split(","):
        prec = code[name]
        extra = [e for e in args.dense_extra.split(",") if e]
        runs = args.grid_precond.split(",") if prec == vie.VIE_GRID_FP64 else ["block"] + extra
        for pc in runs:
            r = run(vie, mesh, prec, pc, args, eps)
            rows.append(r)
            print(json.dumps(r), flush=True)
    ref = next((r for r in rows if r["operator"] == "fp64" and r["precond"] == "block"), None)
    grid = next((r for r in rows if r["operator"] == "grid"), None)   # the first grid form
    if grid and ref:
        summary = {"summary": "grid vs fp64", "N": grid["N"], "fill_speedup": ref["fill_ms"] / grid["fill_ms"],
                   "matvec_speedup": ref["matvec_ms"] / grid["matvec_ms"],
                   "workspace_ratio": ref["workspace_gb"] / grid["workspace_gb"]}
        if args.solve:
            summary["dA_max"] = float(np.max(np.abs(np.array(grid["A"]) - np.array(ref["A"]))))
            summary["time_to_solution_speedup"] = ((ref["fill_ms"] + ref["factor_ms"] + ref["solve_ms"]) /
                                                   (grid["fill_ms"] + grid["solve_ms"]))
        print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
