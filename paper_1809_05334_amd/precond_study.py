"""Preconditioner study of the plasmonic cell (the Sec. 3 comparison of
Figs. 2-3): GMRES with the block-diagonal preconditioner (Sec. 2.3, Eq. 6)
against GMRES with none (M = I), on the same fill.

Geometry: the 200 x 200 nm cell of the bench (active 80 nm, spacer 40 nm,
Drude-Ag sphere r = 20 nm), 18,432 tetrahedra, N = 37,376 unknowns, normal
incidence, FP64 path by default.  For each polarisation the script prints
one JSON line per preconditioner (iterations, restarts, solve time, true
residual, the residual history every `--every` iterations) and one line with
the difference of the two solutions: Eq. 8, ||x_pre - x_none|| / ||x_none||,
and the distribution of the per-unknown relative difference
|x_pre,i - x_none,i| / |x_none,i| (the quantity of Fig. 3).

    python -m paper_1809_05334_amd.precond_study --lambda 400 --tol 1e-8
    python -m paper_1809_05334_amd.precond_study --lambda 400 --tol 1e-8 --restart 1000 --pols TE
"""
import argparse
import json
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lambda", dest="lam", type=float, default=400.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--pols", default="TE,TM")
    args = ap.parse_args()

    from . import vie
    from . import workloads as W

    mesh = W.plasmonic_cell_mesh()
    prec = vie.VIE_FP64 if args.precision == "fp64" else vie.VIE_MIXED_FP32
    s = vie.Solver(0)
    N = s.upload_mesh(mesh)
    s.bind(prec, args.restart)
    eps = W.osc_eps(mesh, args.lam)
    s.fill(args.lam, 0.0, 0.0, eps)
    s.factor()
    print(f"N = {N}, lambda {args.lam} nm, {args.precision}", file=sys.stderr, flush=True)
    pols = [(vie.VIE_TE, "TE"), (vie.VIE_TM, "TM")]
    for pol, pname in [p for p in pols if p[1] in args.pols.split(",")]:
        sol = {}
        for mode, name in ((0, "block"), (1, "none")):
            s.set_option(vie.VIE_OPT_PRECOND, mode)
            info = s.solve(pol, tol=args.tol, max_iter=args.max_iter, restart=args.restart, allow_noconv=True)
            h = s.residual_history()
            sol[name] = s.read_solution()
            A, R, T = s.absorption()
            print(json.dumps({"pol": pname, "precond": name, "iters": info["iters"], "restarts": info["restarts"],
                              "converged": info["converged"], "solve_ms": info["t_solve_ms"],
                              "true_rel_residual": info["true_rel_residual"], "absorptance": list(A), "R": R,
                              "T": T, "history_every": args.every,
                              "history": [float(v) for v in h[args.every - 1::args.every]]}), flush=True)
        xp, xn = sol["block"], sol["none"]
        rel = np.abs(xp - xn) / np.maximum(np.abs(xn), 1e-300)
        print(json.dumps({"pol": pname, "eq8_rel_error": float(np.linalg.norm(xp - xn) / np.linalg.norm(xn)),
                          "per_unknown_rel": {"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
                                              "max": float(rel.max())}}), flush=True)
    s.set_option(vie.VIE_OPT_PRECOND, 0)


if __name__ == "__main__":
    main()
