"""Precision form of the plasmonic cell: mixed-precision path against the FP64
path on the same inputs, case by case.

Geometry: the 200 x 200 nm cell of the bench (active 80 nm, spacer 40 nm,
Drude-Ag sphere r = 20 nm) meshed at ~3.33 nm fine / 20 nm coarse:
38,400 tetrahedra, N = 77,600 unknowns (complex-FP32 Z 48 GB, FP64 Z 96 GB).
Cases: incidence angles theta (deg) at azimuths phi in {0, 45} deg,
wavelengths in nm, TE and TM (theta = 0 shared between the azimuths).
TE and TM of a case are solved together (vie_solve_pair).  Each
polarisation prints one JSON line (absorptance per domain, R, T, GMRES
iterations, stage times; the solve time is that of the pair) as it finishes; at the end one line per case gives
the largest difference between the paths over A, R and T.

    python -m paper_1809_05334_amd.precision_study --thetas 0,40,80 --lambdas 450,550,650
"""
import argparse
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--thetas", default="0,40,80")
    ap.add_argument("--phis", default="0,45")
    ap.add_argument("--lambdas", default="450,550,650")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=150)
    ap.add_argument("--max-iter", type=int, default=3000)
    args = ap.parse_args()
    import torch

    from . import vie
    from . import workloads as W

    mesh = W.plasmonic_cell_fine_mesh()
    thetas = [float(v) for v in args.thetas.split(",")]
    phis = [float(v) for v in args.phis.split(",")]
    lams = [float(v) for v in args.lambdas.split(",")]
    cases = []
    for lam in lams:
        for th in thetas:
            for ph in (phis if th != 0 else phis[:1]):
                cases.append((lam, th, ph))
    results = {}
    for name, prec in (("mixed", vie.VIE_MIXED_FP32), ("fp64", vie.VIE_FP64)):
        s = vie.Solver(0)
        N = s.upload_mesh(mesh)
        ws = s.bind(prec, args.restart)
        print(f"{name}: N = {N}, workspace {ws / 1e9:.1f} GB", file=sys.stderr, flush=True)
        tuned = False
        for (lam, th, ph) in cases:
            eps = W.osc_eps(mesh, lam)
            t0 = time.perf_counter()
            s.fill(lam, np.deg2rad(th), np.deg2rad(ph), eps)
            s.factor()
            if not tuned:
                s.autotune(reps=2)
                tuned = True
            infos = s.solve_pair(tol=args.tol, max_iter=args.max_iter, restart=args.restart, allow_noconv=True)
            for pol in (vie.VIE_TE, vie.VIE_TM):
                info = infos[pol]
                A, R, T = s.absorption(pol=pol)
                r = {"A": A.tolist(), "R": R, "T": T, "iters": info["iters"], "converged": info["converged"],
                     "fill_ms": info["t_fill_ms"], "factor_ms": info["t_factor_ms"],
                     "pair_solve_ms": info["t_solve_ms"]}
                results[(name, lam, th, ph, pol)] = r
                print(json.dumps({"path": name, "lambda_nm": lam, "theta_deg": th, "phi_deg": ph,
                                  "pol": "TE" if pol == 0 else "TM", **r}), flush=True)
            print(f"{name} lambda {lam:.0f} theta {th:.0f} phi {ph:.0f}: {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    worst = 0.0
    for (lam, th, ph) in cases:
        for pol in (0, 1):
            m, f = results[("mixed", lam, th, ph, pol)], results[("fp64", lam, th, ph, pol)]
            dA = max(float(np.max(np.abs(np.array(m["A"]) - np.array(f["A"])))), abs(m["R"] - f["R"]),
                     abs(m["T"] - f["T"]))
            worst = max(worst, dA)
            print(json.dumps({"lambda_nm": lam, "theta_deg": th, "phi_deg": ph, "pol": "TE" if pol == 0 else "TM",
                              "dA": dA, "iters": [m["iters"], f["iters"]]}), flush=True)
    print(json.dumps({"cases": 2 * len(cases), "max_dA": worst, "N": N}), flush=True)


if __name__ == "__main__":
    main()
