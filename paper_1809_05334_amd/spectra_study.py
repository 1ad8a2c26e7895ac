"""Absorption-enhancement spectra against the lattice constant, and the
angular response, of the plasmonic cell (the Sec. 3 studies of Figs. 4 and 6).

Cells: the bench cell's stack (active 80 nm, spacer 40 nm, Drude-Ag sphere
r = 20 nm centred in the spacer) at lattice constants a = b from `--periods`,
meshed at 5 nm over the sphere's span and the spacer, 20 nm elsewhere.
Absorption counts the active layer only (Fig. 4).  Enhancement = A_active with
the particle / A_active on the same mesh with the particle's tetrahedra given
the spacer's permittivity (no particle).  TE and TM are solved together and
averaged (unpolarised light).

Spectra (normal incidence): one JSON line per (a, lambda).  Angular response
(azimuth 0) at lattice constant `--angle-period`: one JSON line per
(lambda, theta) with the absorptance, the enhancement and the absorbed power
normalised to normal incidence, A(theta) cos(theta) / A(0), next to the ideal
Lambertian cos(theta) (Fig. 6).

    python -m paper_1809_05334_amd.spectra_study --periods 60,80,120,200 --lambdas 400:800:50
"""
import argparse
import json
import sys

import numpy as np


def axis(spec):
    if ":" in spec:
        lo, hi, st = (float(v) for v in spec.split(":"))
        return list(np.arange(lo, hi + 0.5 * st, st))
    return [float(v) for v in spec.split(",")]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--periods", default="60,80,120,200")
    ap.add_argument("--lambdas", default="400:800:50")
    ap.add_argument("--angle-period", type=float, default=80.0)
    ap.add_argument("--angle-lambdas", default="500,600,750")
    ap.add_argument("--thetas", default="0,20,40,60,80")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=200)
    args = ap.parse_args()

    from . import vie
    from . import workloads as W

    prec = vie.VIE_MIXED_FP32 if args.precision == "mixed" else vie.VIE_FP64

    def solver(mesh):
        s = vie.Solver(0)
        s.upload_mesh(mesh)
        s.set_option(vie.VIE_OPT_SYM_FILL, 1)   # normal-incidence fills evaluate each far pair once
        s.bind(prec, args.restart)
        return s

    def active(s, mesh, lam, th, eps):
        s.fill(lam, np.deg2rad(th), 0.0, eps)
        s.factor()
        info = s.solve_pair(tol=args.tol, max_iter=4000, restart=args.restart)
        A = [s.absorption(pol=p)[0] for p in (vie.VIE_TE, vie.VIE_TM)]
        return 0.5 * (A[0][W.DOM_ACTIVE] + A[1][W.DOM_ACTIVE]), 0.5 * (A[0][W.DOM_METAL] + A[1][W.DOM_METAL]), \
            [i["iters"] for i in info]

    def eps_pair(mesh, lam):
        e = W.osc_eps(mesh, lam)
        ref = e.copy()
        ref[mesh.tet_domain == W.DOM_METAL] = W.EPS_SPACER
        return e, ref

    def cell(a):
        return W.osc_cell_mesh(a, 80.0, 40.0, 20.0, 5.0, 20.0)

    for a in axis(args.periods):
        mesh = cell(a)
        s = solver(mesh)
        print(f"a = {a} nm: N = {s.num_unknowns()}", file=sys.stderr, flush=True)
        for lam in axis(args.lambdas):
            e, ref = eps_pair(mesh, lam)
            A_np, A_m, it = active(s, mesh, lam, 0.0, e)
            A_ref, _, it_ref = active(s, mesh, lam, 0.0, ref)
            print(json.dumps({"study": "spectrum", "a_nm": a, "lambda_nm": lam, "N": s.num_unknowns(),
                              "A_active": A_np, "A_active_no_particle": A_ref, "enhancement": A_np / A_ref,
                              "A_metal": A_m, "iters": it, "iters_no_particle": it_ref}), flush=True)
        del s
    mesh = cell(args.angle_period)
    s = solver(mesh)
    for lam in axis(args.angle_lambdas):
        A0 = None
        for th in axis(args.thetas):
            e, ref = eps_pair(mesh, lam)
            A_np, _, it = active(s, mesh, lam, th, e)
            A_ref, _, _ = active(s, mesh, lam, th, ref)
            A0 = A_np if A0 is None else A0
            c = float(np.cos(np.deg2rad(th)))
            print(json.dumps({"study": "angle", "a_nm": args.angle_period, "lambda_nm": lam, "theta_deg": th,
                              "A_active": A_np, "enhancement": A_np / A_ref,
                              "normalised_absorbed_power": A_np * c / A0, "lambertian": c, "iters": it}), flush=True)


if __name__ == "__main__":
    main()
