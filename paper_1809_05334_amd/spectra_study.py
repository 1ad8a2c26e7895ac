"""Absorption-enhancement spectra against the lattice constant, and the
angular response, of the plasmonic cell (the Sec. 3 studies of Figs. 4 and 6).

Cells: the bench cell's stack (active 80 nm, spacer 40 nm, Drude-Ag sphere
r = 20 nm centred in the spacer) at lattice constants a = b from `--periods`,
meshed at 5 nm over the sphere's span and the spacer, 20 nm elsewhere.
Absorption counts the active layer only (Fig. 4).  Enhancement = A_active with
the particle / A_active on the same mesh with the particle's tetrahedra given
the spacer's permittivity (no particle).  TE and TM are solved and averaged
(unpolarised light).

Every solve of a study is one request of the batched (default) or served path
(`--path`): a study builds its requests (cell, wavelength, angle,
polarisation, with or without the particle), the batch driver or the serving
loop runs them on the device, and the reductions below turn their absorptances
into enhancement factors and normalised absorbed power.

Spectra (normal incidence): one JSON line per (a, lambda).  Angular response
(azimuth 0) at lattice constant `--angle-period`: one JSON line per
(lambda, theta) with the absorptance, the enhancement and the absorbed power
normalised to normal incidence, A(theta) cos(theta) / A(0), next to the ideal
Lambertian cos(theta) (Fig. 6).

Checkpoint / resume (`--out study.jsonl`): every solve appends one JSON
record, keyed by (a, lambda, theta, phi, polarisation, variant), as soon as its
study group returns; on restart the records already in the file are read back
and only the missing solves run.  A partial last line (a run killed while
writing) is ignored and its solve redone.

    python -m paper_1809_05334_amd.spectra_study --periods 60,80,120,200 --lambdas 400:800:50
"""
import argparse
import json
import os
import sys

import numpy as np

from . import workloads as W

TE, TM = 0, 1


def axis(spec):
    if ":" in spec:
        lo, hi, st = (float(v) for v in spec.split(":"))
        return list(np.arange(lo, hi + 0.5 * st, st))
    return [float(v) for v in spec.split(",")]


def eps_variants(mesh, lam):
    """Per-tetrahedron permittivities with the particle, and with the particle's
    tetrahedra given the spacer's permittivity (the reference cell)."""
    e = W.osc_eps(mesh, lam)
    ref = e.copy()
    ref[mesh.tet_domain == W.DOM_METAL] = W.EPS_SPACER
    return {"particle": e, "none": ref}


def study_requests(mesh, cases, rid0=0):
    """One request per (case, variant, polarisation); cases are
    (lambda nm, theta deg).  Each request carries its tag (case index,
    variant, polarisation)."""
    reqs = []
    for ci, (lam, th) in enumerate(cases):
        for var, eps in eps_variants(mesh, lam).items():
            for pol in (TE, TM):
                reqs.append({"rid": rid0 + len(reqs), "arrival": 0.0, "mesh": mesh, "eps": eps, "lambda": lam,
                             "theta": float(np.deg2rad(th)), "phi": 0.0, "pol": pol, "tag": (ci, var, pol)})
    return reqs


def reduce_active(reqs, results, dom=W.DOM_ACTIVE):
    """Unpolarised absorptance of domain `dom` per (case index, variant):
    the mean over TE and TM."""
    acc = {}
    for rq, rs in zip(reqs, results):
        if not rs.ok:
            raise RuntimeError(f"request {rs.rid} failed: {rs.error}")
        ci, var, _ = rq["tag"]
        acc.setdefault((ci, var), []).append(rs.A[dom])
    return {k: float(np.mean(v)) for k, v in acc.items()}


def enhancement(active, ci):
    """Enhancement of case ci: A_active with the particle / without."""
    return active[(ci, "particle")] / active[(ci, "none")]


def angular_response(active, cases, ci, ci0):
    """Absorbed power at case ci normalised to the normal-incidence case ci0,
    A(theta) cos(theta) / A(0) (with the particle)."""
    return active[(ci, "particle")] * float(np.cos(np.deg2rad(cases[ci][1]))) / active[(ci0, "particle")]


def run_requests(reqs, precision, path="batch", slots=4, tol=1e-8, restart=200):
    """Solve the requests on the batched or the served path; results in
    request order."""
    if path == "batch":
        from . import batch as B
        res, _, _ = B.run_batch(reqs, precision, slots=slots, tol=tol, restart=restart)
        return res
    from . import serve as S
    srv = S.Server(S.VieBackend(precision=precision, tol=tol, restart=restart), slots=slots, hbm_budget=200e9)
    return srv.run_trace(reqs)


def solve_key(a_nm, rq):
    """Checkpoint key of one solve: lattice constant, wavelength, angles,
    polarisation and variant, rounded so a key read back from JSON compares
    equal to the one rebuilt from the request."""
    _, var, pol = rq["tag"]
    return (round(float(a_nm), 9), round(float(rq["lambda"]), 9), round(float(np.rad2deg(rq["theta"])), 9),
            round(float(np.rad2deg(rq["phi"])), 9), int(pol), str(var))


class Checkpoint:
    """Append-only JSONL record of finished solves (one line per solve)."""

    def __init__(self, path):
        self.path = path
        self.done = {}
        if path and os.path.exists(path):
            with open(path, "rb+") as f:
                data = f.read()
                keep = data.rfind(b"\n") + 1
                if keep < len(data):      # partial last line of an interrupted write: cut it off,
                    f.truncate(keep)      # so the next record starts on a line of its own
            for line in data[:keep].decode().splitlines():
                try:
                    r = json.loads(line)
                except json.JSONDecodeError:
                    continue
                self.done[tuple(r["key"])] = r

    def append(self, key, res):
        rec = {"key": list(key), "N": int(res.N), "A": [float(v) for v in res.A], "R": float(res.R),
               "T": float(res.T), "iters": int(res.iters)}
        self.done[key] = rec
        if self.path:
            with open(self.path, "a") as f:
                f.write(json.dumps(rec) + "\n")
                f.flush()
                os.fsync(f.fileno())


def run_with_checkpoint(a_nm, reqs, ckpt, run, **kw):
    """Results of `reqs` in request order: the ones `ckpt` holds are read
    back, the rest are solved by `run(pending, **kw)` and appended to it.
    A failed solve is not recorded (it raises in the reduction and runs again
    on restart)."""
    from .serve import Result
    keys = [solve_key(a_nm, rq) for rq in reqs]
    pending = [i for i, k in enumerate(keys) if k not in ckpt.done]
    out = [None] * len(reqs)
    if pending:
        res = run([reqs[i] for i in pending], **kw)
        for i, rs in zip(pending, res):
            out[i] = rs
            if rs.ok:
                ckpt.append(keys[i], rs)
    for i, k in enumerate(keys):
        if out[i] is None:
            r = ckpt.done[k]
            out[i] = Result(rid=reqs[i]["rid"], N=r["N"], A=list(r["A"]), R=r["R"], T=r["T"], iters=r["iters"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--periods", default="60,80,120,200")
    ap.add_argument("--lambdas", default="400:800:50")
    ap.add_argument("--angle-period", type=float, default=80.0)
    ap.add_argument("--angle-lambdas", default="500,600,750")
    ap.add_argument("--thetas", default="0,20,40,60,80")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--path", choices=["batch", "serve"], default="batch")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--out", default="", help="JSONL checkpoint: append each solve, skip those already there")
    args = ap.parse_args()

    from . import vie

    prec = vie.VIE_MIXED_FP32 if args.precision == "mixed" else vie.VIE_FP64

    def cell(a):
        return W.osc_cell_mesh(a, 80.0, 40.0, 20.0, 5.0, 20.0)

    ckpt = Checkpoint(args.out)
    if ckpt.done:
        print(f"resuming: {len(ckpt.done)} solves read from {args.out}", file=sys.stderr, flush=True)
    kw = dict(precision=prec, path=args.path, slots=args.slots, tol=args.tol, restart=args.restart)

    for a in axis(args.periods):
        mesh = cell(a)
        cases = [(lam, 0.0) for lam in axis(args.lambdas)]
        reqs = study_requests(mesh, cases)
        res = run_with_checkpoint(a, reqs, ckpt, run_requests, **kw)
        act = reduce_active(reqs, res)
        metal = reduce_active(reqs, res, W.DOM_METAL)
        for ci, (lam, _) in enumerate(cases):
            print(json.dumps({"study": "spectrum", "a_nm": a, "lambda_nm": lam, "N": res[0].N,
                              "A_active": act[(ci, "particle")], "A_active_no_particle": act[(ci, "none")],
                              "enhancement": enhancement(act, ci), "A_metal": metal[(ci, "particle")]}), flush=True)
    mesh = cell(args.angle_period)
    thetas = axis(args.thetas)
    for lam in axis(args.angle_lambdas):
        cases = [(lam, th) for th in thetas]
        reqs = study_requests(mesh, cases)
        res = run_with_checkpoint(args.angle_period, reqs, ckpt, run_requests, **kw)
        act = reduce_active(reqs, res)
        ci0 = thetas.index(0.0) if 0.0 in thetas else 0
        for ci, (_, th) in enumerate(cases):
            print(json.dumps({"study": "angle", "a_nm": args.angle_period, "lambda_nm": lam, "theta_deg": th,
                              "A_active": act[(ci, "particle")], "enhancement": enhancement(act, ci),
                              "normalised_absorbed_power": angular_response(act, cases, ci, ci0),
                              "lambertian": float(np.cos(np.deg2rad(th)))}), flush=True)
        print(f"lambda {lam:.0f} nm done", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
