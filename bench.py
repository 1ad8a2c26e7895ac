#!/usr/bin/env python3
"""Throughput of the periodic VIE-MoM hot path on one MI355X.

Workload (the precision form of the plasmonic organic-solar-cell cell, the
angular sweep of Sec. 3 / Fig. 6): period 200 x 200 nm, active layer 80 nm
(eps 3.6+0.6i), spacer 40 nm (eps 2.3+0.05i), Drude-silver sphere r = 20 nm
in the spacer; graded Kuhn brick mesh at 3.33 nm over the sphere span and
the spacer, 20 nm elsewhere: 38,400 tetrahedra, N = 77,600 unknowns, three
material domains (complex-FP32 Z 48 GB, FP64 Z 96 GB).

Cases: theta = 0..80 deg in 5 deg steps at phi in {0, 45} deg (theta = 0
once), lambda in {450, 550, 650} nm: 99 distinct incidences, each solved for
TE and TM.  One step = one case: fill Z at that incidence (Bloch phases of
the oblique wave; each unordered far tetrahedron pair evaluated once, its
swapped block from g_p at the reversed separations, when the staging copy of
Z fits in HBM; --no-sym-fill evaluates every ordered pair), factor the three
diagonal blocks, one paired
right-preconditioned GMRES solve of TE and TM (two GMRES processes in
lockstep sharing each pass over Z and over the factors), absorptance per
domain and R/T for each -> 2 solves.  Steps visit the 99 cases with stride
40 (warm-up steps first), so any run of consecutive steps spreads over the
three wavelengths, both azimuths and the whole angle range.

Paths: the timed steps run on the mixed-precision path (far part of Z stored
in complex FP32, touching-pair terms in FP64, FP32 block factors, FP64
Krylov arithmetic; `value`).  The plain FP64 path then runs a subset of the
same cases (`--fp64-steps`, the first timed ones), and `dA_per_case` gives
the largest absorptance/R/T difference between the paths per case.  Inputs
are resident on the device when the timed region starts (the mesh tables
are uploaded at bind time; the three permittivity vectors are host arrays of
38,400 complex values passed to each fill).

Prints ONE JSON line.  `value` = solves/s of the whole job.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0

LAMBDAS = (450.0, 550.0, 650.0)
STRIDE = 40                      # coprime with the 99 cases


def cases():
    """The 99 distinct incidences (lambda nm, theta deg, phi deg)."""
    out = []
    for lam in LAMBDAS:
        out.append((lam, 0.0, 0.0))
        for ph in (0.0, 45.0):
            for th in range(5, 85, 5):
                out.append((lam, float(th), ph))
    return out


def case_of_step(i, all_cases):
    return all_cases[(STRIDE * i) % len(all_cases)]


FP32_MFMA_PEAK_TFLOPS = 157.3   # dense FP32 matrix-core peak
FAR_PROFILE = os.path.join(ROOT, "profiles", "k_tt_far_rev_counters_osc_cell_N77600.md")
FAR_SOURCES = ["k_fill.hip", "device_math.h", "common.h", "tables.cpp"]   # kernel code and the tables that set its work
LU_PROFILE = os.path.join(ROOT, "profiles", "k_lu_gemm2_counters_osc_cell_N77600.md")
LU_SOURCES = ["k_lu.hip"]


def profile_counters(path, sources):
    """Per-launch figures from a committed counter summary (HBM bytes, and
    hardware FLOPs when recorded), or None when the kernel's sources changed
    after the counters were read."""
    import hashlib
    import re
    try:
        txt = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_1809_05334_amd", "csrc", f), "rb").read())
    m_hash = re.search(r"kernel_source_sha256_16: ([0-9a-f]+)", txt)
    m_val = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", txt)
    m_hw = re.search(r"hw_flops_per_launch: ([0-9.e+]+)", txt)
    if not m_hash or not m_val or m_hash.group(1) != h.hexdigest()[:16]:
        return None
    return {"traffic": float(m_val.group(1)), "hw_flops": float(m_hw.group(1)) if m_hw else None}


def cpu_baseline(mesh, case, n_rows=4, n_lu=3000, seed=0):
    """The CPU oracle on a bounded sample of the same workload, extrapolated:
    fill = (time of n_rows full rows of Z) * N / n_rows; dense LU of Z = time
    of an n_lu x n_lu complex LU * (N / n_lu)^3; two LU solves scaled by
    (N / n_lu)^2.  solves/s = 2 / (fill + LU + 2 solves)."""
    import scipy.linalg as sla

    from oracle import topology as OT
    from oracle import vie as OV
    from paper_1809_05334_amd import workloads as W

    lam, th, ph = case
    t = OT.build(mesh.verts, mesh.tets, mesh.tet_domain, mesh.ndom, mesh.a, mesh.b)
    N = t.N
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(N, n_rows, replace=False))
    wave = OV.make_wave(lam, np.deg2rad(th), np.deg2rad(ph))
    eps = W.osc_eps(mesh, lam)
    from oracle import vie as _v
    pool = _v._pool()
    threads = pool._processes if pool else 1
    t0 = time.perf_counter()
    OV.assemble(t, wave, eps, rows=rows)
    t_rows = time.perf_counter() - t0
    A = rng.standard_normal((n_lu, n_lu)) + 1j * rng.standard_normal((n_lu, n_lu))
    t0 = time.perf_counter()
    f = sla.lu_factor(A)
    t_lu = time.perf_counter() - t0
    bvec = rng.standard_normal(n_lu) + 0j
    t0 = time.perf_counter()
    sla.lu_solve(f, bvec)
    t_sv = time.perf_counter() - t0
    fill = t_rows * N / n_rows
    lu = t_lu * (N / n_lu) ** 3
    sv = t_sv * (N / n_lu) ** 2
    total = fill + lu + 2 * sv
    return {"value": 2.0 / total, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "host_cores": len(os.sched_getaffinity(0)),
            "sample": (f"case lambda {lam:.0f} nm theta {th:.0f} phi {ph:.0f}: {n_rows} rows of Z "
                       f"(x {N} columns, fill on {threads} worker processes) timed and scaled by N/{n_rows}; "
                       f"dense {n_lu}x{n_lu} complex LU and solve (LAPACK threads) timed and scaled by "
                       f"(N/{n_lu})^3, ^2; extrapolated: fill {fill:.0f} s, LU {lu:.0f} s, "
                       f"solve {sv:.1f} s per solve"),
            "seconds_sampled": t_rows + t_lu + t_sv}


def grid_operator(reps=20):
    """The structured-grid operator (VIE_GRID_FP64) on the bench cell's stack
    meshed as a uniform 5 nm Kuhn grid (a = b = 80 nm, 16 x 16 x 24 bricks,
    N = 74,240), 600 nm, theta 0.35, phi 0.6: fill time, time of one product
    y = Z x (HIP events over `reps` products), workspace, and the algorithmic
    HBM bytes of the per-frequency product kernel (the 60^2 kernel tables
    once, the 132 source fields read and the 132 potential fields written).
    Reported beside the headline, not part of it."""
    import gc

    import torch

    from paper_1809_05334_amd import vie
    from paper_1809_05334_amd import workloads as W
    gc.collect()
    torch.cuda.empty_cache()   # the dense legs' workspaces back to the device
    try:
        mesh = W.osc_cell_mesh(80.0, 80.0, 40.0, 20.0, 5.0, 5.0)
        nx, ny, nz = (len(v) - 1 for v in mesh.grid)
        nf = nx * ny * 2 * (nz + 1)
        s = vie.Solver()
        N = s.upload_mesh(mesh)
        ws = s.bind(vie.VIE_GRID_FP64, 20)
        s.fill(600.0, 0.35, 0.6, W.osc_eps(mesh, 600.0))
        fill_ms = s.fill_stats()["t_fill_ms"]
        mv_ms = s.bench_matvec(reps)
        s.close()
        mul_bytes = (60 * 60 + 2 * 132) * nf * 16
        return {"workload": "plasmonic cell on a uniform 5 nm Kuhn grid, 80x80 nm, N=%d, 600 nm, theta 0.35, "
                            "phi 0.6" % N,
                "unknowns": N, "fft_points": nf, "workspace_gb": ws / 1e9, "fill_ms": fill_ms, "matvec_ms": mv_ms,
                "mul_bytes_per_product": mul_bytes, "dtype": "f64"}
    except Exception as e:   # reported, never fatal to the headline line
        return {"error": str(e)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="cases of the timed sequence (the first ones) also run on the FP64 path")
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grid", action="store_true", help="skip the structured-grid operator's figures")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="Arnoldi steps per captured HIP graph (0: plain launches)")
    ap.add_argument("--no-sym-fill", action="store_true",
                    help="evaluate every ordered far pair (no staging copy for the swapped pairs' blocks)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the method's units of parallel work "
              "(sweep points, cells) shard across GPUs without communication: run one process per GPU "
              "on its share of the sweep", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1809_05334_amd import vie
    from paper_1809_05334_amd import workloads as W

    mesh = W.plasmonic_cell_fine_mesh()
    all_cases = cases()
    eps_of = {lam: W.osc_eps(mesh, lam) for lam in LAMBDAS}
    warm = [case_of_step(i, all_cases) for i in range(args.warmup)]
    timed = [case_of_step(args.warmup + i, all_cases) for i in range(args.steps)]

    def run_path(precision, warm_cases, timed_cases):
        """Warm-up + timed steps on one solver; returns its record."""
        name = "mixed" if precision == vie.VIE_MIXED_FP32 else "fp64"
        s = vie.Solver(0)
        N = s.upload_mesh(mesh)
        sym = False
        if not args.no_sym_fill:
            # one lattice-sum evaluation per unordered far pair (staging copy of
            # the far part of Z), when the larger workspace fits the free HBM
            s.set_option(vie.VIE_OPT_SYM_FILL, 1)
            free, _ = torch.cuda.mem_get_info(0)
            sym = s.workspace_bytes(precision, args.restart) + (8 << 30) <= free
            if not sym:
                s.set_option(vie.VIE_OPT_SYM_FILL, 0)
        ws_bytes = s.bind(precision, args.restart)
        if args.graph_steps:
            s.set_option(vie.VIE_OPT_GRAPH_STEPS, args.graph_steps)
        lat, stages, fills, facs, results, step_s = [], [], [], [], [], []

        def step(i, case):
            lam, th, ph = case
            t0 = time.perf_counter()
            s.fill(lam, np.deg2rad(th), np.deg2rad(ph), eps_of[lam])
            fills.append({**s.fill_stats(), "oblique": th != 0})
            s.factor()
            facs.append(s.factor_stats())
            infos = s.solve_pair(tol=args.tol, max_iter=args.max_iter, restart=args.restart, allow_noconv=True)
            out = {}
            for pol in (vie.VIE_TE, vie.VIE_TM):
                A, R, T = s.absorption(pol=pol)
                out[pol] = (infos[pol], A, R, T)
                lat.append((time.perf_counter() - t0) * 1e3)
            step_s.append(time.perf_counter() - t0)
            results.append({"case": list(case), "A": [out[p][1].tolist() for p in (0, 1)],
                            "R": [out[p][2] for p in (0, 1)], "T": [out[p][3] for p in (0, 1)]})
            stages.append({"case": list(case), "fill_ms": out[0][0]["t_fill_ms"],
                           "factor_ms": out[0][0]["t_factor_ms"], "pair_solve_ms": out[0][0]["t_solve_ms"],
                           "iters": [out[p][0]["iters"] for p in (0, 1)],
                           "converged": [out[p][0]["converged"] for p in (0, 1)]})
            print(f"{name} step {i}: lambda {lam:.0f} theta {th:.0f} phi {ph:.0f}  {json.dumps(stages[-1])}",
                  file=sys.stderr, flush=True)

        print(f"bench: N={N}, {name}, workspace {ws_bytes / 1e9:.1f} GB", file=sys.stderr, flush=True)
        # untimed: pick the launch shapes (autotuner) on the operator of the first case
        first = (warm_cases + timed_cases)[0]
        s.fill(first[0], np.deg2rad(first[1]), np.deg2rad(first[2]), eps_of[first[0]])
        s.factor()
        tuning = s.autotune(reps=3)
        print(f"autotune: {json.dumps(tuning)}", file=sys.stderr, flush=True)
        for i, c in enumerate(warm_cases):
            step(i, c)
        lat.clear(); stages.clear(); fills.clear(); facs.clear(); results.clear(); step_s.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, c in enumerate(timed_cases):
            step(len(warm_cases) + i, c)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mv_ms = s.bench_matvec(10)
        s.close()
        del s
        torch.cuda.empty_cache()
        return {"N": N, "ws_bytes": ws_bytes, "dt": dt, "lat": lat, "stages": stages, "fills": fills, "facs": facs,
                "results": results, "mv_ms": mv_ms, "tuning": tuning, "step_s": step_s, "sym": sym}

    mixed = run_path(vie.VIE_MIXED_FP32, warm, timed)
    sub = timed[:max(0, min(args.fp64_steps, len(timed)))]
    fp64 = run_path(vie.VIE_FP64, [], sub) if sub else None
    N = mixed["N"]
    nsolves = 2 * args.steps

    dA_cases = []
    if fp64:
        for rm, rf in zip(mixed["results"], fp64["results"]):
            d = 0.0
            for p in (0, 1):
                d = max(d, float(np.max(np.abs(np.array(rm["A"][p]) - np.array(rf["A"][p])))),
                        abs(rm["R"][p] - rf["R"][p]), abs(rm["T"][p] - rf["T"][p]))
            dA_cases.append({"case": rm["case"], "dA": d})

    def far_rate(fills):
        flops = sum(f["far_flops"] for f in fills)
        ms = sum(f["t_far_ms"] for f in fills)
        launches = sum(f["far_launches"] for f in fills)
        return flops, ms, launches

    # the far tet-pair fill kernel of the oblique cases (with the symmetric
    # fill: k_tt_far_rev, one lattice sum per unordered pair; normal-incidence
    # cases run k_tt_far and are left out)
    obl = [f for f in mixed["fills"] if f["oblique"]] or mixed["fills"]
    far_kernel = "k_tt_far_rev" if mixed["sym"] and obl[0]["oblique"] else "k_tt_far"
    far_flops, far_ms, far_launches = far_rate(obl)
    far_tflops = far_flops / (far_ms * 1e-3) / 1e12
    mv32_bytes = 8.0 * N * N + 32.0 * N
    mv64_bytes = 16.0 * N * N + 32.0 * N
    mv32_gbs = mv32_bytes / (mixed["mv_ms"] * 1e-3) / 1e9
    counters = profile_counters(FAR_PROFILE, FAR_SOURCES) if far_kernel == "k_tt_far_rev" else None
    avg_ms = far_ms / far_launches
    far_roofline = {"bound": "alu", "kernel": far_kernel, "achieved": far_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": far_tflops / FP64_VECTOR_PEAK_TFLOPS,
                    "traffic": counters["traffic"] if counters else None,
                    "traffic_unit": "bytes per launch", "launches": far_launches,
                    "flops_per_launch": far_flops / far_launches, "avg_launch_ms": avg_ms}
    if counters and counters["hw_flops"]:
        # hardware-counted FP64 FLOPs (rocprofv3 VALU counters) over the same launch time
        far_roofline["achieved_hw"] = counters["hw_flops"] / (avg_ms * 1e-3) / 1e12
        far_roofline["frac_hw"] = far_roofline["achieved_hw"] / FP64_VECTOR_PEAK_TFLOPS
    # dominant kernel of a step (largest device time): the block factor's
    # K = 128 trailing update on the FP32 matrix cores, timed live by the
    # library (HIP events around each launch on the context's stream)
    upd_flops = sum(f["update_flops"] for f in mixed["facs"])
    upd_ms = sum(f["t_update_ms"] for f in mixed["facs"])
    upd_n = sum(f["update_launches"] for f in mixed["facs"])
    upd_tflops = upd_flops / (upd_ms * 1e-3) / 1e12
    lu_counters = profile_counters(LU_PROFILE, LU_SOURCES)
    roofline = {"bound": "mfma", "kernel": "k_lu_gemm2_c", "achieved": upd_tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": upd_tflops / FP32_MFMA_PEAK_TFLOPS,
                "traffic": lu_counters["traffic"] if lu_counters else None,
                "traffic_unit": "bytes per launch", "launches": upd_n, "flops_per_launch": upd_flops / upd_n,
                "avg_launch_ms": upd_ms / upd_n,
                "step_share": upd_ms / sum(st["fill_ms"] + st["factor_ms"] + st["pair_solve_ms"]
                                           for st in mixed["stages"]),
                "factor_ms": [f["t_factor_ms"] for f in mixed["facs"]]}
    res = {
        "metric": "solves/s (mixed FP32/FP64 path) vs FP64 path at dA<=1e-4; p50/p99 latency; fill GFLOP/s; "
                  "matvec GB/s",
        "value": nsolves / mixed["dt"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["dt"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 far-Z storage, f64 arithmetic",
        "data": "synthetic",
        "config": {"workload": "precision form of the plasmonic OSC cell: 200x200 nm, Ag sphere r=20 nm, "
                               "3.33/20 nm mesh, N=%d; theta 0-80 deg x phi {0,45} x lambda {450,550,650} nm "
                               "(99 incidences, stride %d), TE+TM per step" % (N, STRIDE),
                   "unknowns": N, "tets": int(mesh.nt), "restart": args.restart, "tol": args.tol,
                   "solve": "pair", "graph_steps": args.graph_steps, "sym_fill": mixed["sym"],
                   "timed_cases": [list(c) for c in timed], "workspace_gb": mixed["ws_bytes"] / 1e9},
        "step_latency_ms": {"p50": float(np.percentile(mixed["lat"], 50)),
                            "p99": float(np.percentile(mixed["lat"], 99))},
        "fill_gflops": far_tflops * 1e3,
        "matvec_gbs": mv32_gbs,
        "matvec_frac_hbm": mv32_gbs / HBM_PEAK_GBS,
        "stages": mixed["stages"],
        "tuning": {"mixed": mixed["tuning"]},
        "fill_stats": mixed["fills"][-1],
        "roofline": roofline,
        "far_fill_roofline": far_roofline,
    }
    if fp64:
        ff, fms, _ = far_rate(fp64["fills"])
        n_sub = len(sub)
        res["fp64"] = {"cases": n_sub, "value": 2 * n_sub / fp64["dt"],
                       "mixed_value_same_cases": 2 * n_sub / sum(mixed["step_s"][:n_sub]),
                       "ms_per_step": fp64["dt"] / n_sub * 1e3, "fill_gflops": ff / (fms * 1e-3) / 1e9,
                       "matvec_gbs": mv64_bytes / (fp64["mv_ms"] * 1e-3) / 1e9,
                       "workspace_gb": fp64["ws_bytes"] / 1e9, "sym_fill": fp64["sym"], "dtype": "f64",
                       "stages": fp64["stages"]}
        res["fp64"]["matvec_frac_hbm"] = res["fp64"]["matvec_gbs"] / HBM_PEAK_GBS
        u_fl = sum(f["update_flops"] for f in fp64["facs"])
        u_ms = sum(f["t_update_ms"] for f in fp64["facs"])
        if u_ms > 0:   # k_lu_gemm2_z on the FP64 matrix cores (peak 78.6 TFLOP/s)
            res["fp64"]["lu_update_tflops"] = u_fl / (u_ms * 1e-3) / 1e12
            res["fp64"]["lu_update_frac_mfma"] = res["fp64"]["lu_update_tflops"] / 78.6
        res["tuning"]["fp64"] = fp64["tuning"]
        res["dA_per_case"] = dA_cases
        res["dA_mixed_vs_fp64"] = max(d["dA"] for d in dA_cases)
    if not args.no_grid:
        print("grid operator (uniform cell)...", file=sys.stderr, flush=True)
        res["grid_operator"] = grid_operator()
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle sample)...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(mesh, timed[0] if timed else all_cases[0])
    print(json.dumps(res))


if __name__ == "__main__":
    main()
