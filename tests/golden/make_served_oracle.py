"""Writes served_oracle.json: oracle absorptance per domain, R and T for a few
cells of the batched/served workload (the batch-cell generator: Drude-Ag sphere in
a spacer layer over an active layer, uneven N, oblique incidence, random
polarisation), one of them at an incidence where a non-specular Floquet
order propagates (a (1 + sin theta) > lambda).

Only the oracle computes here (dense Z, LU solve, Eq. 7, R/T over the
propagating orders, Sec. 2-3); the inputs come from the seeded workload
generator.  Run from the repository root:

    python tests/golden/make_served_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import topology as OT  # noqa: E402
from oracle import vie as OV  # noqa: E402
from paper_1809_05334_amd import workloads as W  # noqa: E402

SEED = 11
PICK = [5, 1, 3, 21, 9]        # cells of batch_cells(40, seed=11, n_lo=1000, n_hi=2500), N 1,250-2,450
DIFFRACT = 9                   # this one is re-aimed so that an order (p, q) != (0, 0) propagates


def requests():
    cells = W.batch_cells(40, seed=SEED, n_lo=1000, n_hi=2500)
    out = []
    for i in PICK:
        c = dict(cells[i])
        lam, th, ph, pol = c["lambda"], c["theta"], c["phi"], c["pol"]
        if i == DIFFRACT:
            th, ph = np.deg2rad(45.0), np.deg2rad(10.0)
            lam = None
            for cand in np.arange(400.0, c["a"] * (1 + np.sin(th)), 1.0):
                if W.wood_margin(c["a"], c["a"], cand, th, ph) >= 0.05:
                    lam = float(cand)
                    break
            assert lam is not None
        cell = {k: c[k] for k in ("a", "t_active", "t_spacer", "radius", "h_fine", "h_coarse", "n_est")}
        out.append({"rid": len(out), "arrival": 0.0, "cell": cell, "lambda": float(lam), "theta": float(th),
                    "phi": float(ph), "pol": int(pol)})
    return out


def main():
    reqs = requests()
    rows = []
    for r in reqs:
        t0 = time.time()
        mesh = W.cell_mesh(r["cell"])
        topo = OT.build(mesh.verts, mesh.tets, mesh.tet_domain, mesh.ndom, mesh.a, mesh.b)
        eps = W.osc_eps(mesh, r["lambda"])
        wave = OV.make_wave(r["lambda"], r["theta"], r["phi"])
        Z = OV.assemble(topo, wave, eps)
        b = OV.rhs(topo, wave, r["pol"])
        x = OV.solve_lu(Z, b)
        A = OV.absorptance(topo, wave, eps, x)
        R, T = OV.reflect_transmit(topo, wave, eps, x, r["pol"])
        k0 = wave.k0
        prop = [(p, q) for p in range(-4, 5) for q in range(-4, 5)
                if (wave.kx + 2 * np.pi * p / topo.a) ** 2 + (wave.ky + 2 * np.pi * q / topo.b) ** 2 < k0 * k0]
        rows.append(dict(r, N=int(topo.N), A=[float(v) for v in A], R=float(R), T=float(T),
                         orders=[list(o) for o in prop]))
        print(f"rid {r['rid']}: N={topo.N} orders={prop} A={A} R={R:.6f} T={T:.6f} ({time.time() - t0:.0f} s)",
              flush=True)
    with open(os.path.join(HERE, "served_oracle.json"), "w") as f:
        json.dump({"source": "oracle LU solve (tests/golden/make_served_oracle.py)",
                   "generator": {"batch_cells": {"n": 40, "seed": SEED, "n_lo": 1000, "n_hi": 2500},
                                 "pick": PICK, "diffracting": DIFFRACT},
                   "requests": rows}, f, indent=1)


if __name__ == "__main__":
    main()
