"""The fused batch (vie_batch_*): many cells filled, factored and solved in
shared launches, against each cell solved alone through the single-context
entry points, and the captured-graph Arnoldi step against plain launches.

Per cell the fused kernels do the arithmetic of the single-context ones; the
reductions of the Gram-Schmidt sums run over fewer blocks for small cells, so
the two paths agree to the solve's tolerance rather than bit for bit: A, R,
T within 1e-9 at tol 1e-12, the same convergence.  Graph replays and plain
launches of the fused step give identical bits.  Cells of uneven size stop
at different iterations; a cell at oblique incidence, one at normal
incidence and one with a propagating non-specular order are mixed."""
import numpy as np
import pytest

import gpu_cases as G
from paper_1809_05334_amd import workloads as W

pytestmark = pytest.mark.gpu


def cells():
    out = []
    for m, lam, th, ph, pol in ((G.osc_small(), 520.0, 0.5, 0.3, 0), (G.osc_rect(), 610.0, 0.3, 1.1, 1),
                                (G.slab_small(), 600.0, 0.0, 0.0, 1), (G.osc_small(), 450.0, 0.9, 0.2, 1)):
        out.append((m, G.eps_for(m, lam), lam, th, ph, pol))
    # a cell where the (-1, 0) order propagates
    xs, ys, zs = np.linspace(0, 300.0, 4), np.linspace(0, 240.0, 4), np.array([0.0, 30.0, 60.0])
    verts, tets = W.brick_grid_mesh(xs, ys, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 30.0, 1, 0).astype(np.int32)
    m = W.Mesh(verts, tets, dom, 2, 300.0, 240.0, (xs, ys, zs))
    out.append((m, np.array([4.0 + 0.3j, 2.3 + 0.05j])[dom], 500.0, np.deg2rad(55.0), np.deg2rad(20.0), 0))
    return out


def run_alone(vie, case, prec, tol):
    m, eps, lam, th, ph, pol = case
    s = vie.Solver(0)
    s.upload_mesh(m)
    s.bind(prec, 60)
    s.fill(lam, th, ph, eps)
    s.factor()
    info = s.solve(pol, tol=tol, max_iter=600, restart=60)
    A, R, T = s.absorption()
    x = s.read_solution()
    s.close()
    return info, A, R, T, x


def run_fused(vie, cases, prec, tol, graph, sym=False):
    solvers = []
    for (m, eps, lam, th, ph, pol) in cases:
        s = vie.Solver(0)
        s.upload_mesh(m)
        if sym:
            s.set_option(vie.VIE_OPT_SYM_FILL, 1)
        s.bind(prec, 60)
        solvers.append(s)
    b = vie.Batch(solvers, graph=graph)
    b.fill([c[2] for c in cases], [c[3] for c in cases], [c[4] for c in cases], [c[1] for c in cases])
    b.factor()
    infos = b.solve([c[5] for c in cases], tol=tol, max_iter=600, restart=60)
    out = []
    for s, inf in zip(solvers, infos):
        A, R, T = s.absorption()
        out.append((inf, A, R, T, s.read_solution()))
    b.close()
    for s in solvers:
        s.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_batch_matches_cells_alone(precision):
    from paper_1809_05334_amd import vie
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    cases = cells()
    print(f"fused batch {precision}: {len(cases)} cells", flush=True)
    fused = run_fused(vie, cases, prec, 1e-12, graph=True)
    for k, case in enumerate(cases):
        info, A, R, T, x = run_alone(vie, case, prec, 1e-12)
        fi, fA, fR, fT, fx = fused[k]
        print(f"  cell {k}: N={len(x)} iters alone {info['iters']} fused {fi['iters']}", flush=True)
        assert info["converged"] and fi["converged"]
        assert abs(fi["iters"] - info["iters"]) <= 1
        assert np.max(np.abs(fA - A)) <= 1e-9 and abs(fR - R) <= 1e-9 and abs(fT - T) <= 1e-9
        assert np.linalg.norm(fx - x) <= 1e-9 * np.linalg.norm(x)


def test_fused_graph_replay_equals_plain_launches():
    from paper_1809_05334_amd import vie
    cases = cells()
    g = run_fused(vie, cases, vie.VIE_MIXED_FP32, 1e-10, graph=True)
    p = run_fused(vie, cases, vie.VIE_MIXED_FP32, 1e-10, graph=False)
    for (gi, gA, gR, gT, gx), (pi, pA, pR, pT, px) in zip(g, p):
        assert gi["iters"] == pi["iters"]
        assert np.array_equal(gA, pA) and gR == pR and gT == pT and np.array_equal(gx, px)


def test_fused_symmetric_fill():
    from paper_1809_05334_amd import vie
    cases = cells()
    plain = run_fused(vie, cases, vie.VIE_FP64, 1e-12, graph=True)
    sym = run_fused(vie, cases, vie.VIE_FP64, 1e-12, graph=True, sym=True)
    for (_, A, R, T, _), (_, sA, sR, sT, _) in zip(plain, sym):
        assert np.max(np.abs(sA - A)) <= 1e-9 and abs(sR - R) <= 1e-9 and abs(sT - T) <= 1e-9
