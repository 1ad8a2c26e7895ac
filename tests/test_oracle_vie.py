"""Whole-method pins for the oracle (Sec. 2-3): the homogeneous periodic slab
against the transfer-matrix closed form at several angles and both
polarisations, convergence under mesh refinement, energy balance, a lossless
slab, exact mirror symmetry of a three-domain cell, the block-preconditioned
GMRES against dense LU, and symmetry/reciprocity of far-field entries."""
import numpy as np
import pytest

from oracle import fresnel as F
from oracle import topology as T
from oracle import vie as V
from paper_1809_05334_amd import workloads as W


def build(mesh):
    return T.build(mesh.verts, mesh.tets, mesh.tet_domain, mesh.ndom, mesh.a, mesh.b)


def solve_case(topo, eps, lam, th, ph, pol):
    wave = V.make_wave(lam, th, ph)
    Z = V.assemble(topo, wave, eps)
    b = V.rhs(topo, wave, pol)
    x = V.solve_lu(Z, b)
    A = V.absorptance(topo, wave, eps, x)
    R, Tt = V.reflect_transmit(topo, wave, eps, x, pol)
    return Z, b, x, A, R, Tt


@pytest.fixture(scope="module")
def slab25():
    m = W.slab_mesh(a=50.0, b=50.0, thickness=50.0, nx=2, ny=2, nz=2)
    return m, build(m)


@pytest.mark.parametrize("th,pol", [(0, 0), (30, 0), (30, 1), (60, 0), (60, 1)])
def test_slab_vs_transfer_matrix(slab25, th, pol):
    m, topo = slab25
    eps = W.slab_eps(m)
    _, _, _, A, R, Tt = solve_case(topo, eps, 600.0, np.deg2rad(th), 0.3 if th else 0.0, pol)
    Rf, Tf, Af = F.slab_rta(W.EPS_SLAB, 50.0, 600.0, np.deg2rad(th), pol)
    assert abs(A[0] - Af) < 3e-3 and abs(R - Rf) < 3e-3 and abs(Tt - Tf) < 3e-3, (A, R, Tt, Af, Rf, Tf)
    assert abs(A[0] + R + Tt - 1.0) < 5e-6
    assert A[0] > 0


def test_refinement_reduces_error(slab25):
    m, topo = slab25
    errs = []
    fine = W.slab_mesh(a=50.0, b=50.0, thickness=50.0, nx=4, ny=4, nz=4)
    Rf, Tf, Af = F.slab_rta(W.EPS_SLAB, 50.0, 600.0, 0.0, 0)
    for mesh in (m, fine):
        tp = topo if mesh is m else build(mesh)
        _, _, _, A, R, Tt = solve_case(tp, W.slab_eps(mesh), 600.0, 0.0, 0.0, 0)
        errs.append(np.array([A[0] - Af, R - Rf, Tt - Tf]))
    # second-order convergence: halving h cuts the error ~4x
    assert np.all(np.abs(errs[1]) < np.abs(errs[0]) / 3.0), errs


def test_lossless_slab(slab25):
    m, topo = slab25
    eps = np.full(m.nt, 3.6 + 0j)
    _, _, _, A, R, Tt = solve_case(topo, eps, 600.0, 0.0, 0.0, 0)
    Rf, Tf, _ = F.slab_rta(3.6, 50.0, 600.0, 0.0, 0)
    assert A[0] == 0.0
    assert abs(R + Tt - 1.0) < 5e-6
    assert abs(R - Rf) < 3e-3


def test_gmres_single_domain_one_iteration(slab25):
    m, topo = slab25
    eps = W.slab_eps(m)
    wave = V.make_wave(600.0, 0.4, 0.2)
    Z = V.assemble(topo, wave, eps)
    b = V.rhs(topo, wave, 1)
    x, it, hist, ok = V.gmres_right_block(Z, b, topo.domain_ranges, tol=1e-12)
    assert ok and it == 1
    assert np.linalg.norm(x - V.solve_lu(Z, b)) < 1e-12 * np.linalg.norm(x)


def test_entries_subblock_matches_full(slab25):
    m, topo = slab25
    eps = W.slab_eps(m)
    wave = V.make_wave(550.0, 0.5, 0.7)
    Z = V.assemble(topo, wave, eps)
    rng = np.random.default_rng(0)
    rows = rng.choice(topo.N, 9, replace=False)
    cols = rng.choice(topo.N, 13, replace=False)
    Zs = V.assemble(topo, wave, eps, rows=rows, cols=cols)
    assert np.max(np.abs(Zs - Z[np.ix_(rows, cols)])) < 1e-13 * np.abs(Z).max()


def far_only_pairs(topo):
    """(m, n) whose tetrahedra never touch under any image and that carry no
    face element (interior full SWGs)."""
    full = np.nonzero(topo.tminus >= 0)[0]
    tets_of = {n: (topo.tplus[n], topo.tminus[n]) for n in full}
    out = []
    for m in full:
        for n in full:
            if m >= n:
                continue
            if all(not T.near_images(topo.canon, topo.voff, topo.tets[t], topo.tets[s])
                   for t in tets_of[m] for s in tets_of[n]):
                out.append((m, n))
    return np.array(out)


def test_far_entries_symmetric_and_reciprocal():
    m = W.slab_mesh(a=60.0, b=60.0, thickness=20.0, nx=3, ny=3, nz=1)
    topo = build(m)
    eps = W.slab_eps(m)
    pairs = far_only_pairs(topo)
    assert len(pairs) > 100
    Z0 = V.assemble(topo, V.make_wave(600.0, 0.0, 0.0), eps)
    r, c = pairs[:, 0], pairs[:, 1]
    scale = np.abs(Z0[r, c]).max()
    assert np.max(np.abs(Z0[r, c] - Z0[c, r])) < 1e-12 * scale
    wp = V.make_wave(600.0, 0.6, 0.4)
    Zp = V.assemble(topo, wp, eps)
    wm = V.make_wave(600.0, -0.6, 0.4)            # kt -> -kt
    Zm = V.assemble(topo, wm, eps)
    assert np.max(np.abs(Zp[r, c] - Zm[c, r])) < 1e-12 * scale
    # and the Bloch phase matters (guards against a dropped phase)
    assert np.max(np.abs(Zp[r, c] - Zp[c, r])) > 1e-6 * scale


@pytest.fixture(scope="module")
def small_osc():
    xs = np.array([0.0, 12.0, 20.0, 28.0, 40.0])
    zs = np.array([0.0, 20.0, 30.0, 40.0])
    verts, tets = W.brick_grid_mesh(xs, xs, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 20.0, W.DOM_ACTIVE, W.DOM_SPACER).astype(np.int32)
    dom[np.sum((c - [20.0, 20.0, 30.0]) ** 2, 1) <= 8.0 ** 2] = W.DOM_METAL
    m = W.Mesh(verts, tets, dom, 3, 40.0, 40.0, (xs, xs, zs))
    return m, build(m)


def test_three_domain_cell(small_osc):
    m, topo = small_osc
    assert set(np.unique(m.tet_domain)) == {0, 1, 2}
    eps = W.osc_eps(m, 520.0)
    wave = V.make_wave(520.0, 0.0, 0.0)
    Z = V.assemble(topo, wave, eps)
    res = {}
    for pol in (0, 1):
        b = V.rhs(topo, wave, pol)
        x = V.solve_lu(Z, b)
        xg, it, hist, ok = V.gmres_right_block(Z, b, topo.domain_ranges, tol=1e-12, restart=60)
        assert ok
        assert np.linalg.norm(xg - x) < 1e-9 * np.linalg.norm(x)
        A = V.absorptance(topo, wave, eps, x)
        R, Tt = V.reflect_transmit(topo, wave, eps, x, pol)
        assert np.all(A > 0)
        assert abs(A.sum() + R + Tt - 1) < 2e-2
        res[pol] = (A, R, Tt)
    # the mesh and the cell are invariant under x <-> y: TE (E along y) and
    # TM (E along x) at normal incidence are mirror images
    assert np.max(np.abs(res[0][0] - res[1][0])) < 1e-11
    assert abs(res[0][1] - res[1][1]) < 1e-11 and abs(res[0][2] - res[1][2]) < 1e-11


# ---- GMRES without a preconditioner (blocks = []: M = I), the reference the
# block preconditioner is compared against in Sec. 3 (Figs. 2-3).  Pins that
# hold for any correct GMRES, independent of the oracle's own arithmetic:
# on I + (rank k) the Krylov space closes after k + 1 steps, so GMRES stops
# there with the exact solution; within one cycle the residual estimate never
# grows (minimal residual over nested spaces) and equals the true residual.

def _rank_k_plus_identity(n, k, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    Vh = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
    return np.eye(n) + 0.1 * U @ Vh


@pytest.mark.parametrize("k", [1, 3, 6])
def test_gmres_no_precond_rank_k_closes_in_k_plus_1(k):
    n = 40
    A = _rank_k_plus_identity(n, k, seed=10 + k)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist, ok = V.gmres_right_block(A, b, [], tol=1e-12, restart=50)
    assert ok and it <= k + 1, (it, hist)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) < 1e-10 * np.linalg.norm(xs)


def test_gmres_no_precond_residual_monotone_and_true():
    n = 30
    rng = np.random.default_rng(3)
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist, ok = V.gmres_right_block(A, b, [], tol=1e-11, restart=n)
    assert ok and it <= n
    h = np.array(hist)
    assert np.all(np.diff(h) <= 1e-14 * h[0]), h
    r = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert r <= 1e-11 * 1.01 and abs(r - h[-1]) < 1e-12


def test_block_preconditioner_beats_none_on_multidomain_cell():
    """Sec. 2.3 / Sec. 3: on a three-domain cell with a metal particle the
    block preconditioner needs fewer GMRES iterations than none, and both
    reach the same solution (Eq. 8 difference at the solver tolerance)."""
    xs = np.array([0.0, 12.0, 20.0, 28.0, 40.0])
    zs = np.array([0.0, 20.0, 30.0, 40.0])
    verts, tets = W.brick_grid_mesh(xs, xs, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 20.0, W.DOM_ACTIVE, W.DOM_SPACER).astype(np.int32)
    dom[np.sum((c - [20.0, 20.0, 30.0]) ** 2, 1) <= 8.0 ** 2] = W.DOM_METAL
    m = W.Mesh(verts, tets, dom, 3, 40.0, 40.0, (xs, xs, zs))
    topo = build(m)
    lam = 400.0
    wave = V.make_wave(lam, 0.0, 0.0)
    Z = V.assemble(topo, wave, W.osc_eps(m, lam))
    b = V.rhs(topo, wave, 0)
    xp, ip, _, okp = V.gmres_right_block(Z, b, topo.domain_ranges, tol=1e-10, restart=60, maxit=3000)
    xn, inn, _, okn = V.gmres_right_block(Z, b, [], tol=1e-10, restart=60, maxit=3000)
    assert okp and okn and ip < inn, (ip, inn)
    xs_ = V.solve_lu(Z, b)
    for x in (xp, xn):
        assert np.linalg.norm(x - xs_) < 1e-7 * np.linalg.norm(xs_)


# ---- per-tetrahedron absorption (Eq. 7 term by term; the maps of Fig. 5).
# Pins: the terms of each domain add up to absorptance() (itself pinned on the
# Fresnel slab and the energy balance); a lossless domain absorbs exactly
# nothing; a passive lossy one nowhere absorbs a negative amount.

def test_absorptance_per_tet_sums_and_signs():
    xs = np.array([0.0, 12.0, 20.0, 28.0, 40.0])
    zs = np.array([0.0, 20.0, 30.0, 40.0])
    verts, tets = W.brick_grid_mesh(xs, xs, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 20.0, W.DOM_ACTIVE, W.DOM_SPACER).astype(np.int32)
    dom[np.sum((c - [20.0, 20.0, 30.0]) ** 2, 1) <= 8.0 ** 2] = W.DOM_METAL
    m = W.Mesh(verts, tets, dom, 3, 40.0, 40.0, (xs, xs, zs))
    topo = build(m)
    lam = 450.0
    eps = np.array(W.osc_eps(m, lam), complex)
    eps[dom == W.DOM_SPACER] = eps[dom == W.DOM_SPACER].real   # a lossless domain
    wave = V.make_wave(lam, 0.2, 0.3)
    Z = V.assemble(topo, wave, eps)
    x = V.solve_lu(Z, V.rhs(topo, wave, 1))
    per = V.absorptance_per_tet(topo, wave, eps, x)
    A = V.absorptance(topo, wave, eps, x)
    for d in range(m.ndom):
        assert abs(per[dom == d].sum() - A[d]) <= 1e-13 * max(abs(A).max(), 1e-30), d
    assert np.all(per[dom == W.DOM_SPACER] == 0.0)
    assert np.all(per[dom != W.DOM_SPACER] >= 0.0) and per.max() > 0


# ---- two-layer stack: the interface between two materials (surface charge
# sigma = kappa(T+) - kappa(T-) on interior faces) and the absorptance per
# domain, against the multilayer transfer matrix (closed form).

@pytest.mark.parametrize("th,pol", [(0, 0), (30, 0), (30, 1), (60, 1)])
def test_multilayer_one_layer_is_the_airy_formula(th, pol):
    e = 3.6 + 0.6j
    R, T_, A = F.multilayer_rta([e], [50.0], 600.0, np.deg2rad(th), pol)
    Rf, Tf, Af = F.slab_rta(e, 50.0, 600.0, np.deg2rad(th), pol)
    assert abs(R - Rf) < 1e-13 and abs(T_ - Tf) < 1e-13 and abs(A[0] - Af) < 1e-13


def test_multilayer_split_layer_and_energy():
    e1, e2 = 3.6 + 0.6j, 1.8 + 0.3j
    R, T_, A = F.multilayer_rta([e1], [50.0], 550.0, 0.5, 1)
    R2, T2, A2 = F.multilayer_rta([e1, e1], [20.0, 30.0], 550.0, 0.5, 1)
    assert abs(R - R2) < 1e-13 and abs(T_ - T2) < 1e-13 and abs(A[0] - sum(A2)) < 1e-13
    R3, T3, A3 = F.multilayer_rta([e1, 2.25, e2], [20.0, 15.0, 25.0], 480.0, 0.3, 0)
    assert abs(R3 + T3 + sum(A3) - 1.0) < 1e-13
    assert abs(A3[1]) < 1e-13 and A3[0] > 0 and A3[2] > 0   # the lossless middle layer absorbs nothing


def two_layer_slab(nxy, nz):
    m = W.slab_mesh(a=50.0, b=50.0, thickness=50.0, nx=nxy, ny=nxy, nz=nz)
    c = W.centroids(m.verts, m.tets)
    dom = np.where(c[:, 2] >= 25.0, 0, 1).astype(np.int32)   # the wave meets domain 0 (top) first
    return W.Mesh(m.verts, m.tets, dom, 2, 50.0, 50.0, m.grid)


def _two_layer_errors(nxy, nz, th, pol):
    e1, e2 = 3.6 + 0.6j, 1.8 + 0.3j
    m = two_layer_slab(nxy, nz)
    topo = build(m)
    eps = np.where(m.tet_domain == 0, e1, e2).astype(complex)
    wave = V.make_wave(600.0, np.deg2rad(th), 0.3 if th else 0.0)
    x = V.solve_lu(V.assemble(topo, wave, eps), V.rhs(topo, wave, pol))
    A = V.absorptance(topo, wave, eps, x)
    R, T_ = V.reflect_transmit(topo, wave, eps, x, pol)
    Rf, Tf, Af = F.multilayer_rta([e1, e2], [25.0, 25.0], 600.0, np.deg2rad(th), pol)
    return np.abs(np.array([A[0] - Af[0], A[1] - Af[1], R - Rf, T_ - Tf]))


@pytest.mark.parametrize("th,pol", [(0, 0), (30, 0), (30, 1)])
def test_two_layer_stack_vs_multilayer_transfer_matrix(th, pol):
    err = _two_layer_errors(2, 4, th, pol)   # N = 200
    assert np.all(err < 1e-3), err


def test_two_layer_stack_refinement():
    coarse, fine = _two_layer_errors(2, 4, 0, 0), _two_layer_errors(3, 6, 0, 0)
    # second order: h / 1.5 cuts the error about 2.25x
    assert fine.max() < coarse.max() / 1.7, (coarse, fine)
