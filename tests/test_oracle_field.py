"""Pins of the oracle's field sampling (field_at, locate_points), the field
maps behind the absorption profiles of Sec. 3 (Fig. 5).

  * SWG normal continuity (Sec. 2.1): every basis function has a unit normal
    component on its face, so for ANY coefficient vector x the normal
    component of D~ at a face point equals x_f seen from both tetrahedra.
    On a wall-paired face the second tetrahedron sits one lattice vector
    away, and the Bloch condition of the periodic problem (Sec. 2.2, Eq. 3:
    every field picks up exp(-j kt.rho) under a shift rho) links the two.
    A wrong coefficient (area over volume, the 1/3, the sign of T-, the
    Bloch phase of a shifted half) fails it.
  * Eq. 7 by sampling: k0 Im(1/eps) |D~|^2 integrated over each tetrahedron
    by the 4-point rule (exact for the quadratic |D~|^2) at points that
    field_at locates and evaluates equals absorptance_per_tet, which
    integrates the same quadratic form in closed form.
  * Points above the structure lie in no tetrahedron."""
import numpy as np

from oracle import quadrature as Q
from oracle import topology as T
from oracle import vie as V
from paper_1809_05334_amd import workloads as W


def cell():
    xs = np.array([0.0, 12.0, 20.0, 28.0, 40.0])
    ys = np.array([0.0, 15.0, 30.0])
    zs = np.array([0.0, 20.0, 30.0, 40.0])
    verts, tets = W.brick_grid_mesh(xs, ys, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 20.0, W.DOM_ACTIVE, W.DOM_SPACER).astype(np.int32)
    dom[np.sum((c - [20.0, 15.0, 30.0]) ** 2, 1) <= 8.0 ** 2] = W.DOM_METAL
    m = W.Mesh(verts, tets, dom, 3, 40.0, 30.0, (xs, ys, zs))
    return m, T.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)


def unit_normal_out(face3, free):
    n = np.cross(face3[1] - face3[0], face3[2] - face3[0])
    n /= np.linalg.norm(n)
    return n if np.dot(face3[0] - free, n) > 0 else -n


def test_normal_component_is_the_coefficient_on_both_sides():
    m, topo = cell()
    wave = V.make_wave(520.0, 0.5, 0.3)
    rng = np.random.default_rng(11)
    x = rng.normal(size=topo.N) + 1j * rng.normal(size=topo.N)
    c = V.tet_field_coeffs(topo, wave, x)
    kt = np.array([wave.kx, wave.ky, 0.0])
    walls = 0
    for f in range(topo.N):
        tp = topo.tplus[f]
        kp = int(np.flatnonzero(topo.t2f[tp] == f)[0])
        v4 = topo.verts[topo.tets[tp]]
        face = np.delete(v4, kp, axis=0)
        rf = face.mean(axis=0)
        n = unit_normal_out(face, v4[kp])
        Dp = sum(c[tp, k] * (rf - v4[k]) for k in range(4))
        assert abs(np.dot(Dp, n) - x[f]) <= 1e-12 * abs(x[f])
        tm = topo.tminus[f]
        if tm < 0:
            continue
        km = int(np.flatnonzero((topo.t2f[tm] == f) & (topo.t2s[tm] == -1))[0])
        w4 = topo.verts[topo.tets[tm]]
        delta = rf - np.delete(w4, km, axis=0).mean(axis=0)   # lattice vector (0 inside the cell)
        walls += np.linalg.norm(delta) > 1e-9
        Dm = sum(c[tm, k] * (rf - delta - w4[k]) for k in range(4)) * np.exp(-1j * np.dot(kt, delta))
        assert abs(np.dot(Dm, n) - x[f]) <= 1e-12 * abs(x[f])
    assert walls > 0


def test_sampled_absorption_matches_closed_form():
    m, topo = cell()
    lam = 520.0
    eps = W.osc_eps(m, lam)
    wave = V.make_wave(lam, 0.4, 1.1)
    rng = np.random.default_rng(12)
    x = rng.normal(size=topo.N) + 1j * rng.normal(size=topo.N)
    bary, w = Q.tet_deg2()
    pts = np.einsum("qk,tkd->tqd", bary, topo.verts[topo.tets]).reshape(-1, 3)
    E, tet = V.field_at(topo, wave, eps, x, pts)
    nt = len(topo.tets)
    assert np.array_equal(tet, np.repeat(np.arange(nt), len(w)))
    epsi = V.internal_eps(eps)
    D2 = np.sum(np.abs(E) ** 2, axis=1).reshape(nt, len(w)) * np.abs(epsi)[:, None] ** 2
    per = (-epsi.imag) / np.abs(epsi) ** 2 * topo.vol * (D2 @ w)
    per *= wave.k0 / (np.cos(wave.theta) * topo.a * topo.b)
    ref = V.absorptance_per_tet(topo, wave, eps, x)
    assert np.max(np.abs(per - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_points_outside_the_structure():
    m, topo = cell()
    eps = W.osc_eps(m, 520.0)
    wave = V.make_wave(520.0, 0.0, 0.0)
    x = np.ones(topo.N, complex)
    E, tet = V.field_at(topo, wave, eps, x, np.array([[5.0, 5.0, 41.0], [5.0, 5.0, -0.5], [20.0, 15.0, 10.0]]))
    assert tet[0] == -1 and tet[1] == -1 and tet[2] >= 0
    assert np.all(E[:2] == 0) and np.any(E[2] != 0)
