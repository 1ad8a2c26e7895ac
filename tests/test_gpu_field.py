"""Field sampling (vie_sample_field): E/E0 at points inside the structure, the
field maps behind the absorption profiles of Sec. 3 (Fig. 5).

Points on a plane through the particle (off the mesh planes, some above and
below the structure) and random points in the cell.  Against the oracle's
field_at at the library's own solution: the same holding tetrahedron for
every point (exact) and E to 1e-12 of max|E|.  Against the oracle's LU
solution (the whole path): 1e-8 (FP64, tol 1e-12) and 1e-4 (mixed)."""
import numpy as np
import pytest

import gpu_cases as G
from oracle import topology as OT
from oracle import vie as OV

pytestmark = pytest.mark.gpu


def sample_points(m, seed):
    xs = np.linspace(0.05 * m.a, 0.95 * m.a, 24)
    zs = np.linspace(-3.0, m.grid[2][-1] + 3.0, 14)
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    plane = np.stack([X.ravel(), np.full(X.size, 0.451 * m.b), Z.ravel()], axis=1)
    rng = np.random.default_rng(seed)
    rnd = rng.uniform([0, 0, 0], [m.a, m.b, m.grid[2][-1]], size=(150, 3))
    return np.concatenate([plane, rnd])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["osc_small", "osc_rect"])
def test_field_matches_oracle(precision, case):
    from paper_1809_05334_amd import vie
    m = getattr(G, case)()
    lam, th, ph = 560.0, 0.45, 0.7
    eps = G.eps_for(m, lam)
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    topo = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    wave = OV.make_wave(lam, th, ph)
    Zo = OV.assemble(topo, wave, eps)
    pts = sample_points(m, 3)
    s = vie.Solver(0)
    s.upload_mesh(m)
    s.bind(prec, 60)
    s.fill(lam, th, ph, eps)
    s.factor()
    s.solve_pair(tol=1e-12 if precision == "fp64" else 1e-9, max_iter=600, restart=60)
    print(f"field {case} {precision}: N={topo.N}, {len(pts)} points", flush=True)
    for pol in (0, 1):
        e, tet = s.sample_field(pts, pol)
        x = s.read_solution(pol)
        Eo, to = OV.field_at(topo, wave, eps, x, pts)
        assert np.array_equal(tet, to)
        assert np.any(tet < 0) and np.sum(tet >= 0) > len(pts) // 2
        mx = np.abs(Eo).max()
        assert np.max(np.abs(e - Eo)) <= 1e-12 * mx, np.max(np.abs(e - Eo)) / mx
        assert np.all(e[tet < 0] == 0)
        xo = OV.solve_lu(Zo, OV.rhs(topo, wave, pol))
        Ex, _ = OV.field_at(topo, wave, eps, xo, pts)
        bar = 1e-8 if precision == "fp64" else 1e-4
        assert np.max(np.abs(e - Ex)) <= bar * np.abs(Ex).max(), (pol, np.max(np.abs(e - Ex)) / np.abs(Ex).max())
    e0, t0 = s.sample_field(np.zeros((0, 3)))
    assert e0.shape == (0, 3) and t0.shape == (0,)
    s.close()


def test_field_needs_a_solve():
    from paper_1809_05334_amd import vie
    m = G.osc_small()
    s = vie.Solver(0)
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 20)
    s.fill(520.0, 0.0, 0.0, G.eps_for(m, 520.0))
    with pytest.raises(vie.VieError) as e:
        s.sample_field(np.array([[10.0, 10.0, 10.0]]))
    assert e.value.code == vie.VIE_ESTATE
    s.close()
