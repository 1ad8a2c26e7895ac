"""Structured-grid far operator (VIE_GRID_FP64) on uniform Kuhn brick grids.

The operator never stores Z: the near part is the FP64 sparse part of the
touching pairs and the far part is applied by FFT over the quadrature-point
sublattices of the grid.  It is the same Z as the dense path (Sec. 2.1, Eq. 2
with the lattice sums of Sec. 2.2, Eqs. 3-4), so:
  * Z x through the grid operator equals the oracle's Z x (oracle Z assembled
    here) and the dense FP64 path's Z x on the same seeded x, at normal and
    oblique incidence, with one domain and with interface surface charges
    (several domains) and half-SWG boundary faces, on the smallest grid (two
    bricks per period, one layer), on a diffracting cell and on unequal x and
    y; the bar 1e-10 relative in the 2-norm (FFT and rounding-order
    differences only);
  * a solve with M = I or M = diag(Z) gives the dense path's iterations,
    absorptance, R and T;
  * meshes that are not uniform Kuhn grids, and the calls the operator does
    not offer, are refused with VIE_EINVAL.
"""
import ctypes

import numpy as np
import pytest

from oracle import topology as OT
from oracle import vie as OV
from paper_1809_05334_amd import workloads as W

from gpu_cases import osc_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


def layered_grid(nx=4, ny=3, nz=4, a=80.0, b=60.0, c=60.0):
    """Uniform grid, three domains: two z layers and a 2 x 1 x 1-brick block
    of a third material in the upper one (interfaces in x, y and z)."""
    xs = np.linspace(0.0, a, nx + 1); ys = np.linspace(0.0, b, ny + 1); zs = np.linspace(0.0, c, nz + 1)
    verts, tets = W.brick_grid_mesh(xs, ys, zs)
    cen = W.centroids(verts, tets)
    dom = (cen[:, 2] > c / 2).astype(np.int32)
    blk = (cen[:, 0] > a / 4) & (cen[:, 0] < 3 * a / 4) & (cen[:, 1] < b / ny) & (cen[:, 2] > c / 2) & (cen[:, 2] < 3 * c / 4)
    dom[blk] = 2
    return W.Mesh(verts, tets, dom, 3, a, b, (xs, ys, zs))


def eps_of(m):
    return np.array([2.25 + 0.1j, 3.1 + 0.4j, -4.0 + 1.5j])[m.tet_domain]


def solver(vie, m, precision, restart=60):
    s = vie.Solver()
    N = s.upload_mesh(m)
    s.bind(precision, restart)
    return s, N


def seeded_x(N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N) + 1j * rng.standard_normal(N)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("lam,th,ph", [(600.0, 0.0, 0.0), (600.0, 0.5, 0.3)])
def test_grid_matches_oracle_on_slab(vie, lam, th, ph):
    m = W.slab_mesh()
    eps = np.full(m.nt, 2.25 + 0.1j)
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    s, N = solver(vie, m, vie.VIE_GRID_FP64)
    print(f"grid slab N={N} lambda={lam} theta={th} phi={ph}", flush=True)
    s.fill(lam, th, ph, eps)
    x = seeded_x(N, 11)
    y = s.apply_Z(x)
    Zo = OV.assemble(t, OV.make_wave(lam, th, ph), eps)
    err = rel(y, Zo @ x)
    print(f"  |Zx - Zo x| / |Zo x| = {err:.3e}", flush=True)
    s.close()
    assert err < 1e-10


@pytest.mark.parametrize("lam,th,ph", [(550.0, 0.0, 0.0), (480.0, 0.6, 1.0)])
def test_grid_matches_dense_with_interfaces(vie, lam, th, ph):
    m = layered_grid()
    eps = eps_of(m)
    g, N = solver(vie, m, vie.VIE_GRID_FP64)
    d, _ = solver(vie, m, vie.VIE_FP64)
    print(f"grid layered N={N} lambda={lam} theta={th} phi={ph}", flush=True)
    g.fill(lam, th, ph, eps)
    d.fill(lam, th, ph, eps)
    for seed in (3, 4):
        x = seeded_x(N, seed)
        yg, yd = g.apply_Z(x), d.apply_Z(x)
        err = rel(yg, yd)
        print(f"  seed {seed}: |Zx_grid - Zx_dense| / |Zx_dense| = {err:.3e}", flush=True)
        assert err < 1e-10
    # a unit vector on a half-SWG (top) face and on an interface face: single columns of Z
    r, c = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    Zd = d.read_Z(r.ravel(), c.ravel()).reshape(N, N)
    for j in (0, N // 2, N - 1):
        e = np.zeros(N, complex); e[j] = 1.0
        assert rel(g.apply_Z(e), Zd[:, j]) < 1e-10
    g.close(); d.close()


@pytest.mark.parametrize("precond", [1, 2])
def uniform_grid(nx, ny, nz, a, b, c, split=True):
    xs = np.linspace(0.0, a, nx + 1); ys = np.linspace(0.0, b, ny + 1); zs = np.linspace(0.0, c, nz + 1)
    verts, tets = W.brick_grid_mesh(xs, ys, zs)
    cen = W.centroids(verts, tets)
    dom = (cen[:, 0] > a / 2).astype(np.int32) if split else np.zeros(len(tets), np.int32)
    return W.Mesh(verts, tets, dom, 2 if split else 1, a, b, (xs, ys, zs))


@pytest.mark.parametrize("name,mesh,lam,th,ph", [
    # two bricks per period and one layer: offsets +1 and -1 are the same ring offset
    ("2x2x1", lambda: uniform_grid(2, 2, 1, 40.0, 40.0, 20.0), 500.0, 0.5, 0.2),
    # a = b = 300 nm at 400 nm, theta 0.7: non-specular Floquet orders propagate
    ("diffracting", lambda: uniform_grid(3, 3, 2, 300.0, 300.0, 100.0), 400.0, 0.7, 0.3),
    # unequal bricks and counts in x and y, one domain
    ("5x2x3", lambda: uniform_grid(5, 2, 3, 70.0, 30.0, 45.0, split=False), 650.0, 0.9, 1.2),
])
def test_grid_edge_cases_match_dense(vie, name, mesh, lam, th, ph):
    m = mesh()
    eps = np.array([2.4 + 0.2j, 3.3 + 0.05j])[m.tet_domain]
    g, N = solver(vie, m, vie.VIE_GRID_FP64)
    d, _ = solver(vie, m, vie.VIE_FP64)
    g.fill(lam, th, ph, eps)
    d.fill(lam, th, ph, eps)
    x = seeded_x(N, 9)
    err = rel(g.apply_Z(x), d.apply_Z(x))
    g.close(); d.close()
    print(f"grid {name} N={N}: |Zx_grid - Zx_dense| / |Zx_dense| = {err:.3e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("precond", [1, 2])
def test_grid_solve_matches_dense(vie, precond):
    """With M = I (1) or M = diag(Z) (2) the grid and dense operators run the
    same method on the same Z: same iterations, same absorptance, R, T."""
    m = layered_grid()
    eps = eps_of(m)
    lam, th, ph = 520.0, 0.4, 0.7
    out, its = {}, {}
    for prec in (vie.VIE_GRID_FP64, vie.VIE_FP64):
        s, N = solver(vie, m, prec, restart=120)
        s.set_option(vie.VIE_OPT_PRECOND, precond)
        s.fill(lam, th, ph, eps)
        infos = s.solve_pair(tol=1e-11, max_iter=3000)
        assert all(i["converged"] for i in infos)
        out[prec] = [s.absorption(pol=p) for p in (0, 1)]
        its[prec] = [i["iters"] for i in infos]
        s.close()
        print(f"  precision {prec}, preconditioner {precond}: iterations {its[prec]}", flush=True)
    assert all(abs(a - b) <= 1 for a, b in zip(its[vie.VIE_GRID_FP64], its[vie.VIE_FP64]))
    for p in (0, 1):
        (Ag, Rg, Tg), (Ad, Rd, Td) = out[vie.VIE_GRID_FP64][p], out[vie.VIE_FP64][p]
        assert np.max(np.abs(np.asarray(Ag) - np.asarray(Ad))) < 1e-8
        assert abs(Rg - Rd) < 1e-8 and abs(Tg - Td) < 1e-8


def test_grid_refusals(vie):
    s = vie.Solver()
    s.upload_mesh(osc_small())                     # graded: not a uniform grid
    assert s.workspace_bytes(vie.VIE_GRID_FP64, 20) == 0
    buf = s.torch.empty(1 << 20, dtype=s.torch.uint8, device="cuda:0")
    off = (-buf.data_ptr()) % 256
    rc = s.lib.vie_bind_workspace(s.h, ctypes.c_void_p(buf.data_ptr() + off), buf.numel() - off, vie.VIE_GRID_FP64, 20)
    assert rc == vie.VIE_EINVAL
    assert "uniform Kuhn brick grid" in s.lib.vie_last_error(s.h).decode()
    m = layered_grid()
    g, N = solver(vie, m, vie.VIE_GRID_FP64)
    g.fill(600.0, 0.0, 0.0, eps_of(m))
    for call in (g.factor, lambda: g.read_Z(np.array([0]), np.array([0])), lambda: g.solve(0, tol=1e-8)):
        with pytest.raises(vie.VieError) as e:
            call()
        assert e.value.code == vie.VIE_EINVAL
    g.set_option(vie.VIE_OPT_PRECOND, 1)
    g.set_option(vie.VIE_OPT_GRAPH_STEPS, 4)
    with pytest.raises(vie.VieError) as e:
        g.solve(0, tol=1e-8)
    assert e.value.code == vie.VIE_EINVAL
    g.close(); s.close()


def test_new_mesh_on_a_context_rebuilds_the_near_pattern(vie):
    """A context that uploads a second mesh builds that mesh's touching-pair
    pattern (the mixed path's sparse part), not the first one's."""
    m1, m2 = W.slab_mesh(nx=3, ny=3, nz=2), layered_grid()
    s = vie.Solver()
    s.upload_mesh(m1)
    s.bind(vie.VIE_MIXED_FP32, 20)
    s.upload_mesh(m2)
    s.bind(vie.VIE_MIXED_FP32, 20)
    f, N = solver(vie, m2, vie.VIE_MIXED_FP32, restart=20)
    for c in (s, f):
        c.fill(600.0, 0.3, 0.2, eps_of(m2))
    x = seeded_x(N, 5)
    same = np.array_equal(s.apply_Z(x), f.apply_Z(x))
    s.close(); f.close()
    assert same


def test_grid_and_jacobi_are_refused_where_not_offered(vie):
    """The grid operator is neither batched nor bound to the library's static
    workspace (its FFT plans allocate), and the batch does not take the
    point-Jacobi preconditioner: each is refused with VIE_EINVAL."""
    m = layered_grid()
    eps = eps_of(m)
    g, _ = solver(vie, m, vie.VIE_GRID_FP64)
    with pytest.raises(vie.VieError) as e:
        vie.Batch([g])
    assert e.value.code == vie.VIE_EINVAL and "grid operator" in str(e.value)
    g.close()
    s = vie.Solver()
    s.upload_mesh(m)
    with pytest.raises(vie.VieError) as e:
        s.bind_static(vie.VIE_GRID_FP64, 20)
    assert e.value.code == vie.VIE_EINVAL
    s.close()
    d, _ = solver(vie, m, vie.VIE_FP64, restart=40)
    d.set_option(vie.VIE_OPT_PRECOND, 2)
    b = vie.Batch([d])
    b.fill([600.0], [0.0], [0.0], [eps])
    b.factor()
    with pytest.raises(vie.VieError) as e:
        b.solve([0], restart=40)
    assert e.value.code == vie.VIE_EINVAL and "Jacobi" in str(e.value)
    d.close()
