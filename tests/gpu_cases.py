"""Small seeded cases shared by the GPU parity tests (inputs only)."""
import numpy as np

from paper_1809_05334_amd import workloads as W


def slab_small():
    return W.slab_mesh(a=50.0, b=50.0, thickness=50.0, nx=2, ny=2, nz=2)


def slab_100nm():
    return W.slab_mesh()


def osc_small():
    xs = np.array([0.0, 12.0, 20.0, 28.0, 40.0])
    zs = np.array([0.0, 20.0, 30.0, 40.0])
    verts, tets = W.brick_grid_mesh(xs, xs, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 20.0, W.DOM_ACTIVE, W.DOM_SPACER).astype(np.int32)
    dom[np.sum((c - [20.0, 20.0, 30.0]) ** 2, 1) <= 8.0 ** 2] = W.DOM_METAL
    return W.Mesh(verts, tets, dom, 3, 40.0, 40.0, (xs, xs, zs))


def osc_rect():
    """Non-square cell with a 2-cell direction and an off-centre particle."""
    xs = np.array([0.0, 20.0, 35.0, 60.0])
    ys = np.array([0.0, 22.5, 45.0])
    zs = np.array([0.0, 15.0, 30.0])
    verts, tets = W.brick_grid_mesh(xs, ys, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 15.0, 1, 0).astype(np.int32)
    dom[np.sum((c - [30.0, 20.0, 20.0]) ** 2, 1) <= 9.0 ** 2] = 2
    return W.Mesh(verts, tets, dom, 3, 60.0, 45.0, (xs, ys, zs), {"kind": "rect"})


def osc_jitter():
    """osc_small's grid with every vertex off the cell walls and the top and
    bottom planes moved by up to 1.5 nm (seeded): tetrahedra that are no
    longer Kuhn-congruent; lossless permittivities (eps_for)."""
    m = osc_small()
    v = m.verts.copy()
    rng = np.random.default_rng(21)
    inner = ((v[:, 0] > 0) & (v[:, 0] < m.a) & (v[:, 1] > 0) & (v[:, 1] < m.b)
             & (v[:, 2] > v[:, 2].min()) & (v[:, 2] < v[:, 2].max()))
    v[inner] += rng.uniform(-1.5, 1.5, size=(int(inner.sum()), 3))
    return W.Mesh(v, m.tets, m.tet_domain, m.ndom, m.a, m.b, m.grid, {"kind": "lossless"})


def eps_for(mesh, lam):
    if mesh.ndom == 1:
        return W.slab_eps(mesh)
    if mesh.info.get("kind") == "lossless":
        table = np.array([2.3 + 0j, 3.6 + 0j, 2.1 + 0j])
        return table[mesh.tet_domain]
    if mesh.info.get("kind") == "rect":
        table = np.array([W.EPS_SPACER, W.EPS_ACTIVE, W.drude_eps(lam)])
        return table[mesh.tet_domain]
    return W.osc_eps(mesh, lam)
