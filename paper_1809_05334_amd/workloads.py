"""Seeded synthetic inputs shaped like the paper's plasmonic solar-cell workloads.

This module only *produces inputs*: tetrahedral unit-cell meshes, per-tetrahedron
relative permittivities and illumination parameters.  It holds none of the
method's arithmetic (no basis functions, Green's functions or matrix terms), so
both the CPU oracle's tests and the HIP path's tests/bench may draw from it.

Geometry follows the device of Fig. 1 (Sec. 2.2): a unit cell of period a x b,
periodic in x and y, holding a layer stack with a metal nanoparticle.  The
paper's measured permittivities are not available; constants and a one-pole
Drude model for silver stand in for them.

Mesh: a tensor-product ("graded") brick grid, each brick split into six
tetrahedra along its (0,0,0)->(1,1,1) diagonal (Kuhn/Freudenthal split), which
is conforming across bricks.  Vertices on the x = a and y = b walls are kept as
separate vertices; the periodic identification is the solver's job.
Materials are assigned per tetrahedron by its centroid.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

HC_EV_NM = 1239.841984  # h*c in eV*nm: photon energy [eV] = HC_EV_NM / lambda[nm]

# Kuhn split: the six vertex paths from corner (0,0,0) to (1,1,1) of a unit
# brick, one per permutation of the three axes.
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


@dataclass
class Mesh:
    verts: np.ndarray          # f64 [nv, 3], nm
    tets: np.ndarray           # i32 [nt, 4], 0-based vertex ids
    tet_domain: np.ndarray     # i32 [nt], material domain id (metal is 0 when present)
    ndom: int
    a: float                   # period along x, nm
    b: float                   # period along y, nm
    grid: tuple = field(default=())   # (xs, ys, zs) breakpoints used to build it
    info: dict = field(default_factory=dict)

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])


def brick_grid_mesh(xs, ys, zs):
    """Kuhn-split tetrahedral mesh of the box grid with breakpoints xs, ys, zs.

    Returns (verts f64[nv,3], tets i32[nt,4]).  Every tetrahedron is positively
    oriented (det[v1-v0, v2-v0, v3-v0] > 0)."""
    xs = np.asarray(xs, float); ys = np.asarray(ys, float); zs = np.asarray(zs, float)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    tets = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                for p in _PERMS:
                    c = [0, 0, 0]
                    path = [vid(i, j, k)]
                    for ax in p:
                        c[ax] += 1
                        path.append(vid(i + c[0], j + c[1], k + c[2]))
                    tets.append(path)
    tets = np.asarray(tets, dtype=np.int64)
    # orient positively
    v = verts[tets]
    det = np.einsum("ij,ij->i", np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), v[:, 3] - v[:, 0])
    neg = det < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    return verts, tets.astype(np.int32)


def graded_axis(length, fine_lo, fine_hi, h_fine, h_coarse):
    """Breakpoints on [0, length]: spacing ~h_fine inside [fine_lo, fine_hi],
    ~h_coarse outside; every piece is split into equal steps."""
    pts = [0.0]

    def add_segment(lo, hi, h):
        if hi - lo <= 1e-12:
            return
        n = max(1, int(np.ceil((hi - lo) / h - 1e-9)))
        for s in range(1, n + 1):
            pts.append(lo + (hi - lo) * s / n)

    fine_lo = max(0.0, fine_lo); fine_hi = min(length, fine_hi)
    add_segment(0.0, fine_lo, h_coarse)
    add_segment(fine_lo, fine_hi, h_fine)
    add_segment(fine_hi, length, h_coarse)
    return np.asarray(pts)


def centroids(verts, tets):
    return verts[tets].mean(axis=1)


def drude_eps(lambda_nm, eps_inf=3.7, wp_ev=9.0, gamma_ev=0.02):
    """Drude permittivity (optics sign, Im >= 0 is lossy):
    eps = eps_inf - wp^2 / (w^2 + i*gamma*w), energies in eV."""
    w = HC_EV_NM / lambda_nm
    return eps_inf - wp_ev ** 2 / (w * w + 1j * gamma_ev * w)


# ---------------------------------------------------------------- homogeneous slab
EPS_SLAB = 3.6 + 0.6j
EPS_ACTIVE = 3.6 + 0.6j
EPS_SPACER = 2.3 + 0.05j


def slab_mesh(a=100.0, b=100.0, thickness=50.0, nx=4, ny=4, nz=2):
    """Homogeneous slab z in [0, thickness] in an a x b cell (single domain)."""
    xs = np.linspace(0.0, a, nx + 1); ys = np.linspace(0.0, b, ny + 1)
    zs = np.linspace(0.0, thickness, nz + 1)
    verts, tets = brick_grid_mesh(xs, ys, zs)
    dom = np.zeros(len(tets), np.int32)
    return Mesh(verts, tets, dom, 1, float(a), float(b), (xs, ys, zs),
                {"kind": "slab", "thickness": thickness})


def slab_eps(mesh, eps=EPS_SLAB):
    return np.full(mesh.nt, eps, dtype=np.complex128)


# ---------------------------------------------------------------- plasmonic cells
DOM_METAL, DOM_SPACER, DOM_ACTIVE = 0, 1, 2


def osc_cell_mesh(a, t_active, t_spacer, radius, h_fine, h_coarse, b=None):
    """Plasmonic organic-solar-cell unit cell (Fig. 1 shape):
    active layer z in [0, t_active], spacer layer z in [t_active, t_active+t_spacer],
    a metal sphere of `radius` centred in the spacer layer at (a/2, b/2).
    Fine spacing over the sphere's x/y span and the whole spacer layer,
    coarse spacing elsewhere.  Domains: 0 metal, 1 spacer, 2 active."""
    b = a if b is None else b
    zc = t_active + 0.5 * t_spacer
    xs = graded_axis(a, a / 2 - radius, a / 2 + radius, h_fine, h_coarse)
    ys = graded_axis(b, b / 2 - radius, b / 2 + radius, h_fine, h_coarse)
    zs_act = graded_axis(t_active, 0.0, 0.0, h_fine, h_coarse)
    zs_sp = t_active + graded_axis(t_spacer, 0.0, t_spacer, h_fine, h_coarse)
    zs = np.concatenate([zs_act, zs_sp[1:]])
    verts, tets = brick_grid_mesh(xs, ys, zs)
    c = centroids(verts, tets)
    dom = np.where(c[:, 2] < t_active, DOM_ACTIVE, DOM_SPACER).astype(np.int32)
    inside = np.sum((c - np.array([a / 2, b / 2, zc])) ** 2, axis=1) <= radius ** 2
    dom[inside] = DOM_METAL
    ndom = 3
    return Mesh(verts, tets, dom, ndom, float(a), float(b), (xs, ys, zs),
                {"kind": "osc", "t_active": t_active, "t_spacer": t_spacer,
                 "radius": radius, "h_fine": h_fine, "h_coarse": h_coarse})


def osc_eps(mesh, lambda_nm, eps_active=EPS_ACTIVE, eps_spacer=EPS_SPACER, drude=None):
    drude = drude or {}
    eps_dom = np.array([drude_eps(lambda_nm, **drude), eps_spacer, eps_active],
                       dtype=np.complex128)
    return eps_dom[mesh.tet_domain]


def plasmonic_cell_mesh():
    """Plasmonic cell: period 200 nm, active 80 nm + spacer 40 nm, Ag sphere r=20 nm;
    5 nm over the sphere span and the spacer layer, 20 nm elsewhere."""
    return osc_cell_mesh(200.0, 80.0, 40.0, 20.0, 5.0, 20.0)


def plasmonic_cell_fine_mesh():
    """The plasmonic cell's geometry at ~3.33 nm fine / 20 nm coarse (N = 77,600)."""
    return osc_cell_mesh(200.0, 80.0, 40.0, 20.0, 40.0 / 12.0, 20.0)


def count_unknowns_paired(xs, ys, zs):
    """Number of SWG unknowns of a Kuhn brick grid with the x/y walls paired.
    Per brick: 6 tets; faces = interior + boundary.  With periodic pairing in
    x and y the count is exact for any tensor grid."""
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    # Each brick contributes: 6 interior faces inside the brick (Kuhn split has
    # 6 internal triangles) + the 6 brick facets, each split in 2 triangles and
    # shared between two bricks (periodic in x,y; top/bottom unshared).
    interior = 6 * nx * ny * nz
    facets_x = nx * ny * nz * 2          # x-facets, periodic: one per brick
    facets_y = nx * ny * nz * 2
    facets_z = nx * ny * (nz + 1) * 2
    return interior + facets_x + facets_y + facets_z


def batch_cells(n_cells=256, seed=0, n_lo=2000, n_hi=15000):
    """Independent cells of uneven size (seeded), for batching and serving.

    Returns a list of dicts with the mesh parameters and one illumination
    (lambda, theta, phi, pol) per cell.  Fine spacing is coarsened from
    U[5, 8] nm until the unknown count fits a target drawn in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    cells = []
    for i in range(n_cells):
        a = rng.uniform(100.0, 300.0)
        t_sp = rng.uniform(30.0, 60.0)
        t_act = rng.uniform(60.0, 100.0)
        h_f0 = rng.uniform(5.0, 8.0)
        r_hi = min(40.0, t_sp / 2.0, a / 2.0 - h_f0)
        radius = rng.uniform(10.0, max(10.0, r_hi))
        n_target = int(rng.uniform(n_lo, n_hi))
        lam = rng.uniform(400.0, 800.0)
        theta = np.deg2rad(rng.uniform(0.0, 60.0))
        phi = np.deg2rad(rng.uniform(0.0, 90.0))
        pol = int(rng.integers(0, 2))
        while wood_margin(a, a, lam, theta, phi) < 0.03:   # keep clear of Rayleigh-Wood anomalies
            lam = rng.uniform(400.0, 800.0)
        h_c = min(40.0, a / 3.0)
        h_f = h_f0
        while True:
            mesh_args = (a, t_act, t_sp, radius, h_f, h_c)
            xs = graded_axis(a, a / 2 - radius, a / 2 + radius, h_f, h_c)
            zs = np.concatenate([graded_axis(t_act, 0, 0, h_f, h_c),
                                 t_act + graded_axis(t_sp, 0, t_sp, h_f, h_c)[1:]])
            n = count_unknowns_paired(xs, xs, zs)
            if n <= n_target or h_f >= h_c / 1.0 or h_f >= 4 * h_f0:
                break
            h_f *= 1.08
        cells.append({"a": a, "t_active": t_act, "t_spacer": t_sp, "radius": radius,
                      "h_fine": h_f, "h_coarse": h_c, "n_est": n,
                      "lambda": lam, "theta": theta, "phi": phi, "pol": pol})
    return cells


def cell_mesh(cell):
    """Mesh of a cell drawn by batch_cells / serve_trace."""
    return osc_cell_mesh(cell["a"], cell["t_active"], cell["t_spacer"], cell["radius"], cell["h_fine"],
                         cell["h_coarse"])


def large_cell(rng, n_lo=15000, n_hi=60000):
    """The plasmonic cell's geometry (200 nm period, 80 + 40 nm layers, r = 20 nm sphere)
    with the fine spacing coarsened from 3.33 nm until N <= N_target."""
    n_target = int(rng.uniform(n_lo, n_hi))
    a, t_act, t_sp, radius, h_c = 200.0, 80.0, 40.0, 20.0, 20.0
    h_f = 40.0 / 12.0
    while True:
        xs = graded_axis(a, a / 2 - radius, a / 2 + radius, h_f, h_c)
        zs = np.concatenate([graded_axis(t_act, 0, 0, h_f, h_c), t_act + graded_axis(t_sp, 0, t_sp, h_f, h_c)[1:]])
        n = count_unknowns_paired(xs, xs, zs)
        if n <= n_target or h_f >= h_c / 2:
            break
        h_f *= 1.05
    return {"a": a, "t_active": t_act, "t_spacer": t_sp, "radius": radius, "h_fine": h_f, "h_coarse": h_c,
            "n_est": n}


def serve_trace(rate, n_requests, seed=1, large_frac=0.1, n_lo=2000, n_hi=15000, large_lo=15000,
                large_hi=60000):
    """Poisson request stream (requests / s) of (cell, lambda, theta, phi, pol):
    1 - large_frac of the cells from batch_cells, large_frac large cells of
    the plasmonic cell's geometry.  Returns dicts with the cell, the
    illumination and the arrival time (s from the start)."""
    rng = np.random.default_rng(seed)
    small = batch_cells(n_requests, seed=seed + 1000, n_lo=n_lo, n_hi=n_hi)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < large_frac:
            cell = large_cell(rng, large_lo, large_hi)
        else:
            cell = {k: small[i][k] for k in ("a", "t_active", "t_spacer", "radius", "h_fine", "h_coarse", "n_est")}
        lam = rng.uniform(400.0, 800.0)
        theta = np.deg2rad(rng.uniform(0.0, 60.0))
        phi = np.deg2rad(rng.uniform(0.0, 90.0))
        while wood_margin(cell["a"], cell["a"], lam, theta, phi) < 0.03:
            lam = rng.uniform(400.0, 800.0)
        out.append({"rid": i, "arrival": t, "cell": cell, "lambda": lam, "theta": theta, "phi": phi,
                    "pol": int(rng.integers(0, 2))})
    return out


def wood_margin(a, b, lambda_nm, theta, phi, M=4):
    """min over non-specular Floquet orders (p,q) != (0,0), |p|,|q| <= M, of
    | |k_t,pq|^2 - k0^2 |^(1/2) / k0 : a small value flags a Rayleigh-Wood
    anomaly (an order grazing the cell plane).  Used only to redraw inputs."""
    k0 = 2 * np.pi / lambda_nm
    kx = k0 * np.sin(theta) * np.cos(phi); ky = k0 * np.sin(theta) * np.sin(phi)
    best = np.inf
    for p in range(-M, M + 1):
        for q in range(-M, M + 1):
            if p == 0 and q == 0:
                continue
            kt2 = (kx + 2 * np.pi * p / a) ** 2 + (ky + 2 * np.pi * q / b) ** 2
            best = min(best, np.sqrt(abs(kt2 - k0 * k0)) / k0)
    return best


def random_points_in_cell(rng, n, a, b, zlo, zhi):
    return np.stack([rng.uniform(0, a, n), rng.uniform(0, b, n), rng.uniform(zlo, zhi, n)], 1)
