"""Pins for the oracle's SWG topology on Kuhn brick grids: face counts
(closed form for a tensor grid with the x/y walls paired), orientation,
periodic shifts, domain-major order and the error paths."""
import numpy as np
import pytest

from oracle import topology as T
from paper_1809_05334_amd import workloads as W


def build(mesh):
    return T.build(mesh.verts, mesh.tets, mesh.tet_domain, mesh.ndom, mesh.a, mesh.b)


def test_slab_100nm_counts():
    m = W.slab_mesh()
    t = build(m)
    assert len(m.tets) == 192
    assert t.N == 416                                   # 448 faces, 32 wall pairs merged
    assert int(t.is_half.sum()) == 64                   # top + bottom
    paired = (t.tminus >= 0) & np.any(t.shift != 0, axis=1)
    assert int(paired.sum()) == 32
    assert len(t.charged) == 64                         # single domain: boundary only
    assert np.all(t.t2f >= 0)
    # every unknown appears in exactly one T+ slot and (if full) one T- slot
    assert np.sum(t.t2s == 1) == t.N and np.sum(t.t2s == -1) == t.N - 64


@pytest.mark.parametrize("nx,ny,nz", [(2, 3, 2), (3, 2, 4), (5, 4, 1)])
def test_face_count_formula(nx, ny, nz):
    m = W.slab_mesh(a=60.0, b=70.0, thickness=30.0, nx=nx, ny=ny, nz=nz)
    t = build(m)
    xs, ys, zs = m.grid
    assert t.N == W.count_unknowns_paired(xs, ys, zs)
    # Euler-type count without pairing: 6 bricks-internal + facet triangles
    unpaired = 6 * nx * ny * nz + 2 * ((nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))
    assert t.N == unpaired - 2 * (ny * nz + nx * nz)


def test_orientation_and_shift():
    m = W.slab_mesh(a=50, b=50, nx=2, ny=2, nz=2)
    t = build(m)
    L = np.array([t.a, t.b, 0.0])
    for n in range(t.N):
        if t.tminus[n] < 0:
            continue
        # the T- copy of the face is the T+ copy translated by the shift
        tm = t.tminus[n]
        k = list(t.t2f[tm]).index(n)
        fm = np.sort([tuple(v) for v in t.verts[np.delete(t.tets[tm], k)]], axis=0)
        fp = np.sort([tuple(v) for v in t.verts[t.face_vid[n]] + t.shift[n, 0] * np.array([t.a, 0, 0])
                      + t.shift[n, 1] * np.array([0, t.b, 0])], axis=0)
        assert np.allclose(np.sort(fm, axis=0), np.sort(fp, axis=0))
        # free vertices lie on opposite sides of the (shifted) face
        pv = t.verts[t.face_vid[n]]
        nrm = np.cross(pv[1] - pv[0], pv[2] - pv[0])
        sp = (t.verts[t.free_plus[n]] - pv[0]) @ nrm
        sm = (t.verts[t.free_minus[n]] - np.append(t.shift[n], 0) * L - pv[0]) @ nrm
        assert sp * sm < 0
        assert t.tplus[n] < t.tminus[n]


def test_domain_major_order_and_charged_faces():
    m = W.osc_cell_mesh(60.0, 40.0, 30.0, 9.0, 6.0, 15.0)
    t = build(m)
    assert np.all(np.diff(t.fdom) >= 0)
    for d, (s, e) in enumerate(t.domain_ranges):
        assert np.all(t.fdom[s:e] == d)
    dp = t.dom[t.tplus]
    dm = np.where(t.tminus >= 0, t.dom[np.maximum(t.tminus, 0)], -1)
    expect = np.nonzero((t.tminus < 0) | (dp != dm))[0]
    assert np.array_equal(np.sort(t.charged), expect)
    # interface faces belong to the lower domain id
    full = t.tminus >= 0
    assert np.all(t.fdom[full] == np.minimum(dp[full], dm[full]))


def test_touching_images_across_walls():
    m = W.slab_mesh(a=50, b=50, nx=2, ny=2, nz=1)
    t = build(m)
    c = m.verts[m.tets].mean(1)
    i = int(np.argmin(c[:, 0]))          # a tet at the x = 0 wall
    j = int(np.argmax(c[:, 0]))          # a tet at the x = a wall
    im = T.near_images(t.canon, t.voff, m.tets[i], m.tets[j])
    assert any(mm == 1 for mm, nn in im)  # source shifted by -a touches the test tet


def test_mesh_errors():
    m = W.slab_mesh(a=50, b=50, nx=1, ny=2, nz=1)
    with pytest.raises(T.MeshError):
        build(m)
    m = W.slab_mesh(a=50, b=50, nx=2, ny=2, nz=1)
    v = m.verts.copy(); v[np.argmax(v[:, 0] + 1e-3 * v[:, 1])] += [0, 0, 1.0]
    with pytest.raises(T.MeshError):
        T.build(v, m.tets, m.tet_domain, 1, 50, 50)
    tets = m.tets.copy(); tets[0, 1] = tets[0, 0]
    with pytest.raises(T.MeshError):
        T.build(m.verts, tets, m.tet_domain, 1, 50, 50)
