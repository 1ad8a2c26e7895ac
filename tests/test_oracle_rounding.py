"""The oracle's own rounding spread on small entries of Z, which sets the floor
of the relative tolerance in the entry-by-entry parity tests.

Z is assembled twice for the same cell: once as given, once with the four
vertices of every tetrahedron listed in another order and the whole mesh
moved by 7.3 nm along z.  Neither changes Z in exact arithmetic (Eq. 2
depends on differences of points only, quadrature rules are symmetric, the
unknown order and orientation depend on vertex ids and tet indices only),
but every quadrature sum and every coordinate difference rounds differently.
Each entry is a sum of terms as large as max|Z|, so the spread is about
1e-16 max|Z| in absolute terms: on entries near 1e-6 max|Z| that is already
~1e-10 relative, the size of the target.  Below 1e-5 max|Z| the parity tests
therefore compare against 1e-10 * 1e-5 max|Z| in absolute terms."""
import numpy as np

from oracle import topology as T
from oracle import vie as V
from paper_1809_05334_amd import workloads as W


def three_domain_cell():
    xs = np.array([0.0, 12.0, 20.0, 28.0, 40.0])
    zs = np.array([0.0, 20.0, 30.0, 40.0])
    verts, tets = W.brick_grid_mesh(xs, xs, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 20.0, W.DOM_ACTIVE, W.DOM_SPACER).astype(np.int32)
    dom[np.sum((c - [20.0, 20.0, 30.0]) ** 2, 1) <= 8.0 ** 2] = W.DOM_METAL
    return W.Mesh(verts, tets, dom, 3, 40.0, 40.0, (xs, xs, zs))


def test_summation_order_spread_on_small_entries():
    m = three_domain_cell()
    eps = W.osc_eps(m, 520.0)
    wave = V.make_wave(520.0, 0.5, 0.3)
    topo1 = T.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    Z1 = V.assemble(topo1, wave, eps)
    mx = np.abs(Z1).max()
    small = np.abs(Z1) < 1e-5 * mx
    rows = np.unique(np.nonzero(small)[0])[:48]
    assert len(rows) >= 8
    rng = np.random.default_rng(5)
    tets2 = np.array([t[rng.permutation(4)] for t in m.tets], np.int32)
    v2 = m.verts.copy()
    v2[:, 2] += 7.3
    topo2 = T.build(v2, tets2, m.tet_domain, m.ndom, m.a, m.b)
    assert np.array_equal(topo2.tplus, topo1.tplus) and np.array_equal(topo2.face_vid, topo1.face_vid)
    Z2 = V.assemble(topo2, wave, eps, rows=rows)
    d = np.abs(Z1[rows] - Z2)
    a1 = np.abs(Z1[rows])
    # both orders agree to rounding of the largest contributions
    assert d.max() < 2e-14 * mx
    sel = small[rows] & (a1 > 0)
    # on the small entries that rounding is 1e-16 max|Z| in absolute terms ...
    assert d[sel].max() < 1e-15 * mx
    # ... which is far from negligible relative to the entries themselves
    rel = d[sel] / a1[sel]
    assert rel.max() > 1e-11, rel.max()
