"""Pins for the closed-form potentials (triangle and tetrahedron) against
brute-force quadrature.  Singular observation points are handled by splitting
the element at the point into sub-elements that have the point as a vertex and
integrating each with a collapsed-coordinate Gauss rule whose Jacobian
cancels the 1/R singularity."""
import numpy as np
from scipy.special import roots_jacobi, roots_legendre

from oracle import potentials as P

TRI = np.array([[0, 0, 0], [10, 1, 0], [3, 8, 1.0]])
TET = np.array([[0, 0, 0], [10, 0, 0], [2, 9, 0], [3, 3, 7.0]])


def gl01(n):
    x, w = roots_legendre(n)
    return (x + 1) / 2, w / 2


def tri_apex_rule(apex, b, c, n=60):
    """Points/weights on triangle (apex, b, c); Duffy map with Jacobian ~ s,
    geometrically graded panels in s so that points just off the plane
    (near-singular integrands) are resolved."""
    edges = np.concatenate([[0.0], np.logspace(-9, 0, 10)])
    x, w = gl01(20)
    s = np.concatenate([lo + (hi - lo) * x for lo, hi in zip(edges[:-1], edges[1:])])
    ws = np.concatenate([(hi - lo) * w for lo, hi in zip(edges[:-1], edges[1:])])
    t, wt = gl01(n)
    S, T = np.meshgrid(s, t, indexing="ij"); W = np.outer(ws, wt)
    pts = apex + S[..., None] * ((b - apex) + T[..., None] * (c - b))
    area2 = np.linalg.norm(np.cross(b - apex, c - apex))
    return pts.reshape(-1, 3), (W * S * area2).ravel()


def tet_apex_rule(apex, b, c, d, n=40):
    """Points/weights on tet (apex,b,c,d): x = apex + u[(b-apex) + v((c-b) + w(d-c))]."""
    u, wu = gl01(n); v, wv = gl01(n); w, ww = gl01(n)
    U, V, Wc = np.meshgrid(u, v, w, indexing="ij")
    pts = apex + U[..., None] * ((b - apex) + V[..., None] * ((c - b) + Wc[..., None] * (d - c)))
    vol6 = abs(np.linalg.det(np.array([b - apex, c - apex, d - apex])))
    W = np.einsum("i,j,k->ijk", wu, wv, ww) * U ** 2 * V * vol6
    return pts.reshape(-1, 3), W.ravel()


def brute_tri(r, tri):
    """Split the triangle at the projection of r into three signed triangles
    with that point as apex (handles points on or near the plane)."""
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    nh = nrm / np.linalg.norm(nrm)
    q = r - np.dot(r - tri[0], nh) * nh
    pts = []; wts = []
    for b, c in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])):
        p, w = tri_apex_rule(q, b, c)
        pts.append(p); wts.append(w * np.sign(np.dot(np.cross(b - q, c - q), nrm)))
    pts = np.vstack(pts); wts = np.concatenate(wts)
    R = np.linalg.norm(pts - r, axis=1)
    return np.sum(wts / R), np.sum(wts * R)


def brute_tet(r, tet):
    faces = [(1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1)]
    tot = 0.0; totv = np.zeros(3)
    c = tet.mean(0)
    for f in faces:
        b, cc, d = tet[list(f)]
        p, w = tet_apex_rule(r, b, cc, d)
        n = np.cross(cc - b, d - b)
        sgn = np.sign(np.dot(b - r, n)) * np.sign(np.dot(b - c, n))
        R = np.linalg.norm(p - r, axis=1)
        tot += sgn * np.sum(w / R)
        totv += sgn * np.sum(w[:, None] * (p - r) / R[:, None], axis=0)
    return tot, totv


def test_triangle_off_and_on_plane():
    nrm = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]); nrm /= np.linalg.norm(nrm)
    pts = [np.array([2, 2, 3.0]), np.array([5, 5, -2.0]), np.array([20, 3, 1.0]), np.array([4, 3, 0.7]),
           TRI.mean(0), TRI[0] + 0.3 * (TRI[1] - TRI[0]) + 0.2 * (TRI[2] - TRI[0]),
           TRI[0] + 1.5 * (TRI[1] - TRI[0]), TRI.mean(0) + 1e-3 * nrm]
    for r in pts:
        a1, b1 = P.tri_potentials(r, TRI)
        a2, b2 = brute_tri(r, TRI)
        assert abs(a1 - a2) < 1e-10 * abs(a2), (r, a1, a2)
        assert abs(b1 - b2) < 1e-10 * abs(b2), (r, b1, b2)


def test_tetrahedron_inside_and_outside():
    pts = [np.array([20, 20, 20.0]), np.array([5, 5, 10.0]), np.array([12, 1, 1.0]),
           np.array([3.0, 3.0, 2.0]), TET.mean(0), np.array([2.0, 1.0, 0.0])]
    for r in pts:
        p1, v1 = P.tet_potentials(r, TET)
        p2, v2 = brute_tet(r, TET)
        assert abs(p1 - p2) < 1e-9 * abs(p2), (r, p1, p2)
        assert np.max(np.abs(v1 - v2)) < 1e-9 * np.max(np.abs(v2)), (r, v1, v2)


def test_broadcast_matches_loop():
    rng = np.random.default_rng(0)
    tets = TET[None] + rng.normal(0, 1, (5, 4, 3))
    r = rng.normal(3, 4, (5, 7, 3))
    Pb, Vb = P.tet_potentials(r, tets[:, None])
    for i in range(5):
        Pl, Vl = P.tet_potentials(r[i], tets[i])
        assert np.allclose(Pb[i], Pl, rtol=1e-14) and np.allclose(Vb[i], Vl, rtol=1e-13)
