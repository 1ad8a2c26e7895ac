"""Closed-form potential integrals over a flat triangle and a tetrahedron.

Used for the 1/(4 pi R) part extracted from g_p on touching element pairs
(the singular behaviour of the kernel in Sec. 2.1's integrals).  The triangle
formulas are the classical ones for a polygon (Wilton, Rao, Glisson, Schaubert,
Al-Bundak, Butler 1984): with the observation point r at signed height d over
the plane, projection rho0, and for each edge i its outward in-plane normal u_i,
t_i = (edge point - rho0).u_i, l_i^{+/-} the edge end coordinates along the
edge, R_i^{+/-} the end distances and R0_i^2 = t_i^2 + d^2:
    int_F 1/R dS = sum_i t_i f_i - |d| sum_i beta_i
    int_F R   dS = (1/3) [ d^2 int_F 1/R dS + (1/2) sum_i t_i (R0_i^2 f_i + l+ R+ - l- R-) ]
    f_i = ln((R+ + l+) / (R- + l-)),
    beta_i = atan(t l+ / (R0^2 + |d| R+)) - atan(t l- / (R0^2 + |d| R-)).
Tetrahedron by the divergence theorem over its faces (outward normals n_f,
d_f = (face point - r).n_f):
    int_T 1/R dV       = (1/2) sum_f d_f int_f 1/R dS      (div((r'-r)/R) = 2/R)
    int_T (r'-r)/R dV  = sum_f n_f int_f R dS             (grad' R = (r'-r)/R)

Arrays broadcast: points r [..., 3] against elements [..., 3, 3] / [..., 4, 3].
Pins: brute-force quadrature with the singularity removed by a Duffy-type
split at the observation point (tests).
"""
import numpy as np

_TINY = 1e-300


def _dot(u, v):
    return np.sum(u * v, axis=-1)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _edge_log(Rp, Rm, lp, lm):
    """ln((R+ + l+)/(R- + l-)) in a form that avoids 0/0 when both end
    coordinates are negative (then use the reciprocal identity)."""
    neg = (lp < 0) & (lm < 0)
    num = np.where(neg, Rm - lm, Rp + lp)
    den = np.where(neg, Rp - lp, Rm + lm)
    ok = (num > 0) & (den > 0)
    return np.where(ok, np.log(np.where(ok, num, 1.0) / np.where(ok, den, 1.0)), 0.0)


def tri_potentials(r, tri):
    """int_F 1/|r-r'| dS' and int_F |r-r'| dS' for points r [..., 3] and
    triangles tri [..., 3, 3] (broadcast).  Returns (I_inv, I_one)."""
    r = np.asarray(r, float)
    tri = np.asarray(tri, float)
    A, B, C = tri[..., 0, :], tri[..., 1, :], tri[..., 2, :]
    nrm = _unit(np.cross(B - A, C - A))
    d = _dot(r - A, nrm)
    ad = np.abs(d)
    rho0 = r - d[..., None] * nrm
    Iinv = 0.0
    Iedge = 0.0
    for i in range(3):
        Pm = tri[..., i, :]
        Pp = tri[..., (i + 1) % 3, :]
        opp = tri[..., (i + 2) % 3, :]
        lhat = _unit(Pp - Pm)
        w = Pm - opp
        u = _unit(w - _dot(w, lhat)[..., None] * lhat)      # outward in-plane edge normal
        t = _dot(Pm - rho0, u)
        lp = _dot(Pp - r, lhat)
        lm = _dot(Pm - r, lhat)
        Rp = np.linalg.norm(Pp - r, axis=-1)
        Rm = np.linalg.norm(Pm - r, axis=-1)
        R02 = t * t + d * d
        f = np.where(np.abs(t) > 0, _edge_log(Rp, Rm, lp, lm), 0.0)
        dp = R02 + ad * Rp
        dm = R02 + ad * Rm
        beta = (np.arctan2(t * lp, np.where(dp > _TINY, dp, _TINY))
                - np.arctan2(t * lm, np.where(dm > _TINY, dm, _TINY)))
        Iinv = Iinv + t * f - ad * beta
        Iedge = Iedge + t * (R02 * f + lp * Rp - lm * Rm)
    Ione = (d * d * Iinv + 0.5 * Iedge) / 3.0
    return Iinv, Ione


_TET_FACES = ((1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1))


def tet_potentials(r, tet):
    """int_T 1/|r-r'| dV' and int_T (r'-r)/|r-r'| dV' for points r [..., 3]
    and tetrahedra tet [..., 4, 3]; the leading dimensions broadcast (insert
    singleton axes as needed).  Returns (P, V1[..., 3])."""
    r = np.asarray(r, float)
    tet = np.asarray(tet, float)
    c = tet.mean(axis=-2)
    P = 0.0
    V1 = 0.0
    for fidx in _TET_FACES:
        tri = tet[..., list(fidx), :]
        n = _unit(np.cross(tri[..., 1, :] - tri[..., 0, :], tri[..., 2, :] - tri[..., 0, :]))
        n = n * np.sign(_dot(tri[..., 0, :] - c, n))[..., None]      # outward
        Iinv, Ione = tri_potentials(r, tri)
        df = _dot(tri[..., 0, :] - r, n)
        P = P + 0.5 * df * Iinv
        V1 = V1 + Ione[..., None] * n
    return P, V1
