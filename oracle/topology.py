"""SWG topology of a periodic tetrahedral unit cell (Sec. 2.1; Sec. 2.2 for the
unit-cell reduction).

One SWG unknown per face (Sec. 2.1: SWG basis on tetrahedra, normal
continuity).  Readings of what the paper leaves open:
  * faces on the x = 0 / x = a (and y) walls are identified by translation and
    form ONE Bloch-periodic SWG whose second tetrahedron is an in-cell
    tetrahedron plus a lattice shift rho;
  * T+ is the tetrahedron with the lower global index; a face on the top or
    bottom of the structure is a half-SWG with T+ only (outward normal);
  * f = +/- (a_n / (3 V)) (r - p) on T+/T-, p the free vertex (unit normal
    component on the face);
  * the face's domain is the lower domain id of its tetrahedra; unknowns are
    ordered by domain, then by their sorted canonical vertex key, so each
    domain's block A_dd (Sec. 2.3, Eq. 5) is a contiguous diagonal block;
  * a face is a surface-charge element when it bounds the structure or
    separates two domains;
  * two elements (tetrahedra or faces) are "near" under lattice image
    (m, n) when the source element shifted by -(m a, n b) shares a vertex with
    the test element (integer test on canonical vertex ids).
"""
from dataclasses import dataclass
import numpy as np


class MeshError(ValueError):
    pass


@dataclass
class Topology:
    a: float
    b: float
    verts: np.ndarray        # [nv, 3]
    tets: np.ndarray         # [nt, 4]
    dom: np.ndarray          # [nt]
    ndom: int
    canon: np.ndarray        # [nv] canonical vertex id
    voff: np.ndarray         # [nv, 2] lattice offset of each vertex
    vol: np.ndarray          # [nt]
    # per unknown (sorted order)
    N: int
    face_vid: np.ndarray     # [N, 3] vertex ids of the face as it sits in T+
    tplus: np.ndarray        # [N]
    tminus: np.ndarray       # [N] (-1 for half-SWG)
    shift: np.ndarray        # [N, 2] integer lattice shift of T-'s copy of the face
    fdom: np.ndarray         # [N]
    area: np.ndarray         # [N]
    free_plus: np.ndarray    # [N] vertex id of the free vertex in T+
    free_minus: np.ndarray   # [N] (-1 for half-SWG)
    key: list                # [N] canonical key
    # per tet
    t2f: np.ndarray          # [nt, 4] unknown on the face opposite local vertex k
    t2s: np.ndarray          # [nt, 4] +1 / -1
    t2shift: np.ndarray      # [nt, 4, 2] lattice shift of this tet's copy (0 for T+)
    charged: np.ndarray      # [Nc] unknown ids of surface-charge faces
    domain_ranges: list      # [(start, end)] per domain
    ncanon: int

    @property
    def is_half(self):
        return self.tminus < 0


def _canonical_vertices(verts, a, b):
    tol = 1e-6 * max(a, b)
    x, y = verts[:, 0], verts[:, 1]
    if np.any(x < -tol) or np.any(x > a + tol) or np.any(y < -tol) or np.any(y > b + tol):
        raise MeshError("vertex outside the unit cell")
    ox = (np.abs(x - a) < tol).astype(np.int64)
    oy = (np.abs(y - b) < tol).astype(np.int64)
    cpos = verts.copy()
    cpos[:, 0] -= ox * a
    cpos[:, 1] -= oy * b
    q = np.round(cpos / tol).astype(np.int64)
    table = {}
    for i in range(len(verts)):
        if ox[i] == 0 and oy[i] == 0:
            k = tuple(q[i])
            if k in table:
                raise MeshError("duplicate vertex")
            table[k] = i
    canon_of_vertex = np.empty(len(verts), np.int64)
    for i in range(len(verts)):
        k = tuple(q[i])
        if k not in table:
            raise MeshError("vertex on a periodic wall has no partner on the opposite wall")
        canon_of_vertex[i] = table[k]
    # renumber canonical ids densely in increasing vertex-id order
    uniq = np.unique(canon_of_vertex)
    remap = -np.ones(len(verts), np.int64)
    remap[uniq] = np.arange(len(uniq))
    return remap[canon_of_vertex], np.stack([ox, oy], 1), len(uniq)


def build(verts, tets, tet_domain, ndom, a, b):
    verts = np.asarray(verts, float)
    tets = np.asarray(tets, np.int64)
    dom = np.asarray(tet_domain, np.int64)
    nt = len(tets)
    canon, voff, ncanon = _canonical_vertices(verts, a, b)
    v = verts[tets]
    vol6 = np.einsum("ij,ij->i", np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), v[:, 3] - v[:, 0])
    if np.any(np.abs(vol6) <= 1e-12 * max(a, b) ** 3):
        raise MeshError("degenerate tetrahedron")
    vol = np.abs(vol6) / 6.0
    ext = v.max(axis=1) - v.min(axis=1)
    if np.any(ext[:, 0] > 0.5 * a * (1 + 1e-9)) or np.any(ext[:, 1] > 0.5 * b * (1 + 1e-9)):
        raise MeshError("fewer than 2 cells per periodic direction")

    groups = {}
    for t in range(nt):
        for k in range(4):
            loc = [j for j in range(4) if j != k]
            vid = tets[t, loc]
            order = np.argsort(canon[vid], kind="stable")
            vid = vid[order]
            c = canon[vid]
            off = voff[vid]
            rel = off - off[0]
            key = (int(c[0]), int(c[1]), int(c[2]),
                   int(rel[1, 0]), int(rel[1, 1]), int(rel[2, 0]), int(rel[2, 1]))
            groups.setdefault(key, []).append((t, k, vid, off[0].copy()))

    recs = []
    for key, lst in groups.items():
        if len(lst) > 2:
            raise MeshError("non-manifold face")
        lst = sorted(lst, key=lambda r: r[0])
        tp, kp, vidp, offp = lst[0]
        if len(lst) == 2:
            tm, km, vidm, offm = lst[1]
            shift = offm - offp
            fdom = min(dom[tp], dom[tm])
            free_m = tets[tm, km]
        else:
            pv = verts[vidp]
            for ax, L in ((0, a), (1, b)):
                if np.all(np.abs(pv[:, ax]) < 1e-6 * L) or np.all(np.abs(pv[:, ax] - L) < 1e-6 * L):
                    raise MeshError("periodic wall face has no partner")
            tm, km, shift, fdom, free_m = -1, -1, np.zeros(2, np.int64), dom[tp], -1
        pv = verts[vidp]
        area = 0.5 * np.linalg.norm(np.cross(pv[1] - pv[0], pv[2] - pv[0]))
        recs.append(dict(key=key, tp=tp, kp=kp, tm=tm, km=km, vid=vidp, shift=shift,
                         fdom=int(fdom), area=area, free_p=tets[tp, kp], free_m=free_m))
    recs.sort(key=lambda r: (r["fdom"],) + r["key"])
    N = len(recs)
    t2f = -np.ones((nt, 4), np.int64)
    t2s = np.zeros((nt, 4), np.int64)
    t2shift = np.zeros((nt, 4, 2), np.int64)
    for i, r in enumerate(recs):
        t2f[r["tp"], r["kp"]] = i
        t2s[r["tp"], r["kp"]] = 1
        if r["tm"] >= 0:
            t2f[r["tm"], r["km"]] = i
            t2s[r["tm"], r["km"]] = -1
            t2shift[r["tm"], r["km"]] = r["shift"]
    fdom = np.array([r["fdom"] for r in recs])
    tminus = np.array([r["tm"] for r in recs])
    tplus = np.array([r["tp"] for r in recs])
    charged = np.array([i for i, r in enumerate(recs)
                        if r["tm"] < 0 or dom[r["tp"]] != dom[r["tm"]]], np.int64)
    ranges = []
    for d in range(ndom):
        idx = np.nonzero(fdom == d)[0]
        ranges.append((int(idx[0]), int(idx[-1]) + 1) if len(idx) else (0, 0))
    return Topology(a=a, b=b, verts=verts, tets=tets, dom=dom, ndom=ndom, canon=canon, voff=voff,
                    vol=vol, N=N, face_vid=np.array([r["vid"] for r in recs]),
                    tplus=tplus, tminus=tminus,
                    shift=np.array([r["shift"] for r in recs]), fdom=fdom,
                    area=np.array([r["area"] for r in recs]),
                    free_plus=np.array([r["free_p"] for r in recs]),
                    free_minus=np.array([r["free_m"] for r in recs]),
                    key=[r["key"] for r in recs], t2f=t2f, t2s=t2s, t2shift=t2shift,
                    charged=charged, domain_ranges=ranges, ncanon=ncanon)


def near_images(canon, voff, vid_test, vid_src):
    """Set of lattice images (m, n) under which the source element (vertex ids
    vid_src) shifted by -(m a, n b) shares a vertex with the test element."""
    out = set()
    for v in vid_test:
        for w in vid_src:
            if canon[v] == canon[w]:
                d = voff[w] - voff[v]
                out.add((int(d[0]), int(d[1])))
    return sorted(out)
