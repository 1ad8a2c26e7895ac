"""Impedance matrix, right-hand side, solves and outputs of the periodic SWG VIE.

Formulation (Sec. 2.1, Eqs. 1-2), written for D~ = D / eps0 = eps_r E after
multiplying Eq. 1 by eps0 (reading of the garbled Eq. 2, recorded with the
other readings):
    D~/eps_r - k0^2 int g_p kappa D~ dV' + grad Phi~ = E^i,
    Phi~ = int g_p rho~ dV',  rho~ = -div(kappa D~)  (volume + surface parts),
    kappa = 1 - 1/eps_r (Sec. 2.1, below Eq. 2).
Galerkin testing with the SWG functions f_m (integration by parts moves the
gradient onto f_m; the boundary term survives only on half-SWG faces):
  Z_mn = <f_m, f_n / eps_r>                                       (mass)
       - k0^2 sum_{T,T'} kappa_T' s_m s_n a_m a_n / (9 V_T V_T') II (r-p).(r'-q) g_p
       + sum_{T,T'} kappa_T' s_m s_n a_m a_n / (V_T V_T') II g_p   (volume charges)
       - sum_T s_m a_m / V_T sigma_n I_T I_{F_n} g_p              (surface charge)
       + [m half] I_{F_m} Phi~_n                                  (boundary term)
  b_m  = sum_T s_m a_m / (3 V_T) I_T (r - p).E^i dV,
with sigma_n = kappa(T+) - kappa(T-) (0 outside the structure).
Periodicity (Sec. 2.2): the T- half of a wall-paired SWG sits in the cell at a
lattice shift rho; its source phase is exp(-j kt.rho) and its test phase
exp(+j kt.rho), and every interaction uses g_p.

Conventions: exp(j w t) internally (Sec. 2.1).  Permittivities passed in use
the optics sign (Im >= 0 lossy); internally eps = conj(eps_in).
Incident wave from +z: k = k0 (sin th cos ph, sin th sin ph, -cos th),
E^i = e exp(-j k.r), TE e = (-sin ph, cos ph, 0), TM e = (cos th cos ph,
cos th sin ph, sin th), |E0| = 1.

Quadrature (readings): elements that share no vertex under any lattice image
use degree-2 product rules (tet 4 points, triangle 3 points); touching
elements use a degree-5 outer rule on the test element (tet 14 points,
triangle 7 points), the closed-form 1/R and (r'-r)/R integrals for every
touching image, and the degree-2 inner rule for the remainder
g_p - sum_near e^{j kt.rho}/(4 pi R).
"""
from dataclasses import dataclass
import numpy as np
import scipy.linalg as sla

from . import quadrature as Q
from . import pgf as PG
from . import potentials as POT
from . import topology as TOPO

FOUR_PI = 4.0 * np.pi
TE, TM = 0, 1


@dataclass
class Wave:
    lam: float
    theta: float
    phi: float
    k0: float
    kx: float
    ky: float
    kinc: np.ndarray

    def pol_vector(self, pol):
        th, ph = self.theta, self.phi
        if pol == TE:
            return np.array([-np.sin(ph), np.cos(ph), 0.0])
        return np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.sin(th)])


def make_wave(lam, theta, phi):
    k0 = 2.0 * np.pi / lam
    kx = k0 * np.sin(theta) * np.cos(phi)
    ky = k0 * np.sin(theta) * np.sin(phi)
    return Wave(lam, theta, phi, k0, kx, ky, np.array([kx, ky, -k0 * np.cos(theta)]))


# ----------------------------------------------------------------- elements
class Elements:
    """Tetrahedra (ids 0..nt-1) and surface-charge faces (ids nt..nt+Nc-1)."""

    def __init__(self, topo):
        self.topo = topo
        self.nt = len(topo.tets)
        self.charged = topo.charged
        self.slot_of_face = {int(n): i for i, n in enumerate(topo.charged)}
        lam4, w4 = Q.tet_deg2()
        lam5, w5 = Q.tet_deg5()
        lam3, w3 = Q.tri_deg2()
        lam7, w7 = Q.tri_deg5()
        tv = topo.verts[topo.tets]                       # [nt,4,3]
        self.tet_verts = tv
        self.tet_far_pts = np.einsum("qk,tkd->tqd", lam4, tv)
        self.tet_far_w = w4[None, :] * topo.vol[:, None]
        self.tet_near_pts = np.einsum("qk,tkd->tqd", lam5, tv)
        self.tet_near_w = w5[None, :] * topo.vol[:, None]
        fv = topo.verts[topo.face_vid[topo.charged]] if len(topo.charged) else np.zeros((0, 3, 3))
        self.face_verts = fv
        area = topo.area[topo.charged]
        self.face_far_pts = np.einsum("qk,fkd->fqd", lam3, fv)
        self.face_far_w = w3[None, :] * area[:, None]
        self.face_near_pts = np.einsum("qk,fkd->fqd", lam7, fv)
        self.face_near_w = w7[None, :] * area[:, None]

    def vids(self, kind, i):
        if kind == "t":
            return self.topo.tets[i]
        return self.topo.face_vid[self.charged[i]]


def _near(topo, vt, vs):
    return TOPO.near_images(topo.canon, topo.voff, vt, vs)


_POOL = None


def _pool():
    """Worker processes for the lattice sums (fork; the oracle is CPU-only)."""
    global _POOL
    if _POOL is None:
        import multiprocessing as mp
        import os
        n = min(16, len(os.sched_getaffinity(0)))
        _POOL = mp.get_context("fork").Pool(n) if n > 1 else False
    return _POOL


def _pgf_chunk(args):
    d, k0, kx, ky, a, b, E, M = args
    return PG.pgf_ewald(d, k0, kx, ky, a, b, E=E, M=M, self_limit=True)


class Kernel:
    def __init__(self, topo, wave, M=4, E=None, parallel=True):
        self.topo, self.w, self.M = topo, wave, M
        self.E = PG.ewald_split(topo.a, topo.b) if E is None else E
        self.parallel = parallel

    def g(self, delta):
        flat = np.asarray(delta, float).reshape(-1, 3)
        args = (self.w.k0, self.w.kx, self.w.ky, self.topo.a, self.topo.b, self.E, self.M)
        pool = _pool() if self.parallel and len(flat) > 20000 else False
        if pool:
            chunks = np.array_split(flat, max(1, len(flat) // 20000))
            out = np.concatenate(pool.map(_pgf_chunk, [(c,) + args for c in chunks]))
        else:
            out = _pgf_chunk((flat,) + args)
        return out.reshape(np.shape(delta)[:-1])

    def singular(self, delta, m, n):
        """e^{j kt.rho_mn} / (4 pi |delta + rho_mn|) (0 where the distance is 0)."""
        rho = np.array([m * self.topo.a, n * self.topo.b, 0.0])
        R = np.linalg.norm(delta + rho, axis=-1)
        ph = np.exp(1j * (self.w.kx * rho[0] + self.w.ky * rho[1]))
        return np.where(R > 0, ph / (FOUR_PI * np.where(R > 0, R, 1.0)), 0.0)


IMAGES = [(m, n) for m in (-1, 0, 1) for n in (-1, 0, 1)]


def touching_images(topo, VT, VS):
    """mask [P, 9] over IMAGES: element pair p touches under image (m, n)
    (source shifted by -(m a, n b) shares a vertex with the test element)."""
    ct = topo.canon[VT][:, :, None]
    cs = topo.canon[VS][:, None, :]
    eq = ct == cs
    d = topo.voff[VS][:, None, :, :] - topo.voff[VT][:, :, None, :]
    idx = (d[..., 0] + 1) * 3 + (d[..., 1] + 1)
    mask = np.zeros((len(VT), 9), bool)
    p, i, j = np.nonzero(eq)
    mask[p, idx[p, i, j]] = True
    return mask


# ------------------------------------------------------- pair integrals
def far_pairs(kern, Xt, Wt, Ys, Ws, Vt=None, Vs=None, chunk=200000):
    """Product-rule integrals for P element pairs.
    Xt [P,qt,3], Wt [P,qt], Ys [P,qs,3], Ws [P,qs].  Returns M0 [P] and, when
    the vertex arrays Vt [P,4,3], Vs [P,4,3] are given, I [P,4,4] with
    I[k,l] = II (r - v_k).(r' - v'_l) g_p."""
    P = len(Xt)
    M0 = np.zeros(P, complex)
    I = np.zeros((P, 4, 4), complex) if Vt is not None else None
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        d = Xt[s:e, :, None, :] - Ys[s:e, None, :, :]
        g = kern.g(d)
        ww = Wt[s:e, :, None] * Ws[s:e, None, :] * g
        M0[s:e] = ww.sum(axis=(1, 2))
        if I is not None:
            A = Xt[s:e, :, None, :] - Vt[s:e, None, :, :]      # [p,i,k,d]
            B = Ys[s:e, :, None, :] - Vs[s:e, None, :, :]      # [p,j,l,d]
            I[s:e] = np.einsum("pij,pikd,pjld->pkl", ww, A, B)
    return M0, I


def near_pairs(kern, Xo, Wo, src_kind, SV, Yi, Wi, mask, Vt=None, Vs=None, chunk=20000):
    """Touching pairs: outer rule (Xo [P,no,3], Wo) on the test element; for
    each touching image the closed-form inner integrals of 1/R (and r'/R for
    tetrahedra) over the source element SV; the inner rule (Yi, Wi) for the
    remainder g_p - sum_touching e^{j kt.rho}/(4 pi R).  Returns M0 [P] and
    optionally I [P,4,4]."""
    P = len(Xo)
    M0 = np.zeros(P, complex)
    I = np.zeros((P, 4, 4), complex) if Vt is not None else None
    topo, kx, ky = kern.topo, kern.w.kx, kern.w.ky
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        X, msk = Xo[s:e], mask[s:e]
        s0 = np.zeros(X.shape[:2], complex)
        s1 = np.zeros(X.shape, complex)
        for im, (m, n) in enumerate(IMAGES):
            sel = msk[:, im]
            if not sel.any():
                continue
            rho = np.array([m * topo.a, n * topo.b, 0.0])
            ph = np.exp(1j * (kx * rho[0] + ky * rho[1])) / FOUR_PI
            o = X[sel] + rho
            if src_kind == "t":
                Pv, V1 = POT.tet_potentials(o, SV[s:e][sel][:, None])
                s0[sel] += ph * Pv
                s1[sel] += ph * (V1 + o * Pv[..., None])          # int r'/R = V1 + o P
            else:
                Iinv, _ = POT.tri_potentials(o, SV[s:e][sel][:, None])
                s0[sel] += ph * Iinv
        d = X[:, :, None, :] - Yi[s:e, None, :, :]
        g = kern.g(d)
        for im, (m, n) in enumerate(IMAGES):
            sel = msk[:, im]
            if sel.any():
                g[sel] -= kern.singular(d[sel], m, n)
        gw = g * Wi[s:e, None, :]
        s0 += gw.sum(axis=2)
        s1 += np.einsum("pij,pjd->pid", gw, Yi[s:e])
        M0[s:e] = np.sum(Wo[s:e] * s0, axis=1)
        if I is not None:
            A = X[:, :, None, :] - Vt[s:e, None, :, :]                        # [p,i,k,d]
            B = s1[:, :, None, :] - Vs[s:e, None, :, :] * s0[:, :, None, None]  # [p,i,l,d]
            I[s:e] = np.einsum("pi,pikd,pild->pkl", Wo[s:e], A, B)
    return M0, I


def element_pair_integrals(kern, el, kind_t, it, kind_s, js, with_vp):
    """Integrals over all pairs (test it[p], source js[p]) of one kind."""
    topo = kern.topo
    VT = topo.tets[it] if kind_t == "t" else topo.face_vid[el.charged[it]]
    VS = topo.tets[js] if kind_s == "t" else topo.face_vid[el.charged[js]]
    mask = touching_images(topo, VT, VS)
    near = mask.any(axis=1)
    P = len(it)
    M0 = np.zeros(P, complex)
    I = np.zeros((P, 4, 4), complex) if with_vp else None

    def pts(kind, idx, which):
        if kind == "t":
            return ((el.tet_far_pts[idx], el.tet_far_w[idx]) if which == "far"
                    else (el.tet_near_pts[idx], el.tet_near_w[idx]))
        return ((el.face_far_pts[idx], el.face_far_w[idx]) if which == "far"
                else (el.face_near_pts[idx], el.face_near_w[idx]))

    f = np.nonzero(~near)[0]
    if len(f):
        Xt, Wt = pts(kind_t, it[f], "far")
        Ys, Ws = pts(kind_s, js[f], "far")
        m0, ii = far_pairs(kern, Xt, Wt, Ys, Ws,
                           el.tet_verts[it[f]] if with_vp else None,
                           el.tet_verts[js[f]] if with_vp else None)
        M0[f] = m0
        if with_vp:
            I[f] = ii
    nn = np.nonzero(near)[0]
    if len(nn):
        Xo, Wo = pts(kind_t, it[nn], "near")
        Yi, Wi = pts(kind_s, js[nn], "far")
        SV = el.tet_verts[js[nn]] if kind_s == "t" else el.face_verts[js[nn]]
        m0, ii = near_pairs(kern, Xo, Wo, kind_s, SV, Yi, Wi, mask[nn],
                            el.tet_verts[it[nn]] if with_vp else None,
                            el.tet_verts[js[nn]] if with_vp else None)
        M0[nn] = m0
        if with_vp:
            I[nn] = ii
    return M0, I, near


# ------------------------------------------------------------- assembly
def internal_eps(eps_in):
    return np.conj(np.asarray(eps_in, complex))


def _tet_quad_form(verts4, p, q):
    """I_T (r - p).(r - q) dV in closed form (second moments of a tet)."""
    V = abs(np.linalg.det(verts4[1:] - verts4[0])) / 6.0
    S = verts4.sum(axis=0)
    rr = V / 20.0 * (np.sum(verts4 * verts4) + S @ S)
    return rr - (p + q) @ (V * S / 4.0) + V * (p @ q)


def assemble(topo, wave, eps_in, rows=None, cols=None, M=4, E=None, verbose=False, parallel=True):
    """Dense Z restricted to rows x cols (all unknowns by default)."""
    N = topo.N
    rows = np.arange(N) if rows is None else np.asarray(rows)
    cols = np.arange(N) if cols is None else np.asarray(cols)
    rpos = -np.ones(N + 1, np.int64); rpos[rows] = np.arange(len(rows))
    cpos = -np.ones(N + 1, np.int64); cpos[cols] = np.arange(len(cols))
    Zp = np.zeros((len(rows) + 1, len(cols) + 1), complex)      # last row/col = sink
    eps = internal_eps(eps_in)
    kappa = 1.0 - 1.0 / eps
    kern = Kernel(topo, wave, M=M, E=E, parallel=parallel)
    el = Elements(topo)
    L = np.array([topo.a, topo.b])
    kt = np.array([wave.kx, wave.ky])
    k0 = wave.k0
    t2f, t2s = topo.t2f, topo.t2s
    chi = np.exp(1j * (topo.t2shift @ (kt * L)))        # test phase   [nt,4]
    psi = np.conj(chi)                                   # source phase [nt,4]
    area, vol = topo.area, topo.vol
    km = np.zeros(N, complex)
    has_m = topo.tminus >= 0
    km[has_m] = kappa[topo.tminus[has_m]]
    sigma = kappa[topo.tplus] - km

    def tets_of(us):
        tm = topo.tminus[us]
        return np.unique(np.concatenate([topo.tplus[us], tm[tm >= 0]]))

    test_tets = tets_of(rows)
    src_tets = tets_of(cols)
    half_rows = rows[topo.tminus[rows] < 0]
    cset = set(int(c) for c in cols)
    charged_cols = np.array([n for n in topo.charged if int(n) in cset], np.int64)
    slot = el.slot_of_face

    def rix(m):
        r = rpos[m]
        return np.where(r < 0, len(rows), r)

    def cix(n):
        c = cpos[n]
        return np.where(c < 0, len(cols), c)

    # ---- tetrahedron x tetrahedron: vector potential + volume charges
    it = np.repeat(test_tets, len(src_tets))
    js = np.tile(src_tets, len(test_tets))
    M0, I, near = element_pair_integrals(kern, el, "t", it, "t", js, True)
    if verbose:
        print(f"tet pairs {len(it)} touching {near.sum()}")
    for k in range(4):
        m = t2f[it, k]
        for l in range(4):
            n = t2f[js, l]
            c = (chi[it, k] * psi[js, l] * t2s[it, k] * t2s[js, l] * area[m] * area[n]
                 * kappa[js] / (vol[it] * vol[js]))
            np.add.at(Zp, (rix(m), cix(n)), c * (M0 - k0 * k0 / 9.0 * I[:, k, l]))

    # ---- test tetrahedron x surface charge on face n
    if len(charged_cols):
        it = np.repeat(test_tets, len(charged_cols))
        nf = np.tile(charged_cols, len(test_tets))
        jf = np.array([slot[int(n)] for n in nf], np.int64)
        M0, _, _ = element_pair_integrals(kern, el, "t", it, "f", jf, False)
        for k in range(4):
            m = t2f[it, k]
            np.add.at(Zp, (rix(m), cix(nf)),
                      chi[it, k] * sigma[nf] * (-t2s[it, k] * area[m] / vol[it]) * M0)

    # ---- half-SWG test face x (source tetrahedron, surface charge)
    if len(half_rows):
        hf = np.array([slot[int(m)] for m in half_rows], np.int64)
        im_ = np.repeat(hf, len(src_tets))
        mrow = np.repeat(half_rows, len(src_tets))
        js = np.tile(src_tets, len(half_rows))
        M0, _, _ = element_pair_integrals(kern, el, "f", im_, "t", js, False)
        for l in range(4):
            n = t2f[js, l]
            np.add.at(Zp, (rix(mrow), cix(n)),
                      psi[js, l] * (-kappa[js] * t2s[js, l] * area[n] / vol[js]) * M0)
        if len(charged_cols):
            im_ = np.repeat(hf, len(charged_cols))
            mrow = np.repeat(half_rows, len(charged_cols))
            nf = np.tile(charged_cols, len(half_rows))
            jf = np.array([slot[int(n)] for n in nf], np.int64)
            M0, _, _ = element_pair_integrals(kern, el, "f", im_, "f", jf, False)
            np.add.at(Zp, (rix(mrow), cix(nf)), sigma[nf] * M0)

    # ---- mass <f_m, f_n / eps_r>
    for t in test_tets:
        v4 = el.tet_verts[t]
        for k in range(4):
            m = t2f[t, k]
            for l in range(4):
                n = t2f[t, l]
                qf = _tet_quad_form(v4, v4[k], v4[l])
                Zp[rix(m), cix(n)] += (chi[t, k] * psi[t, l] / eps[t] * t2s[t, k] * t2s[t, l]
                                       * area[m] * area[n] / (9.0 * vol[t] ** 2) * qf)
    return Zp[:-1, :-1].copy()


def rhs(topo, wave, pol, rows=None):
    """b_m = <f_m, E^i> with the degree-5 tetrahedron rule."""
    N = topo.N
    lam5, w5 = Q.tet_deg5()
    e = wave.pol_vector(pol)
    L = np.array([topo.a, topo.b])
    kt = np.array([wave.kx, wave.ky])
    chi = np.exp(1j * (topo.t2shift @ (kt * L)))
    b = np.zeros(N, complex)
    for t in range(len(topo.tets)):
        v4 = topo.verts[topo.tets[t]]
        X = lam5 @ v4
        Ei = np.exp(-1j * (X @ wave.kinc))[:, None] * e[None, :]
        for k in range(4):
            m = topo.t2f[t, k]
            val = np.sum(w5 * topo.vol[t] * np.einsum("qd,qd->q", X - v4[k], Ei))
            b[m] += chi[t, k] * topo.t2s[t, k] * topo.area[m] / (3.0 * topo.vol[t]) * val
    return b if rows is None else b[rows]


# ---------------------------------------------------------------- solves
def solve_lu(Z, b):
    return sla.lu_solve(sla.lu_factor(Z), b)


def gmres_right_block(Z, b, blocks, tol=1e-12, restart=100, maxit=2000):
    """Right-preconditioned restarted GMRES (Sec. 2.3, Eq. 6 with the block
    inverse applied on the right; Sec. 3 for GMRES), x0 = 0, classical
    Gram-Schmidt applied twice, Givens rotations.  `blocks` = [(start, end)]
    diagonal blocks of the preconditioner.  Returns x, iterations, history
    of the relative residual estimate, converged flag."""
    N = len(b)
    facs = [(s, e, sla.lu_factor(Z[s:e, s:e])) for (s, e) in blocks if e > s]

    def Minv(v):
        out = v.copy()
        for s, e, f in facs:
            out[s:e] = sla.lu_solve(f, v[s:e])
        return out

    x = np.zeros(N, complex)
    bnorm = np.linalg.norm(b)
    hist = []
    it = 0
    while True:
        r = b - Z @ x
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or it >= maxit:
            return x, it, hist, beta / bnorm <= tol
        V = np.zeros((N, restart + 1), complex)
        H = np.zeros((restart + 1, restart), complex)
        cs = np.zeros(restart, complex); sn = np.zeros(restart, complex)
        g = np.zeros(restart + 1, complex); g[0] = beta
        V[:, 0] = r / beta
        j_end = 0
        for j in range(restart):
            w = Z @ Minv(V[:, j])
            h = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0:
                V[:, j + 1] = w / hn
            for i in range(j):
                t1 = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t1
            den = np.hypot(abs(H[j, j]), abs(H[j + 1, j]))
            cs[j] = H[j, j] / den if den > 0 else 1.0
            sn[j] = H[j + 1, j] / den if den > 0 else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            it += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or it >= maxit:
                break
        y = sla.solve_triangular(H[:j_end, :j_end], g[:j_end])
        x = x + Minv(V[:, :j_end] @ y)


# --------------------------------------------------------------- outputs
def tet_field_coeffs(topo, wave, x):
    """c[t, k] such that D~ on tet t = sum_k c[t,k] (r - v_k)."""
    L = np.array([topo.a, topo.b])
    kt = np.array([wave.kx, wave.ky])
    psi = np.exp(-1j * (topo.t2shift @ (kt * L)))
    return (x[topo.t2f] * psi * topo.t2s * topo.area[topo.t2f]
            / (3.0 * topo.vol[:, None]))


def absorptance(topo, wave, eps_in, x):
    """Absorbed fraction of the incident power per domain (Sec. 3, Eq. 7,
    normalised by the power cos(theta) a b |E0|^2 / (2 eta0) crossing the cell):
    A_d = k0 sum_{T in d} (-Im eps_T) / |eps_T|^2 I_T |D~|^2 dV / (cos th a b)."""
    eps = internal_eps(eps_in)
    c = tet_field_coeffs(topo, wave, x)
    out = np.zeros(topo.ndom)
    for t in range(len(topo.tets)):
        v4 = topo.verts[topo.tets[t]]
        s = 0.0 + 0.0j
        for k in range(4):
            for l in range(4):
                s += c[t, k] * np.conj(c[t, l]) * _tet_quad_form(v4, v4[k], v4[l])
        out[topo.dom[t]] += (-eps[t].imag) / abs(eps[t]) ** 2 * s.real
    return out * wave.k0 / (np.cos(wave.theta) * topo.a * topo.b)


def locate_points(topo, points, tol=1e-12):
    """Tetrahedron holding each point (-1 if none): the lowest index among the
    tetrahedra whose barycentric coordinates of the point are all >= -tol."""
    V = topo.verts[topo.tets]                                   # [nt, 4, 3]
    M = np.transpose(V[:, 1:, :] - V[:, :1, :], (0, 2, 1))      # columns v_k - v_0
    Minv = np.linalg.inv(M)
    out = np.full(len(points), -1, np.int64)
    for i, p in enumerate(np.asarray(points, float)):
        lam = np.einsum("tij,tj->ti", Minv, p[None, :] - V[:, 0, :])
        inside = np.flatnonzero(np.all(lam >= -tol, axis=1) & (lam.sum(axis=1) <= 1.0 + tol))
        if len(inside):
            out[i] = inside[0]
    return out


def field_at(topo, wave, eps_in, x, points):
    """The field of the solution inside the structure (Sec. 3, the field maps
    behind Fig. 5): at each point, E~ = D~ / eps_T with D~ = sum_k c_k (r - v_k)
    on the tetrahedron T holding it (internal convention, |E0| = 1).  Returns
    (E [npts, 3] complex, tet [npts]); points outside every tetrahedron get
    tet -1 and E = 0."""
    eps = internal_eps(eps_in)
    c = tet_field_coeffs(topo, wave, x)
    pts = np.asarray(points, float)
    tet = locate_points(topo, pts)
    E = np.zeros((len(pts), 3), complex)
    for i, t in enumerate(tet):
        if t < 0:
            continue
        v4 = topo.verts[topo.tets[t]]
        D = sum(c[t, k] * (pts[i] - v4[k]) for k in range(4))
        E[i] = D / eps[t]
    return E, tet


def absorptance_per_tet(topo, wave, eps_in, x):
    """Each tetrahedron's term of Eq. 7 (Sec. 3) with the normalisation of
    absorptance(): k0 (-Im eps_T)/|eps_T|^2 I_T |D~|^2 dV / (cos th a b), so the
    terms of a domain add up to its absorptance.  Divided by V_T it is the
    absorption density mapped in Sec. 3 (Fig. 5)."""
    eps = internal_eps(eps_in)
    c = tet_field_coeffs(topo, wave, x)
    out = np.zeros(len(topo.tets))
    for t in range(len(topo.tets)):
        v4 = topo.verts[topo.tets[t]]
        s = 0.0 + 0.0j
        for k in range(4):
            for l in range(4):
                s += c[t, k] * np.conj(c[t, l]) * _tet_quad_form(v4, v4[k], v4[l])
        out[t] = (-eps[t].imag) / abs(eps[t]) ** 2 * s.real
    return out * wave.k0 / (np.cos(wave.theta) * topo.a * topo.b)


def reflect_transmit(topo, wave, eps_in, x, pol, P=4):
    """Floquet-mode reflectance and transmittance (sum over propagating orders)
    of the radiated field of P~ = kappa D~ plus the incident wave."""
    eps = internal_eps(eps_in)
    kappa = 1.0 - 1.0 / eps
    c = tet_field_coeffs(topo, wave, x)
    lam5, w5 = Q.tet_deg5()
    k0, a, b = wave.k0, topo.a, topo.b
    e_inc = wave.pol_vector(pol)
    beta00 = k0 * np.cos(wave.theta)
    pts = np.einsum("qk,tkd->tqd", lam5, topo.verts[topo.tets])          # [nt,14,3]
    wts = w5[None, :] * topo.vol[:, None]
    # D~ at the points: sum_k c_k (X - v_k)
    D = np.einsum("tk,tqkd->tqd", c, pts[:, :, None, :] - topo.verts[topo.tets][:, None, :, :])
    Pt = kappa[:, None, None] * D
    R = 0.0; T = 0.0
    for p in range(-P, P + 1):
        for q in range(-P, P + 1):
            ktx = wave.kx + 2 * np.pi * p / a
            kty = wave.ky + 2 * np.pi * q / b
            kt2 = ktx * ktx + kty * kty
            if kt2 >= k0 * k0:
                continue
            beta = np.sqrt(k0 * k0 - kt2)
            gam = 1j * beta
            for sgn in (+1, -1):
                kv = np.array([ktx, kty, sgn * beta])
                ph = np.exp(1j * (pts @ kv))
                v = np.einsum("tq,tq,tqd->d", wts, ph, Pt)
                e = (k0 * k0 * v - kv * (kv @ v)) / (2 * a * b * gam)
                if sgn < 0 and p == 0 and q == 0:
                    e = e + e_inc
                if sgn > 0:
                    R += np.vdot(e, e).real * beta / beta00
                else:
                    T += np.vdot(e, e).real * beta / beta00
    return R, T
