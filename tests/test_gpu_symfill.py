"""Normal-incidence fill with one evaluation per unordered far pair
(VIE_OPT_SYM_FILL).

At kt = 0 the lattice sum is even in the separation, so the moments of a far
tetrahedron pair (T, S) also give those of (S, T).  The symmetric fill must
give the oracle's Z to the usual tolerance (|dZ| <= 1e-10 max(|Z_ij|, 1e-5
max|Z|)), the plain fill's Z to rounding (FP64) or to the FP32 rounding of
far entries (mixed), the same solutions, and evaluate half the far pairs.
The far (half-SWG face, tet) entries come from the tet-face kernel's
evaluation of the same pair, written transposed into the staging copy.
At oblique incidence the option also evaluates each unordered far pair once:
g_p at the reversed separations is the conjugate of g_p at the separations
plus a term of the propagating Floquet orders, so the swapped pair's
moments come from the same lattice sums; checked the same way, including a
cell where a non-specular order propagates."""
import numpy as np
import pytest

from oracle import topology as OT
from oracle import vie as OV

from gpu_cases import eps_for, osc_rect, osc_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


def solver(vie, m, prec, sym, restart=40):
    s = vie.Solver()
    s.upload_mesh(m)
    if sym:
        s.set_option(vie.VIE_OPT_SYM_FILL, 1)
    assert s.get_option(vie.VIE_OPT_SYM_FILL) == int(sym)
    s.bind(prec, restart)
    return s


def full_Z(s):
    N = s.num_unknowns()
    r, c = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return s.read_Z(r.ravel(), c.ravel()).reshape(N, N)


@pytest.mark.parametrize("case", ["osc_small", "osc_rect"])
def test_symmetric_fill_matches_oracle_and_plain_fill(vie, case):
    m = {"osc_small": osc_small, "osc_rect": osc_rect}[case]()
    lam = 520.0
    eps = eps_for(m, lam)
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    Zo = OV.assemble(t, OV.make_wave(lam, 0.0, 0.0), eps)
    scale = np.abs(Zo).max()
    # the structure's top and bottom faces are half-SWGs: their rows take the
    # swapped (face, tet) entries of the tet-face kernel
    assert t.is_half.sum() > 0
    for prec in (vie.VIE_FP64, vie.VIE_MIXED_FP32):
        sp = solver(vie, m, prec, False)
        ss = solver(vie, m, prec, True)
        assert ss.workspace_bytes(prec, 40) > sp.workspace_bytes(prec, 40)
        sp.fill(lam, 0.0, 0.0, eps)
        ss.fill(lam, 0.0, 0.0, eps)
        fp, fs = sp.fill_stats(), ss.fill_stats()
        assert fp["far_symmetric"] == 0 and fs["far_symmetric"] == 1
        assert 2 * fs["far_pairs"] == fp["far_pairs"] and fs["far_launches"] < fp["far_launches"]
        Zp, Zs = full_Z(sp), full_Z(ss)
        if prec == vie.VIE_FP64:
            bad = np.abs(Zs - Zo) > 1e-10 * np.maximum(np.abs(Zo), 1e-5 * scale)
            assert not bad.any(), np.max(np.abs(Zs - Zo) / np.maximum(np.abs(Zo), 1e-5 * scale))
            assert np.max(np.abs(Zs - Zp)) < 1e-13 * scale
        else:
            # far entries in complex FP32 on both sides, summed in another order
            assert np.max(np.abs(Zs - Zo)) < 1e-6 * scale
            assert np.max(np.abs(Zs - Zp)) < 1e-6 * scale
        for s in (sp, ss):
            s.factor()
        ip = sp.solve_pair(tol=1e-10, max_iter=300, restart=40)
        is_ = ss.solve_pair(tol=1e-10, max_iter=300, restart=40)
        for p in (0, 1):
            assert ip[p]["converged"] and is_[p]["converged"]
            xp, xs = sp.read_solution(p), ss.read_solution(p)
            tol = 1e-9 if prec == vie.VIE_FP64 else 1e-5
            assert np.linalg.norm(xs - xp) < tol * np.linalg.norm(xp), (prec, p)


def grating():
    """A 300 x 240 nm cell, two layers of 3 x 3 bricks: at 500 nm, 55 deg
    the (-1, 0) order propagates."""
    from paper_1809_05334_amd import workloads as W
    xs, ys, zs = np.linspace(0, 300.0, 4), np.linspace(0, 240.0, 4), np.array([0.0, 30.0, 60.0])
    verts, tets = W.brick_grid_mesh(xs, ys, zs)
    c = W.centroids(verts, tets)
    dom = np.where(c[:, 2] < 30.0, 1, 0).astype(np.int32)
    dom[(c[:, 2] > 30.0) & (c[:, 0] < 100.0)] = 0
    return W.Mesh(verts, tets, dom, 2, 300.0, 240.0, (xs, ys, zs), {"kind": "grating"})


@pytest.mark.parametrize("case", ["osc_small", "osc_rect", "grating"])
def test_oblique_symmetric_fill(vie, case):
    m = {"osc_small": osc_small, "osc_rect": osc_rect, "grating": grating}[case]()
    lam, th, ph = (500.0, np.deg2rad(55.0), np.deg2rad(20.0)) if case == "grating" else (480.0, 0.5, 0.3)
    if case == "grating":
        eps = np.array([4.0 + 0.3j, 2.3 + 0.05j])[m.tet_domain]
    else:
        eps = eps_for(m, lam)
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    wave = OV.make_wave(lam, th, ph)
    Zo = OV.assemble(t, wave, eps)
    scale = np.abs(Zo).max()
    for prec in (vie.VIE_FP64, vie.VIE_MIXED_FP32):
        sp = solver(vie, m, prec, False)
        ss = solver(vie, m, prec, True)
        sp.fill(lam, th, ph, eps)
        ss.fill(lam, th, ph, eps)
        fp, fs = sp.fill_stats(), ss.fill_stats()
        assert fp["far_symmetric"] == 0 and fs["far_symmetric"] == 1
        assert 2 * fs["far_pairs"] == fp["far_pairs"]
        Zp, Zs = full_Z(sp), full_Z(ss)
        if prec == vie.VIE_FP64:
            bad = np.abs(Zs - Zo) > 1e-10 * np.maximum(np.abs(Zo), 1e-5 * scale)
            assert not bad.any(), np.max(np.abs(Zs - Zo) / np.maximum(np.abs(Zo), 1e-5 * scale))
            assert np.max(np.abs(Zs - Zp)) < 1e-13 * scale
        else:
            assert np.max(np.abs(Zs - Zo)) < 1e-6 * scale
            assert np.max(np.abs(Zs - Zp)) < 1e-6 * scale
        for s in (sp, ss):
            s.factor()
        ip = sp.solve_pair(tol=1e-10, max_iter=300, restart=40)
        is_ = ss.solve_pair(tol=1e-10, max_iter=300, restart=40)
        for p in (0, 1):
            assert ip[p]["converged"] and is_[p]["converged"]
            xp, xs = sp.read_solution(p), ss.read_solution(p)
            tol = 1e-9 if prec == vie.VIE_FP64 else 1e-5
            assert np.linalg.norm(xs - xp) < tol * np.linalg.norm(xp), (prec, p)


def test_option_is_refused_after_bind(vie):
    m = osc_small()
    s = solver(vie, m, vie.VIE_FP64, False)
    with pytest.raises(vie.VieError) as e:
        s.set_option(vie.VIE_OPT_SYM_FILL, 1)
    assert e.value.code == vie.VIE_ESTATE
