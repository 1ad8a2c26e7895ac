"""Full-size cases.  The timed workload: the plasmonic cell (200 x 200 nm,
18,432 tetrahedra, N = 37,376) filled as the bench fills it (normal incidence,
one evaluation per unordered far pair), on both precision paths.

Checked on outputs the oracle computes one by one at this size (sampled Z
entries: far pairs, touching pairs around the sampled rows, face terms and
the diagonal; the whole right-hand side) and on properties that hold at any
size: the paired solve's true residuals, the energy balance of absorptance
plus R plus T, and TE = TM at normal incidence on this square cell, which is
symmetric under the exchange of x and y."""
import numpy as np
import pytest

from oracle import topology as OT
from oracle import vie as OV
from paper_1809_05334_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


@pytest.fixture(scope="module")
def cell():
    m = W.plasmonic_cell_mesh()
    return m, OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_full_size_cell_as_benched(vie, cell, precision):
    m, t = cell
    assert t.N == 37376
    lam = 450.0
    eps = W.osc_eps(m, lam)
    wave = OV.make_wave(lam, 0.0, 0.0)
    prec = vie.VIE_MIXED_FP32 if precision == "mixed" else vie.VIE_FP64
    s = vie.Solver()
    s.upload_mesh(m)
    s.set_option(vie.VIE_OPT_SYM_FILL, 1)
    s.bind(prec, 200)
    s.fill(lam, 0.0, 0.0, eps)
    assert s.fill_stats()["far_symmetric"] == 1

    rng = np.random.default_rng(7)
    rows = rng.choice(t.N, 24, replace=False)
    near = np.unique(t.t2f[t.tplus[rows[:8]]].ravel())   # faces of the sampled rows' tetrahedra: touching pairs
    cols = np.unique(np.concatenate([rows, near, rng.choice(t.N, 24, replace=False)]))
    Zo = OV.assemble(t, wave, eps, rows=rows, cols=cols)
    r, c = np.meshgrid(rows, cols, indexing="ij")
    Zg = s.read_Z(r.ravel(), c.ravel()).reshape(len(rows), len(cols))
    scale = np.abs(Zo).max()
    if precision == "fp64":
        bad = np.abs(Zg - Zo) > 1e-10 * np.maximum(np.abs(Zo), 1e-5 * scale)
        assert not bad.any(), np.max(np.abs(Zg - Zo) / np.maximum(np.abs(Zo), 1e-5 * scale))
    else:
        assert np.max(np.abs(Zg - Zo)) < 1e-6 * scale

    s.factor()
    info = s.solve_pair(tol=1e-8, max_iter=2000, restart=200)
    b = s.read_rhs()   # the last polarisation of the pair: TM
    bo = OV.rhs(t, wave, 1)
    assert np.max(np.abs(b - bo)) < 1e-12 * np.abs(bo).max()
    out = []
    for pol in (0, 1):
        assert info[pol]["converged"] and info[pol]["true_rel_residual"] < 2e-8, info[pol]
        A, R, T = s.absorption(pol=pol)
        assert abs(A.sum() + R + T - 1.0) < 1e-2, (A, R, T)
        assert np.all(A >= 0) and R >= 0 and T >= 0
        out.append((A, R, T))
    # the mirror maps Z onto itself exactly, but the mixed path rounds the
    # mirrored far entries to FP32 independently: symmetry to that rounding
    sym = 1e-9 if precision == "fp64" else 1e-6
    assert abs(info[0]["iters"] - info[1]["iters"]) <= (0 if precision == "fp64" else 2)
    assert np.max(np.abs(out[0][0] - out[1][0])) < sym * out[0][0].max()
    assert abs(out[0][1] - out[1][1]) < sym and abs(out[0][2] - out[1][2]) < sym


def test_precision_form_at_full_size(vie):
    """The precision form of the cell (3.33 nm over the particle and spacer,
    38,400 tetrahedra, N = 77,600) at one oblique incidence: the mixed path's
    sampled Z entries against the oracle, then absorptance per domain, R and T
    of both polarisations against the FP64 path on the same inputs."""
    m = W.plasmonic_cell_fine_mesh()
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    assert t.N == 77600
    lam, th, ph = 550.0, np.deg2rad(40.0), np.deg2rad(45.0)
    eps = W.osc_eps(m, lam)
    wave = OV.make_wave(lam, th, ph)
    rng = np.random.default_rng(11)
    rows = rng.choice(t.N, 16, replace=False)
    cols = np.unique(np.concatenate([rows, t.t2f[t.tplus[rows[:6]]].ravel(), rng.choice(t.N, 16, replace=False)]))
    Zo = OV.assemble(t, wave, eps, rows=rows, cols=cols)
    out = {}
    for name, prec in (("mixed", vie.VIE_MIXED_FP32), ("fp64", vie.VIE_FP64)):
        s = vie.Solver()
        s.upload_mesh(m)
        s.bind(prec, 150)
        s.fill(lam, th, ph, eps)
        if name == "mixed":
            r, c = np.meshgrid(rows, cols, indexing="ij")
            Zg = s.read_Z(r.ravel(), c.ravel()).reshape(len(rows), len(cols))
            assert np.max(np.abs(Zg - Zo)) < 1e-6 * np.abs(Zo).max()
        s.factor()
        info = s.solve_pair(tol=1e-8, max_iter=3000, restart=150)
        assert all(i["converged"] for i in info), info
        out[name] = [s.absorption(pol=p) for p in (0, 1)]
        s.close()   # free this path's workspace before the next
    for pol in (0, 1):
        (Am, Rm, Tm), (Af, Rf, Tf) = out["mixed"][pol], out["fp64"][pol]
        d = max(np.max(np.abs(Am - Af)), abs(Rm - Rf), abs(Tm - Tf))
        assert d < 1e-6, (pol, d)
