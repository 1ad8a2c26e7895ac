"""Per-tetrahedron absorption (vie_absorption_per_tet): each tetrahedron's
term of Eq. 7, the quantity behind the absorption maps of Sec. 3 (Fig. 5).
Compared with the oracle's terms for the oracle's solution of the same case,
and the library's own domain sums against vie_absorption."""
import numpy as np
import pytest

from oracle import topology as OT
from oracle import vie as OV

from gpu_cases import eps_for, osc_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_tet_absorption_matches_oracle(vie, precision):
    m = osc_small()
    lam, th, ph = 520.0, 0.3, 0.2
    eps = eps_for(m, lam)
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    wave = OV.make_wave(lam, th, ph)
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, 60)
    s.fill(lam, th, ph, eps)
    s.factor()
    per_pol = {}
    for pol in (0, 1):
        s.solve(pol, tol=1e-11, max_iter=500, restart=60)
        per = s.absorption_per_tet()
        A, _, _ = s.absorption()
        assert per.shape == (len(m.tets),)
        for d in range(m.ndom):
            assert abs(per[m.tet_domain == d].sum() - A[d]) <= 1e-12 * np.abs(A).max(), d
        per_pol[pol] = per
        Zo = OV.assemble(t, wave, eps)
        xo = OV.solve_lu(Zo, OV.rhs(t, wave, pol))
        po = OV.absorptance_per_tet(t, wave, eps, xo)
        bound = (1e-7 if precision == "fp64" else 1e-4) * po.max()
        assert np.max(np.abs(per - po)) <= bound, (pol, np.max(np.abs(per - po)) / po.max())
    # after a paired solve both polarisations are reachable
    s.solve_pair(tol=1e-11, max_iter=500, restart=60)
    for pol in (0, 1):
        assert np.max(np.abs(s.absorption_per_tet(pol) - per_pol[pol])) <= 1e-9 * per_pol[pol].max()


def test_per_tet_absorption_needs_a_solve(vie):
    m = osc_small()
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 20)
    s.fill(520.0, 0.0, 0.0, eps_for(m, 520.0))
    with pytest.raises(vie.VieError) as e:
        s.absorption_per_tet()
    assert e.value.code == vie.VIE_ESTATE
