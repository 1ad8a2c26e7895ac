"""Mixed-precision path (VIE_MIXED_FP32) against the oracle and the FP64 path.

The mixed operator stores the far part of Z in complex FP32 and the
touching-pair (singular, near-neighbour and mass) contributions in FP64, and
runs every Krylov operation in FP64 on that operator.  Bounds:
  * Z entries: each far contribution is rounded once to FP32 (relative
    2^-24) and an entry sums at most a few dozen of them, so
    |dZ| <= 1e-6 max|Z| (the FP64 near part adds nothing);
  * absorptance, R and T: |dA| <= 1e-4 against the oracle (the target for the
    mixed path), and the mixed and FP64 GPU results agree to 1e-6;
  * the GMRES true residual (FP64, on the mixed operator) meets tol.
"""
import numpy as np
import pytest

from oracle import topology as OT
from oracle import vie as OV
from paper_1809_05334_amd import workloads as W

from gpu_cases import eps_for, osc_rect, osc_small, slab_100nm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


CASES = {"slab_100nm": slab_100nm, "osc_small": osc_small, "osc_rect": osc_rect}
ILLUM = {"slab_100nm": (600.0, 0.5, 0.3), "osc_small": (520.0, 0.35, 0.6), "osc_rect": (450.0, 0.6, 1.1)}


def solver(vie, m, precision, restart=60):
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(precision, restart)
    return s


def test_mixed_workspace_is_smaller(vie):
    m = W.slab_mesh(nx=8, ny=8, nz=4)
    s = vie.Solver()
    s.upload_mesh(m)
    b64 = s.workspace_bytes(vie.VIE_FP64, 50)
    b32 = s.workspace_bytes(vie.VIE_MIXED_FP32, 50)
    N = s.num_unknowns()
    assert b32 < b64
    assert b64 - b32 > 0.8 * 8 * N * N    # the dense Z at half the bytes, less the near part


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_matches_oracle(vie, name):
    m = CASES[name]()
    lam, th, ph = ILLUM[name]
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    eps = eps_for(m, lam)
    s = solver(vie, m, vie.VIE_MIXED_FP32)
    s.fill(lam, th, ph, eps)
    N = t.N
    r, c = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    Zg = s.read_Z(r.ravel(), c.ravel()).reshape(N, N)
    wave = OV.make_wave(lam, th, ph)
    Zo = OV.assemble(t, wave, eps)
    err = np.abs(Zg - Zo).max() / np.abs(Zo).max()
    assert err < 1e-6, err
    assert err > 0.0          # the far part really is stored in FP32
    s.factor()
    for pol in (0, 1):
        info = s.solve(pol, tol=1e-10, max_iter=500, restart=60)
        assert info["converged"] and info["true_rel_residual"] < 1e-9
        A, R, T = s.absorption()
        xo = OV.solve_lu(Zo, OV.rhs(t, wave, pol))
        Ao = OV.absorptance(t, wave, eps, xo)
        Ro, To = OV.reflect_transmit(t, wave, eps, xo, pol)
        dA = max(np.max(np.abs(A - Ao)), abs(R - Ro), abs(T - To))
        assert dA < 1e-4, (A, Ao, R, Ro, T, To)


def test_mixed_matches_fp64_path_on_multiblock_cell(vie):
    """3-domain 8x8x4 slab (N = 3,200): mixed vs FP64 GPU path, same sweep point."""
    m = W.slab_mesh(nx=8, ny=8, nz=4)
    c = W.centroids(m.verts, m.tets)
    m.tet_domain = np.digitize(c[:, 2], [15.0, 32.0]).astype(np.int32)
    m.ndom = 3
    out = {}
    for prec in (vie.VIE_FP64, vie.VIE_MIXED_FP32):
        s = solver(vie, m, prec)
        s.fill(600.0, 0.3, 0.2, W.slab_eps(m))
        s.factor()
        info = s.solve(1, tol=1e-10, max_iter=300, restart=30)
        assert info["converged"]
        out[prec] = (s.absorption(), info["iters"])
    (A64, R64, T64), it64 = out[vie.VIE_FP64]
    (A32, R32, T32), it32 = out[vie.VIE_MIXED_FP32]
    assert np.max(np.abs(A32 - A64)) < 1e-6 and abs(R32 - R64) < 1e-6 and abs(T32 - T64) < 1e-6
    assert abs(it32 - it64) <= 2
