"""Two-layer stack on the GPU against the multilayer transfer matrix (closed
form): the library's absorptance per domain, R and T for a planar stack of two
lossy materials, which exercises the surface charge on the interface between
them (Sec. 2.1) and Eq. 7 per domain, at the mesh where the oracle's own
discretisation error is below 1e-4."""
import numpy as np
import pytest

from oracle import fresnel as F
from paper_1809_05334_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_layer_stack_vs_transfer_matrix(vie, precision):
    e1, e2 = 3.6 + 0.6j, 1.8 + 0.3j
    m0 = W.slab_mesh(a=50.0, b=50.0, thickness=50.0, nx=4, ny=4, nz=8)
    c = W.centroids(m0.verts, m0.tets)
    dom = np.where(c[:, 2] >= 25.0, 0, 1).astype(np.int32)   # the wave meets domain 0 (top) first
    m = W.Mesh(m0.verts, m0.tets, dom, 2, 50.0, 50.0, m0.grid)
    eps = np.where(dom == 0, e1, e2).astype(complex)
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, 60)
    for th, ph, pol in ((0.0, 0.0, 0), (30.0, 0.3, 0), (30.0, 0.3, 1), (60.0, 0.3, 1)):
        s.fill(600.0, np.deg2rad(th), ph, eps)
        s.factor()
        info = s.solve(pol, tol=1e-11, max_iter=500, restart=60)
        assert info["converged"]
        A, R, T = s.absorption()
        Rf, Tf, Af = F.multilayer_rta([e1, e2], [25.0, 25.0], 600.0, np.deg2rad(th), pol)
        err = max(abs(A[0] - Af[0]), abs(A[1] - Af[1]), abs(R - Rf), abs(T - Tf))
        assert err < 2e-4, (th, pol, A, R, T, Af, Rf, Tf)
