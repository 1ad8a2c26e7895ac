"""The triangular-solve steps of the preconditioner as one cooperative launch
(VIE_OPT_TRSV_COOP) give exactly the results of one launch per step: the
blocks run the same work items in the same arithmetic order, so the solution,
the iteration count and the residual history must agree bit for bit.  Cases
with 3 domains and with 10 domains (more than one launch's domain slots per
step) in both precisions, and with graph capture on (captured steps use the
per-step launches)."""
import numpy as np
import pytest

from paper_1809_05334_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


def slab(ndom):
    m = W.slab_mesh(nx=8, ny=8, nz=4)
    c = W.centroids(m.verts, m.tets)
    if ndom == 3:
        m.tet_domain = np.digitize(c[:, 2], [15.0, 32.0]).astype(np.int32)
    else:
        xs = np.digitize(c[:, 0], [20.0, 40.0, 60.0, 80.0])
        m.tet_domain = (2 * xs + (c[:, 2] > 25.0)).astype(np.int32)
    m.ndom = ndom
    return m


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ndom", [3, 10])
def test_cooperative_apply_matches_per_step_launches(vie, precision, ndom):
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    m = slab(ndom)
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, 40)
    s.fill(580.0, 0.3, 0.5, W.slab_eps(m, 3.2 + 0.3j))
    s.factor()
    rng = np.random.default_rng(5)
    v = rng.standard_normal(s.num_unknowns()) + 1j * rng.standard_normal(s.num_unknowns())
    z0 = s.precond_apply(v)
    i0 = s.solve(0, tol=1e-10, max_iter=300, restart=40)
    x0, h0 = s.read_solution(), s.residual_history()
    s.set_option(vie.VIE_OPT_TRSV_COOP, 1)
    assert s.get_option(vie.VIE_OPT_TRSV_COOP) == 1
    for rep in range(2):
        assert np.array_equal(s.precond_apply(v), z0)
        info = s.solve(0, tol=1e-10, max_iter=300, restart=40)
        assert info["iters"] == i0["iters"]
        assert np.array_equal(s.read_solution(), x0) and np.array_equal(s.residual_history(), h0)
    # graph capture with the cooperative option set: captured steps use per-step launches
    s.set_option(vie.VIE_OPT_GRAPH_STEPS, 4)
    info = s.solve(0, tol=1e-10, max_iter=300, restart=40)
    assert info["iters"] == i0["iters"] and np.array_equal(s.read_solution(), x0)
