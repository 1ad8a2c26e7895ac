"""Served solves on the GPU: requests admitted while others run give the same
absorptance, R and T as the same requests solved alone.

Every kernel of the path is deterministic (fixed reduction orders, no
floating-point atomics), so concurrency on separate streams must not change
any result: the bound is 1e-12, far below the 1e-4 target."""
import numpy as np
import pytest

from paper_1809_05334_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import serve as S
    return S


def small_trace(n):
    tr = W.serve_trace(rate=1000.0, n_requests=n, seed=3, large_frac=0.0, n_lo=1000, n_hi=2500)
    return tr


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_results_same_alone_and_in_the_mix(serve, precision):
    from paper_1809_05334_amd import vie
    prec = vie.VIE_MIXED_FP32 if precision == "mixed" else vie.VIE_FP64
    trace = small_trace(6)
    alone = {}
    for r in trace:
        one = dict(r, arrival=0.0)
        srv = serve.Server(serve.VieBackend(precision=prec, tol=1e-9), slots=1, hbm_budget=100e9)
        (res,) = srv.run_trace([one])
        assert res.ok, res.error
        alone[r["rid"]] = res
    srv = serve.Server(serve.VieBackend(precision=prec, tol=1e-9), slots=3, hbm_budget=100e9)
    mix = srv.run_trace(trace)
    assert srv.peak_running >= 2          # requests really overlapped
    for res in mix:
        assert res.ok, res.error
        a = alone[res.rid]
        assert res.N == a.N and res.iters == a.iters
        assert np.max(np.abs(np.array(res.A) - np.array(a.A))) <= 1e-12
        assert abs(res.R - a.R) <= 1e-12 and abs(res.T - a.T) <= 1e-12
        assert 0.0 <= res.R <= 1.0 and 0.0 <= res.T <= 1.0 and min(res.A) >= -1e-9
