"""Served and batched solves against the oracle (Sec. 3, Eq. 7 absorptance per
domain; R and T over the propagating Floquet orders).

Five cells of the batched/served workload (Drude-Ag sphere in a spacer over
an active layer, N = 1,250-2,450, oblique incidence, random polarisation; one
at an incidence where the (p, q) != (0, 0) order propagates) go through the
serving loop with three slots (arrivals staggered so that they overlap) and
through the batch driver, on the mixed and the FP64 path.  The expected
values are the oracle's LU solutions, written by
tests/golden/make_served_oracle.py.  Bars: absorptance, R and T within 1e-4
of the oracle on the mixed path, 1e-8 on the FP64 path."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "served_oracle.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)["requests"]


def requests(gold, spacing):
    keys = ("rid", "cell", "lambda", "theta", "phi", "pol")
    return [dict({k: g[k] for k in keys}, arrival=spacing * i) for i, g in enumerate(gold)]


def check(results, gold, bar):
    assert len(results) == len(gold)
    for r, g in zip(results, gold):
        assert r.ok, r.error
        assert r.N == g["N"]
        dA = max(float(np.max(np.abs(np.array(r.A) - np.array(g["A"])))), abs(r.R - g["R"]), abs(r.T - g["T"]))
        print(f"  rid {r.rid}: N={r.N} orders={len(g['orders'])} iters={r.iters} dA={dA:.2e}", flush=True)
        assert dA <= bar, (r.rid, dA)


def test_golden_covers_a_diffracting_cell(gold):
    assert any(len(g["orders"]) > 1 for g in gold)
    assert all(1000 <= g["N"] <= 2500 for g in gold)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_solves_match_oracle(gold, precision):
    from paper_1809_05334_amd import serve as S
    from paper_1809_05334_amd import vie
    prec = vie.VIE_MIXED_FP32 if precision == "mixed" else vie.VIE_FP64
    print(f"served {precision}", flush=True)
    be = S.VieBackend(precision=prec, tol=1e-8 if precision == "mixed" else 1e-11, restart=100)
    srv = S.Server(be, slots=3, hbm_budget=100e9)
    res = srv.run_trace(requests(gold, 0.02))
    assert srv.peak_running >= 2
    check(res, gold, 1e-4 if precision == "mixed" else 1e-8)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_solves_match_oracle(gold, precision):
    from paper_1809_05334_amd import batch as B
    from paper_1809_05334_amd import vie
    prec = vie.VIE_MIXED_FP32 if precision == "mixed" else vie.VIE_FP64
    print(f"batched {precision}", flush=True)
    res, dt, _ = B.run_batch(requests(gold, 0.0), prec, slots=3, budget_gb=100.0,
                             tol=1e-8 if precision == "mixed" else 1e-11, restart=100)
    check(res, gold, 1e-4 if precision == "mixed" else 1e-8)
