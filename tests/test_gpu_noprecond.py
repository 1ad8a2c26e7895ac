"""GMRES without a preconditioner (VIE_OPT_PRECOND = 1, M = I): the reference
against which Sec. 3 (Figs. 2-3) measures the block-diagonal preconditioner;
and with the point-Jacobi scaling M = diag(Z) (VIE_OPT_PRECOND = 2) against
the oracle's GMRES with 1 x 1 diagonal blocks.

The library's unpreconditioned solve is compared with the oracle's GMRES on
the same Z with no blocks (M = I): iteration count, the residual history's
first iterations and the solution, at a restart length that converges in one
cycle and at a shorter one that needs several.  The block preconditioner
must need fewer iterations on the same fill; the paired solve, graph replays
and the option's checks are covered as for the preconditioned path."""
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


@pytest.fixture(scope="module")
def case():
    m = osc_small()
    lam = 480.0
    eps = eps_for(m, lam)
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    wave = OV.make_wave(lam, 0.0, 0.0)
    Zo = OV.assemble(t, wave, eps)
    return m, lam, eps, t, wave, Zo


def unpreconditioned(vie, m, lam, eps, prec, restart):
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, restart)
    s.set_option(vie.VIE_OPT_PRECOND, 1)
    assert s.get_option(vie.VIE_OPT_PRECOND) == 1
    s.fill(lam, 0.0, 0.0, eps)   # no factorisation: M = I needs none
    return s


@pytest.mark.parametrize("restart", [200, 100])
def test_no_precond_matches_oracle(vie, case, restart):
    m, lam, eps, t, wave, Zo = case
    tol = 1e-8
    for pol in (0, 1):
        xo, it, hist, ok = OV.gmres_right_block(Zo, OV.rhs(t, wave, pol), [], tol=tol, restart=restart, maxit=2000)
        assert ok
        s = unpreconditioned(vie, m, lam, eps, vie.VIE_FP64, restart)
        info = s.solve(pol, tol=tol, max_iter=2000, restart=restart)
        assert info["converged"] and abs(info["iters"] - it) <= 2, (pol, info["iters"], it)
        h = s.residual_history()
        n = min(60, len(h), len(hist))
        assert np.allclose(h[:n], hist[:n], rtol=1e-6, atol=0), (pol, np.max(np.abs(h[:n] / np.array(hist[:n]) - 1)))
        x = s.read_solution()
        assert np.linalg.norm(x - xo) < 1e-5 * np.linalg.norm(xo), pol
        assert info["true_rel_residual"] < 10 * tol


def test_block_preconditioner_needs_fewer_iterations(vie, case):
    m, lam, eps, t, wave, Zo = case
    s = unpreconditioned(vie, m, lam, eps, vie.VIE_FP64, 200)
    none = s.solve(0, tol=1e-8, max_iter=2000, restart=200)
    xn = s.read_solution()
    s.set_option(vie.VIE_OPT_PRECOND, 0)
    with pytest.raises(vie.VieError) as e:   # the block preconditioner needs its factors
        s.solve(0, tol=1e-8, max_iter=2000, restart=200)
    assert e.value.code == vie.VIE_ESTATE
    s.factor()
    blk = s.solve(0, tol=1e-8, max_iter=2000, restart=200)
    xb = s.read_solution()
    assert none["converged"] and blk["converged"] and blk["iters"] < none["iters"], (blk["iters"], none["iters"])
    # Eq. 8 between the two solutions: both solve Z x = b to the tolerance
    assert np.linalg.norm(xb - xn) < 1e-5 * np.linalg.norm(xn)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_no_precond_pair_matches_single_solves(vie, case, precision):
    m, lam, eps, t, wave, Zo = case
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    s = unpreconditioned(vie, m, lam, eps, prec, 100)
    single = []
    for pol in (0, 1):
        info = s.solve(pol, tol=1e-8, max_iter=2000, restart=100)
        single.append((info["iters"], s.read_solution()))
    pair = s.solve_pair(tol=1e-8, max_iter=2000, restart=100)
    for pol in (0, 1):
        assert pair[pol]["iters"] == single[pol][0]
        assert np.array_equal(s.read_solution(pol), single[pol][1]), pol


def test_no_precond_graph_replays_match_plain(vie, case):
    m, lam, eps, t, wave, Zo = case
    s = unpreconditioned(vie, m, lam, eps, vie.VIE_FP64, 100)
    ref = s.solve(1, tol=1e-8, max_iter=2000, restart=100)
    x0, h0 = s.read_solution(), s.residual_history()
    s.set_option(vie.VIE_OPT_GRAPH_STEPS, 8)
    for rep in range(2):
        info = s.solve(1, tol=1e-8, max_iter=2000, restart=100)
        assert info["iters"] == ref["iters"] and info["restarts"] == ref["restarts"], rep
        assert np.array_equal(s.read_solution(), x0) and np.array_equal(s.residual_history(), h0), rep


def test_precond_option_checks(vie):
    s = vie.Solver()
    assert s.get_option(vie.VIE_OPT_PRECOND) == 0
    for bad in (3, -1):
        with pytest.raises(vie.VieError) as e:
            s.set_option(vie.VIE_OPT_PRECOND, bad)
        assert e.value.code == vie.VIE_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_jacobi_matches_oracle(vie, case, prec):
    """VIE_OPT_PRECOND = 2, M = diag(Z): the oracle's right-preconditioned
    GMRES with 1 x 1 diagonal blocks is the same method on the same Z."""
    m, lam, eps, t, wave, Zo = case
    tol, restart = 1e-8, 60
    ones = [(i, i + 1) for i in range(t.N)]
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64 if prec == "fp64" else vie.VIE_MIXED_FP32, restart)
    s.set_option(vie.VIE_OPT_PRECOND, 2)
    s.fill(lam, 0.0, 0.0, eps)   # no factorisation: M = diag(Z) needs none
    for pol in (0, 1):
        xo, it, hist, ok = OV.gmres_right_block(Zo, OV.rhs(t, wave, pol), ones, tol=tol, restart=restart, maxit=2000)
        assert ok
        _, it_none, _, _ = OV.gmres_right_block(Zo, OV.rhs(t, wave, pol), [], tol=tol, restart=restart, maxit=2000)
        info = s.solve(pol, tol=tol, max_iter=2000, restart=restart)
        print(f"  {prec} pol {pol}: jacobi {info['iters']} iterations (oracle {it}, oracle with M = I {it_none})",
              flush=True)
        assert info["converged"] and abs(info["iters"] - it) <= 2, (pol, info["iters"], it)
        assert it < it_none
        x = s.read_solution()
        bar = 1e-5 if prec == "fp64" else 1e-4
        assert np.linalg.norm(x - xo) < bar * np.linalg.norm(xo), pol
        if prec == "fp64":
            h = s.residual_history()
            n = min(40, len(h), len(hist))
            assert np.allclose(h[:n], hist[:n], rtol=1e-6, atol=0)
