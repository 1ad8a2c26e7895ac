"""Paired TE + TM solve (both polarisations in lockstep).

The pair shares each pass over Z and over the LU factors between the two
GMRES processes, but every sum a process computes runs in the same order as
in a solve of its own, and each process takes its stopping decisions on its
own values.  So each polarisation of a pair must reproduce the single solve
bit for bit (iterations, restarts, residual history, solution, absorptance),
including the cycles where one process has converged and the other goes on
alone, with plain launches, captured graphs and cooperative solves, and at
max_iter."""
import numpy as np
import pytest

from paper_1809_05334_amd import workloads as W

from gpu_cases import eps_for, osc_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vie():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1809_05334_amd import vie as V
    return V


def three_domain_slab():
    m = W.slab_mesh(nx=8, ny=8, nz=4)
    c = W.centroids(m.verts, m.tets)
    m.tet_domain = np.digitize(c[:, 2], [15.0, 32.0]).astype(np.int32)
    m.ndom = 3
    return m


def singles(vie, s, tol, max_iter, restart):
    out = {}
    for p in (vie.VIE_TE, vie.VIE_TM):
        info = s.solve(p, tol=tol, max_iter=max_iter, restart=restart, allow_noconv=True)
        out[p] = (info, s.read_solution(), s.residual_history(), s.absorption())
    return out


def check_pair(vie, s, ref, tol, max_iter, restart):
    info = s.solve_pair(tol=tol, max_iter=max_iter, restart=restart, allow_noconv=True)
    for p in (vie.VIE_TE, vie.VIE_TM):
        i0, x0, h0, a0 = ref[p]
        ip = info[p]
        for k in ("iters", "restarts", "converged", "true_rel_residual"):
            assert ip[k] == i0[k], (p, k, ip[k], i0[k])
        assert np.array_equal(s.read_solution(p), x0), p
        A, R, T = s.absorption(pol=p)
        assert np.array_equal(A, a0[0]) and R == a0[1] and T == a0[2], p
    # after a pair the polarisation-free read-backs refer to TM
    assert np.array_equal(s.residual_history(), ref[vie.VIE_TM][2])
    assert np.array_equal(s.read_solution(), ref[vie.VIE_TM][1])
    return info


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", ["plain", "graph", "coop"])
def test_pair_matches_single_solves_bitwise(vie, precision, mode):
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    m = osc_small()
    lam = 520.0
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, 40)
    if mode == "graph":
        s.set_option(vie.VIE_OPT_GRAPH_STEPS, 4)
    if mode == "coop":
        s.set_option(vie.VIE_OPT_TRSV_COOP, 1)
    s.fill(lam, 0.6, 0.3, eps_for(m, lam))
    s.factor()
    # a short restart so that both processes run several cycles
    tol, restart = 1e-11, 12
    ref = singles(vie, s, tol, 400, restart)
    print("single iterations TE/TM:", ref[0][0]["iters"], ref[1][0]["iters"], flush=True)
    assert ref[0][0]["converged"] and ref[1][0]["converged"]
    assert ref[0][0]["restarts"] > 0 and ref[1][0]["restarts"] > 0
    for rep in range(2):
        check_pair(vie, s, ref, tol, 400, restart)
        s.bench_matvec(1)   # other work between the runs


def test_pair_on_three_domains_and_at_max_iter(vie):
    m = three_domain_slab()
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 30)
    s.fill(560.0, 0.4, 0.3, W.slab_eps(m, 3.0 + 0.2j))
    s.factor()
    ref = singles(vie, s, 1e-10, 400, 30)
    check_pair(vie, s, ref, 1e-10, 400, 30)
    # stopped by max_iter: VIE_ENOCONV, both solutions still written
    ref = singles(vie, s, 1e-14, 7, 5)
    assert not ref[0][0]["converged"] and not ref[1][0]["converged"]
    check_pair(vie, s, ref, 1e-14, 7, 5)
    with pytest.raises(vie.VieError) as e:
        s.solve_pair(tol=1e-14, max_iter=7, restart=5)
    assert e.value.code == vie.VIE_ENOCONV


def test_single_solve_leaves_other_polarisation_unavailable(vie):
    m = three_domain_slab()
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 20)
    s.fill(600.0, 0.0, 0.0, W.slab_eps(m))
    s.factor()
    s.solve_pair(tol=1e-10, max_iter=200, restart=20)
    A_te = s.absorption(pol=vie.VIE_TE)
    s.solve(vie.VIE_TM, tol=1e-10, max_iter=200, restart=20)
    with pytest.raises(vie.VieError) as e:
        s.absorption(pol=vie.VIE_TE)
    assert e.value.code == vie.VIE_ESTATE
    s.solve(vie.VIE_TE, tol=1e-10, max_iter=200, restart=20)
    assert np.array_equal(s.absorption(pol=vie.VIE_TE)[0], A_te[0])


def test_pair_matches_oracle(vie):
    from oracle import topology as OT
    from oracle import vie as OV
    m = osc_small()
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    lam = 480.0
    eps = eps_for(m, lam)
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 30)
    s.fill(lam, 0.2, 0.1, eps)
    s.factor()
    info = s.solve_pair(tol=1e-10, max_iter=500, restart=30)
    wave = OV.make_wave(lam, 0.2, 0.1)
    Zo = OV.assemble(t, wave, eps)
    for p in (vie.VIE_TE, vie.VIE_TM):
        xo, it, hist, ok = OV.gmres_right_block(Zo, OV.rhs(t, wave, p), t.domain_ranges, tol=1e-10, restart=30)
        assert ok and info[p]["converged"] and abs(info[p]["iters"] - it) <= 1
        assert np.linalg.norm(s.read_solution(p) - xo) < 1e-8 * np.linalg.norm(xo)


def test_pair_with_more_domains_than_one_launch_carries(vie):
    """Ten domains (8 x 8 x 4 slab split by x slice and z half): the paired
    triangular solves and block LU run in two launches per step."""
    m = W.slab_mesh(nx=8, ny=8, nz=4)
    c = W.centroids(m.verts, m.tets)
    xs = np.digitize(c[:, 0], [20.0, 40.0, 60.0, 80.0])
    m.tet_domain = (2 * xs + (c[:, 2] > 25.0)).astype(np.int32)
    m.ndom = 10
    for prec in (vie.VIE_FP64, vie.VIE_MIXED_FP32):
        s = vie.Solver()
        s.upload_mesh(m)
        s.bind(prec, 30)
        s.fill(600.0, 0.3, 0.2, W.slab_eps(m, 3.0 + 0.2j))
        s.factor()
        assert len(s.domain_ranges()) == 10
        ref = singles(vie, s, 1e-10, 300, 30)
        assert ref[0][0]["converged"] and ref[1][0]["converged"]
        check_pair(vie, s, ref, 1e-10, 300, 30)
