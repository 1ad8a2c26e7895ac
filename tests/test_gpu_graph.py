"""Graph-captured Arnoldi steps and the autotuner.

The captured graph issues exactly the launches of the plain path, so every
replay must reproduce the plain solve bit for bit: the same iteration count,
residual history and solution.  The graph is replayed in several solves with
plain-launch work and synchronisations between them, and each replay is
checked.  The autotuner's variants change launch shapes only (the per-row
sums keep their order), so its pick must not change any result either."""
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


def solved(vie, s, pol, restart):
    info = s.solve(pol, tol=1e-10, max_iter=400, restart=restart)
    return info, s.read_solution(), s.residual_history()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("steps,restart", [(4, 40), (8, 30)])
def test_graph_replays_match_plain_launches(vie, precision, steps, restart):
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    m = three_domain_slab()
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, 60)
    s.fill(560.0, 0.4, 0.3, W.slab_eps(m, 3.0 + 0.2j))
    s.factor()
    ref = {p: solved(vie, s, p, restart) for p in (0, 1)}
    assert ref[0][0]["converged"] and ref[0][0]["iters"] > steps
    s.set_option(vie.VIE_OPT_GRAPH_STEPS, steps)
    assert s.get_option(vie.VIE_OPT_GRAPH_STEPS) == steps
    for rep in range(3):
        for p in (0, 1):
            info, x, h = solved(vie, s, p, restart)
            i0, x0, h0 = ref[p]
            assert info["iters"] == i0["iters"] and info["restarts"] == i0["restarts"], (rep, p)
            assert np.array_equal(x, x0), (rep, p)
            assert np.array_equal(h, h0), (rep, p)
        # plain-launch work and synchronisations between the replays (the
        # captured graphs stay alive)
        v = np.random.default_rng(rep).standard_normal(s.num_unknowns()) + 0j
        s.precond_apply(v)
        s.bench_matvec(2)


def test_graph_mode_needs_a_stream_of_its_own(vie):
    import torch
    m = three_domain_slab()
    s = vie.Solver(stream=torch.cuda.default_stream())
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 20)
    s.fill(560.0, 0.0, 0.0, W.slab_eps(m))
    s.factor()
    s.set_option(vie.VIE_OPT_GRAPH_STEPS, 4)
    with pytest.raises(vie.VieError) as e:
        s.solve(0, tol=1e-8, max_iter=50, restart=20)
    assert e.value.code == vie.VIE_EINVAL


def test_graph_mode_iterations_match_oracle(vie):
    from oracle import topology as OT
    from oracle import vie as OV
    m = osc_small()
    t = OT.build(m.verts, m.tets, m.tet_domain, m.ndom, m.a, m.b)
    lam = 480.0
    eps = eps_for(m, lam)
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, 30)
    s.set_option(vie.VIE_OPT_GRAPH_STEPS, 4)
    s.fill(lam, 0.2, 0.1, eps)
    s.factor()
    info = s.solve(1, tol=1e-10, max_iter=500, restart=30)
    wave = OV.make_wave(lam, 0.2, 0.1)
    Zo = OV.assemble(t, wave, eps)
    xo, it, hist, ok = OV.gmres_right_block(Zo, OV.rhs(t, wave, 1), t.domain_ranges, tol=1e-10, restart=30)
    assert ok and info["converged"] and abs(info["iters"] - it) <= 1
    assert np.linalg.norm(s.read_solution() - xo) < 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_picks_a_variant_without_changing_results(vie, precision):
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    m = three_domain_slab()
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(prec, 40)
    s.fill(610.0, 0.2, 0.7, W.slab_eps(m))
    s.factor()
    base = solved(vie, s, 0, 40)
    tun = s.autotune(reps=3)
    assert tun["matvec_rows"] in (2, 4, 8) and tun["trsv_chunk"] in (1024, 2048)
    assert all(t > 0 for t in tun["matvec_ms"] + tun["apply_ms"])
    assert s.get_option(vie.VIE_OPT_MATVEC_ROWS) == tun["matvec_rows"]
    for mv in (2, 4, 8):
        for tr in (1024, 2048):
            s.set_option(vie.VIE_OPT_MATVEC_ROWS, mv)
            s.set_option(vie.VIE_OPT_TRSV_CHUNK, tr)
            info, x, h = solved(vie, s, 0, 40)
            assert info["iters"] == base[0]["iters"] and np.array_equal(x, base[1]), (mv, tr)
