"""The block-diagonal preconditioner and the solve on cells whose domains span
several 256-row diagonal blocks with ragged tails (Sec. 2.3, Eqs. 5-6).

At these sizes the oracle is too slow to assemble Z, so the checks are
properties that hold at any size, taken on the library's own Z read back
through the C-ABI:
  * M^{-1} v solves every diagonal block: Z_dd z_d = v_d (and equals a dense
    LAPACK solve of Z_dd), including more domains than one launch carries;
  * with one domain M = Z, so right-preconditioned GMRES stops after one
    iteration;
  * tournament pivoting (the default) and partial pivoting column by column
    both factor every block: their M^{-1} v agree, on both precision paths;
  * the GMRES solution satisfies Z x = b.
"""
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


def slab_3200(split):
    """8 x 8 x 4 slab (N = 3,200) with domains by z layer (3) or by x slice
    and z half (10, more than one triangular-solve launch carries)."""
    m = W.slab_mesh(nx=8, ny=8, nz=4)
    c = W.centroids(m.verts, m.tets)
    if split == 1:
        m.tet_domain = np.zeros(m.nt, np.int32); m.ndom = 1
    elif split == 3:
        m.tet_domain = np.digitize(c[:, 2], [15.0, 32.0]).astype(np.int32); m.ndom = 3
    else:
        xs = np.digitize(c[:, 0], [20.0, 40.0, 60.0, 80.0])
        m.tet_domain = (2 * xs + (c[:, 2] > 25.0)).astype(np.int32); m.ndom = 10
    return m


def solver(vie, m, restart=60):
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(vie.VIE_FP64, restart)
    return s


def read_block(s, lo, hi):
    r, c = np.meshgrid(np.arange(lo, hi), np.arange(lo, hi), indexing="ij")
    return s.read_Z(r.ravel(), c.ravel()).reshape(hi - lo, hi - lo)


@pytest.mark.parametrize("split", [3, 10])
def test_precond_apply_solves_each_diagonal_block(vie, split):
    m = slab_3200(split)
    s = solver(vie, m)
    eps = W.slab_eps(m)
    s.fill(600.0, 0.3, 0.2, eps)
    s.factor()
    ranges = s.domain_ranges()
    sizes = [int(e - b) for b, e in ranges]
    assert sum(sizes) == 3200 and len(sizes) == split
    assert max(sizes) > 256
    rng = np.random.default_rng(11)
    N = s.num_unknowns()
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    z = s.precond_apply(v)
    for (lo, hi) in ranges:
        A = read_block(s, int(lo), int(hi))
        zd, vd = z[lo:hi], v[lo:hi]
        res = np.linalg.norm(A @ zd - vd) / np.linalg.norm(vd)
        assert res < 1e-12, (lo, hi, res)
        ref = np.linalg.solve(A, vd)
        assert np.linalg.norm(zd - ref) < 1e-10 * np.linalg.norm(ref)


def test_single_domain_multiblock_converges_in_one_iteration(vie):
    m = slab_3200(1)
    s = solver(vie, m)
    s.fill(600.0, 0.3, 0.2, W.slab_eps(m))
    s.factor()
    for pol in (0, 1):
        info = s.solve(pol, tol=1e-12, max_iter=20)
        assert info["iters"] == 1 and info["converged"], info


def test_multidomain_solution_satisfies_Zx_eq_b(vie):
    m = slab_3200(3)
    s = solver(vie, m)
    s.fill(600.0, 0.3, 0.2, W.slab_eps(m))
    s.factor()
    info = s.solve(0, tol=1e-10, max_iter=200, restart=30)
    assert info["converged"] and info["iters"] < 40, info
    N = s.num_unknowns()
    x, b = s.read_solution(), s.read_rhs()
    r = b.copy()
    for lo in range(0, N, 800):
        rows = np.arange(lo, min(N, lo + 800))
        rr, cc = np.meshgrid(rows, np.arange(N), indexing="ij")
        Zr = s.read_Z(rr.ravel(), cc.ravel()).reshape(len(rows), N)
        r[rows] -= Zr @ x
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tournament_and_partial_pivoting_agree(vie, prec):
    """One domain of 3,200 unknowns: 50 panels, a tournament tree of up to 25
    leaves with odd node counts on several levels."""
    m = slab_3200(1)
    p = vie.VIE_FP64 if prec == "fp64" else vie.VIE_MIXED_FP32
    s = vie.Solver()
    s.upload_mesh(m)
    s.bind(p, 30)
    s.fill(600.0, 0.3, 0.2, W.slab_eps(m))
    N = s.num_unknowns()
    rng = np.random.default_rng(5)
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert s.get_option(vie.VIE_OPT_LU_PIVOT) == 0
    s.factor()
    z_t = s.precond_apply(v)
    # the timed K = 128 updates: their algorithmic work is 8 rows cols 128 per panel pair
    st = s.factor_stats()
    exp = sum(8.0 * (N - k0 - 128) ** 2 * 128 for k0 in range(0, N, 128) if N - k0 - 128 > 0)
    assert st["update_flops"] == exp and abs(st["factor_flops"] - 8.0 / 3.0 * N ** 3) < 1e-6 * N ** 3
    assert 0 < st["t_update_ms"] < st["t_factor_ms"] and st["update_launches"] == 2 * (len(range(0, N, 128)) - 1)
    s.set_option(vie.VIE_OPT_LU_PIVOT, 1)
    assert s.get_option(vie.VIE_OPT_LU_PIVOT) == 1
    s.factor()
    z_p = s.precond_apply(v)
    assert s.factor_stats()["update_flops"] == 0 and s.factor_stats()["update_launches"] == 0
    with pytest.raises(vie.VieError):
        s.set_option(vie.VIE_OPT_LU_PIVOT, 2)
    A = read_block(s, 0, N)
    if prec == "fp64":
        assert np.linalg.norm(z_t - z_p) < 1e-10 * np.linalg.norm(z_p)
        for z in (z_t, z_p):
            assert np.linalg.norm(A @ z - v) < 1e-12 * np.linalg.norm(v)
    else:
        # FP32 factors: the tournament's error is that of partial pivoting's
        # up to a small factor (both are backward-stable FP32 eliminations)
        zs = np.linalg.solve(A, v)
        e_t = np.linalg.norm(z_t - zs) / np.linalg.norm(zs)
        e_p = np.linalg.norm(z_p - zs) / np.linalg.norm(zs)
        assert e_p < 1e-3 and e_t < 3 * e_p + 1e-6, (e_t, e_p)
