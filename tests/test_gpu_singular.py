"""A zero pivot in the block factorisation (Sec. 2.3, Eq. 6) and what the
library does after it.

No physical input makes a diagonal block exactly singular (the permittivity
term is a Gram matrix over 1/eps, and zero or non-finite permittivities are
rejected by vie_fill), so the condition is forced from the host: the test owns
the workspace and clears it between a fill and the factorisation, which leaves
Z all zeros.  The kernels take a zero pivot in bounds by design (no division,
ties to the smaller row), so the run ends normally and the error is reported
through the return code:
  * vie_precond_factor returns VIE_ESINGULAR and names domain 0, column 0;
  * the factors of the earlier, successful factorisation are void: vie_solve,
    vie_solve_pair and vie_precond_apply return VIE_ESTATE;
  * a new bind (which uploads the mesh tables again), fill and factorisation
    give the same solution as before the failure.
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


def slab():
    """8 x 8 x 3 slab, one domain per z layer (every domain spans two 512-row
    diagonal blocks)."""
    m = W.slab_mesh(nx=8, ny=8, nz=3)
    c = W.centroids(m.verts, m.tets)
    m.tet_domain = np.digitize(c[:, 2], [50.0 / 3, 100.0 / 3]).astype(np.int32)
    m.ndom = 3
    return m


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_pivot_is_reported_and_voids_the_factors(vie, precision):
    torch = vie.Solver().torch
    prec = vie.VIE_FP64 if precision == "fp64" else vie.VIE_MIXED_FP32
    m = slab()
    eps = np.full(m.nt, 2.25 + 0.1j)
    s = vie.Solver()
    N = s.upload_mesh(m)
    print(f"singular {precision}: N = {N}, domains {s.domain_ranges().tolist()}", flush=True)
    tol = 1e-10 if precision == "fp64" else 1e-8
    s.bind(prec, 40)
    s.fill(600.0, 0.0, 0.0, eps)
    s.factor()
    s.solve(vie.VIE_TE, tol=tol)
    x0 = s.read_solution()

    with torch.cuda.stream(s.stream):
        s.ws.zero_()
    torch.cuda.synchronize()
    with pytest.raises(vie.VieError) as e:
        s.factor()
    assert e.value.code == vie.VIE_ESINGULAR
    assert "zero pivot in block 0 at column 0" in str(e.value)
    print(f"  factor: {e.value}", flush=True)
    for call in (lambda: s.solve(vie.VIE_TE, tol=tol), lambda: s.solve_pair(tol=tol),
                 lambda: s.precond_apply(np.ones(N, np.complex128))):
        with pytest.raises(vie.VieError) as e:
            call()
        assert e.value.code == vie.VIE_ESTATE

    s.bind(prec, 40, workspace=s.ws)
    s.fill(600.0, 0.0, 0.0, eps)
    s.factor()
    s.solve(vie.VIE_TE, tol=tol)
    x1 = s.read_solution()
    assert np.linalg.norm(x1 - x0) <= (1e-11 if precision == "fp64" else 1e-8) * np.linalg.norm(x0)
    s.close()
