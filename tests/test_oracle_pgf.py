"""Pins for the oracle's Ewald periodic Green's function (Sec. 2.2, Eqs. 3-4).

Independent facts: the direct lattice sum (Eq. 3 as written, convergent for a
lossy background), the pure spectral (Floquet) series for |z| > 0, the
independence of the Ewald result from the split parameter E, the Bloch
quasi-periodicity and reciprocity of Eq. 3, the Helmholtz equation away from
the lattice points, and the small-R behaviour 1/(4 pi R) + finite limit."""
import numpy as np
import pytest

from oracle import pgf

A, B = 100.0, 130.0
LAM = 600.0
K0 = 2 * np.pi / LAM


def kt(theta, phi, k=K0):
    return k * np.sin(theta) * np.cos(phi), k * np.sin(theta) * np.sin(phi)


def pts(n, seed=0, zmax=60.0):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-A, A, n), rng.uniform(-B, B, n), rng.uniform(-zmax, zmax, n)], 1)


@pytest.mark.parametrize("theta,phi", [(0.0, 0.0), (0.5, 0.3), (1.2, 1.0)])
def test_split_independence(theta, phi):
    kx, ky = kt(theta, phi)
    d = pts(30, 1)
    E = pgf.ewald_split(A, B)
    g0 = pgf.pgf_ewald(d, K0, kx, ky, A, B)
    for f, M in ((0.8, 4), (1.25, 4), (2.0, 7), (0.5, 7)):
        g = pgf.pgf_ewald(d, K0, kx, ky, A, B, E=f * E, M=M)
        assert np.max(np.abs(g - g0) / np.abs(g0)) < 1e-12, f


def test_direct_sum_lossy():
    k = K0 * (1 - 0.3j)
    kx, ky = kt(0.4, 0.7)
    d = pts(4, 2)
    ge = pgf.pgf_ewald(d, k, kx, ky, A, B)
    gd = pgf.pgf_direct(d, k, kx, ky, A, B, L=300)
    assert np.max(np.abs(ge - gd) / np.abs(gd)) < 1e-13


@pytest.mark.parametrize("theta", [0.0, 0.7, 1.3])
def test_spectral_series(theta):
    kx, ky = kt(theta, 0.4)
    d = pts(6, 3)
    d[:, 2] = np.where(d[:, 2] >= 0, 1, -1) * np.maximum(np.abs(d[:, 2]), 0.2 * A)
    gs = pgf.pgf_spectral(d, K0, kx, ky, A, B, P=60)
    ge = pgf.pgf_ewald(d, K0, kx, ky, A, B)
    assert np.max(np.abs(ge - gs) / np.abs(gs)) < 1e-13


def test_quasi_periodicity_and_reciprocity():
    kx, ky = kt(0.9, 0.5)
    d = pts(10, 4)
    g = pgf.pgf_ewald(d, K0, kx, ky, A, B)
    for m, n in ((1, 0), (0, -1), (2, 1)):
        rho = np.array([m * A, n * B, 0.0])
        gs = pgf.pgf_ewald(d + rho, K0, kx, ky, A, B)
        assert np.max(np.abs(gs - np.exp(-1j * (kx * rho[0] + ky * rho[1])) * g)) < 1e-13 * np.abs(g).max()
    gr = pgf.pgf_ewald(-d, K0, -kx, -ky, A, B)
    assert np.max(np.abs(gr - g) / np.abs(g)) < 1e-12


def test_helmholtz_residual():
    kx, ky = kt(0.6, 0.2)
    d0 = np.array([[23.0, -31.0, 17.0], [-40.0, 12.0, -25.0]])
    h = 0.5
    lap = 0
    c = np.array([-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12])
    for ax in range(3):
        for i, s in enumerate((-2, -1, 0, 1, 2)):
            dd = d0.copy(); dd[:, ax] += s * h
            lap = lap + c[i] * pgf.pgf_ewald(dd, K0, kx, ky, A, B) / h ** 2
    g = pgf.pgf_ewald(d0, K0, kx, ky, A, B)
    res = np.abs(lap + K0 ** 2 * g)
    assert np.all(res < 1e-4 * np.abs(K0 ** 2 * g)), res / np.abs(K0 ** 2 * g)


def test_small_R_limit():
    kx, ky = kt(0.3, 0.9)
    E = pgf.ewald_split(A, B)
    g0 = pgf.pgf_ewald(np.zeros((1, 3)), K0, kx, ky, A, B, self_limit=True)[0]
    diffs = []
    for r in (1e-2, 1e-3):
        dd = np.array([[r * 0.6, r * 0.8, 0.0]])
        g = pgf.pgf_ewald(dd, K0, kx, ky, A, B)[0] - 1 / (4 * np.pi * r)
        diffs.append(abs(g - g0))
    # g_p - 1/(4 pi R) is continuous with an O(R) deviation from its limit
    assert diffs[1] < 0.2 * diffs[0] and diffs[1] < 1e-5 * abs(g0)
    # the closed form of the self-image limit against a difference quotient
    r = 1e-5
    y = K0 / (2 * E)
    from scipy.special import erfc
    t = (np.exp(-1j * K0 * r) * erfc(r * E - 1j * y) + np.exp(1j * K0 * r) * erfc(r * E + 1j * y)) / (8 * np.pi * r)
    assert abs((t - 1 / (4 * np.pi * r)) - pgf.self_limit_value(K0, E)) < 1e-8


def test_branch_and_truncation_error():
    # truncation at M = 4: the omitted terms are below 1e-15 relative
    kx, ky = kt(1.0, 0.2)
    d = pts(10, 5, zmax=160)
    g4 = pgf.pgf_ewald(d, K0, kx, ky, A, B, M=4)
    g8 = pgf.pgf_ewald(d, K0, kx, ky, A, B, M=8)
    assert np.max(np.abs(g4 - g8) / np.abs(g8)) < 1e-14
    g = pgf.propagation_constant(np.array([0.5 * K0 ** 2, 2 * K0 ** 2]), K0)
    assert g[0].real == 0 and g[0].imag > 0 and g[1].real > 0
