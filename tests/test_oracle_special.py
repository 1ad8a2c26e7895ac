"""Pins for the library special functions the oracle relies on: scipy's complex
erfc / erfi against mpmath at 50 digits over the argument ranges the Ewald
series use (R E in [0, 12], k/2E up to ~1.5, gamma/2E and z E up to ~12)."""
import mpmath as mp
import numpy as np
from scipy.special import erfc, erfi

mp.mp.dps = 50


def test_erfc_complex_vs_mpmath():
    rng = np.random.default_rng(3)
    zs = list(rng.uniform(0, 12, 40) - 1j * rng.uniform(0, 1.5, 40))
    zs += list(rng.uniform(-3, 12, 40) + 1j * rng.uniform(-1.5, 1.5, 40))
    zs += list(1j * rng.uniform(0, 1.5, 10) + rng.uniform(-3, 3, 10))
    for z in zs:
        ref = complex(mp.erfc(mp.mpc(z.real, z.imag)))
        got = erfc(z)
        assert abs(got - ref) <= 2e-14 * abs(ref) + 1e-300, (z, got, ref)


def test_erfi_real_vs_mpmath():
    for y in np.linspace(0, 2, 21):
        assert abs(erfi(y) - float(mp.erfi(y))) <= 1e-15 * max(1, abs(float(mp.erfi(y))))
