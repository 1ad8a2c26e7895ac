"""Pins for the oracle's transfer-matrix slab (the homogeneous-slab closed form
the whole method is checked against).

Independent of its Airy formula: the one-dimensional wave equation across the
slab integrated numerically (TE: E_y'' + k0^2 (eps - s^2) E_y = 0; TM:
(H_y' / eps)' + k0^2 (1 - s^2 / eps) H_y = 0, with H_y and H_y' / eps
continuous), shooting from the transmitted wave below the slab and matching
incident plus reflected waves above it.  The table of the 50 nm slab
(eps = 3.6 + 0.6i, 600 nm) is the set of transfer-matrix values the workload
specification quotes for it."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import fresnel as F

SLAB_EPS, SLAB_D, SLAB_LAM = 3.6 + 0.6j, 50.0, 600.0

# (theta deg, pol, R, T, A) as quoted for the 50 nm slab at 600 nm
TABLE = [
    (0, 0, 0.216452, 0.623277, 0.160271),
    (30, 0, 0.268098, 0.565016, 0.166886),
    (30, 1, 0.150882, 0.682603, 0.166515),
    (60, 0, 0.498160, 0.333389, 0.168451),
    (60, 1, 0.004179, 0.827916, 0.167905),
]


def shoot_rt(eps, d, lam, theta, pol):
    """R, T of a slab z in [0, d] in vacuum by integrating the field ODE."""
    k0 = 2 * np.pi / lam
    s2 = np.sin(theta) ** 2
    kz0 = k0 * np.cos(theta)
    eps = complex(eps)
    if pol == 0:
        def rhs(z, y):        # y = (E, E')
            return [y[1], -k0 * k0 * (eps - s2) * y[0]]
        y0 = [1.0 + 0j, -1j * kz0]              # transmitted wave exp(-i kz0 z) below
    else:
        def rhs(z, y):        # y = (H, U = H' / eps)
            return [eps * y[1], -k0 * k0 * (1 - s2 / eps) * y[0]]
        y0 = [1.0 + 0j, -1j * kz0]
    sol = solve_ivp(rhs, (0.0, d), np.array(y0, complex), rtol=1e-12, atol=1e-14, method="DOP853")
    F0, F1 = sol.y[0, -1], sol.y[1, -1]
    # above: a exp(-i kz0 (z - d)) + r_un exp(+i kz0 (z - d)); derivative -i kz0 a + i kz0 r_un
    a = 0.5 * (F0 - F1 / (1j * kz0))
    r_un = 0.5 * (F0 + F1 / (1j * kz0))
    return abs(r_un / a) ** 2, abs(1.0 / a) ** 2


@pytest.mark.parametrize("th,pol", [(0, 0), (30, 0), (30, 1), (60, 0), (60, 1), (75, 1)])
@pytest.mark.parametrize("eps", [SLAB_EPS, 3.6 + 0j, -4.7 + 0.05j])
def test_slab_rta_against_wave_equation(eps, th, pol):
    R, T, A = F.slab_rta(eps, SLAB_D, SLAB_LAM, np.deg2rad(th), pol)
    Rs, Ts = shoot_rt(eps, SLAB_D, SLAB_LAM, np.deg2rad(th), pol)
    assert abs(R - Rs) < 1e-9 and abs(T - Ts) < 1e-9, (R, Rs, T, Ts)
    assert A >= -1e-15


@pytest.mark.parametrize("th,pol,R0,T0,A0", TABLE)
def test_slab_table(th, pol, R0, T0, A0):
    R, T, A = F.slab_rta(SLAB_EPS, SLAB_D, SLAB_LAM, np.deg2rad(th), pol)
    assert abs(R - R0) < 1e-6 and abs(T - T0) < 1e-6 and abs(A - A0) < 1e-6, (R, T, A)


def test_lossless_slab_table():
    R, T, A = F.slab_rta(3.6, SLAB_D, SLAB_LAM, 0.0, 0)
    assert abs(R - 0.247894) < 1e-6 and abs(T - 0.752106) < 1e-6 and abs(A) < 1e-15


def shoot_stack(eps_layers, d_layers, lam, theta, pol):
    """R, T and the absorption of each layer of a planar stack (layers listed
    from the incidence side) by the same integration, layer by layer from the
    exit side.  The normal power flux is proportional to Im(conj(F) F'),
    F = E_y (TE) or (H_y, H_y'/eps) (TM), continuous across interfaces; a
    layer absorbs the drop of that flux across it."""
    k0 = 2 * np.pi / lam
    s2 = np.sin(theta) ** 2
    kz0 = k0 * np.cos(theta)
    y = np.array([1.0 + 0j, -1j * kz0])
    flux = [(np.conj(y[0]) * y[1]).imag]           # below the stack
    for eps, d in zip(reversed(eps_layers), reversed(d_layers)):
        eps = complex(eps)
        if pol == 0:
            f = lambda z, y, e=eps: [y[1], -k0 * k0 * (e - s2) * y[0]]
        else:
            f = lambda z, y, e=eps: [e * y[1], -k0 * k0 * (1 - s2 / e) * y[0]]
        y = solve_ivp(f, (0.0, d), y, rtol=1e-12, atol=1e-14, method="DOP853").y[:, -1]
        flux.append((np.conj(y[0]) * y[1]).imag)
    a = 0.5 * (y[0] - y[1] / (1j * kz0))
    r_un = 0.5 * (y[0] + y[1] / (1j * kz0))
    inc = abs(a) ** 2 * kz0                          # |Im(conj(F) F')| of the incident wave alone
    flux = flux[::-1]                                # above layer 0, ..., below the last
    absorbed = [(flux[j + 1] - flux[j]) / inc for j in range(len(eps_layers))]
    return abs(r_un / a) ** 2, abs(1.0 / a) ** 2, absorbed


@pytest.mark.parametrize("pol", [0, 1])
def test_multilayer_against_wave_equation(pol):
    layers = [2.3 + 0.05j, -4.7 + 0.05j, 3.6 + 0.6j]
    ds = [20.0, 15.0, 45.0]
    R, T, absorbed = F.multilayer_rta(layers, ds, 480.0, 0.6, pol)
    Rs, Ts, As = shoot_stack(layers, ds, 480.0, 0.6, pol)
    assert abs(R - Rs) < 1e-9 and abs(T - Ts) < 1e-9, (R, Rs, T, Ts)
    assert np.max(np.abs(np.array(absorbed) - np.array(As))) < 1e-9, (absorbed, As)
    assert abs(sum(As) - (1 - Rs - Ts)) < 1e-9 and all(x > 0 for x in As)
