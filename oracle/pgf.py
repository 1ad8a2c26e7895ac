"""Two-dimensional periodic Green's function (Sec. 2.2, Eqs. 3-4).

Definition (paper's convention, time dependence exp(j w t)):
    g_p(r, r') = sum_{m,n} exp(-j k R_mn) / (4 pi R_mn) * exp(+j (kx m a + ky n b)),
    R_mn = | r - r' + (m a, n b, 0) |,
with the Bloch wavenumbers kx = k0 sin(theta) cos(phi), ky = k0 sin(theta) sin(phi).

Ewald evaluation (Sec. 2.2: spatial series by the Ewald identity, spectral
series by Poisson summation).  Split parameter E; both series truncated at
|m|,|n| <= M and |p|,|q| <= M:
  spatial  : sum_mn e^{j kt.rho_mn} [e^{-jkR} erfc(R E - j k/2E) + e^{jkR} erfc(R E + j k/2E)] / (8 pi R)
  spectral : 1/(4ab) sum_pq e^{-j k_t,pq . Delta_t} / gamma_pq
                 [e^{gamma z} erfc(gamma/2E + z E) + e^{-gamma z} erfc(gamma/2E - z E)]
with k_t,pq = kt + (2 pi p / a, 2 pi q / b), gamma_pq = sqrt(|k_t,pq|^2 - k^2),
Re gamma >= 0 and +j sqrt(k^2 - |k_t,pq|^2) for propagating orders.
The transverse separation is first wrapped to the nearest image; the
quasi-periodicity g_p(Delta + rho) = e^{-j kt.rho} g_p(Delta) restores it.

Also here, for the pins only: the direct lattice sum (lossy k) and the pure
spectral sum (|z| > 0).  Special functions: scipy.special.erfc / erfi (complex),
themselves pinned against mpmath in the tests.
"""
import numpy as np
from scipy.special import erfc, erfi

FOUR_PI = 4.0 * np.pi


def ewald_split(a, b):
    """Default split parameter E = sqrt(pi / (a b))."""
    return np.sqrt(np.pi / (a * b))


def propagation_constant(kt2, k):
    """gamma = sqrt(kt^2 - k^2) on the branch Re >= 0, and +j sqrt(k^2 - kt^2)
    when the order propagates (real k, kt^2 < k^2)."""
    g = np.sqrt(np.asarray(kt2, dtype=complex) - complex(k) ** 2)
    g = np.where(g.real < 0, -g, g)
    g = np.where((g.real == 0) & (g.imag < 0), -g, g)
    return g


def wrap(delta, a, b):
    """Nearest-image wrap of the transverse separation; returns wrapped delta
    and the integer shifts (m0, n0) with delta = wrapped + (m0 a, n0 b, 0)."""
    delta = np.asarray(delta, float)
    m0 = np.rint(delta[..., 0] / a)
    n0 = np.rint(delta[..., 1] / b)
    w = delta.copy()
    w[..., 0] -= m0 * a
    w[..., 1] -= n0 * b
    return w, m0, n0


def pgf_ewald(delta, k, kx, ky, a, b, E=None, M=4, self_limit=False):
    """Ewald evaluation of g_p at separations delta [..., 3] = r - r'.

    k may be complex (lossy background, used by the pins).  If self_limit is
    True, a zero-length image term is replaced by the finite limit of
    (spatial image term - 1/(4 pi R)) as R -> 0, i.e. the value of
    g_p - 1/(4 pi |delta|) at delta = 0."""
    E = ewald_split(a, b) if E is None else E
    delta = np.atleast_2d(np.asarray(delta, float))
    dw, m0, n0 = wrap(delta, a, b)
    phase0 = np.exp(-1j * (kx * m0 * a + ky * n0 * b))
    z = dw[:, 2]
    y = k / (2.0 * E)
    S = np.zeros(len(dw), complex)
    for m in range(-M, M + 1):
        for n in range(-M, M + 1):
            X = dw[:, 0] + m * a
            Y = dw[:, 1] + n * b
            R = np.sqrt(X * X + Y * Y + z * z)
            ph = np.exp(1j * (kx * m * a + ky * n * b))
            zero = R == 0.0
            Rs = np.where(zero, 1.0, R)
            t = (np.exp(-1j * k * Rs) * erfc(Rs * E - 1j * y)
                 + np.exp(1j * k * Rs) * erfc(Rs * E + 1j * y)) / (2.0 * FOUR_PI * Rs)
            if np.any(zero):
                if not self_limit:
                    t = np.where(zero, np.inf, t)
                else:
                    t = np.where(zero, self_limit_value(k, E), t)
            S += ph * t
    K = np.zeros(len(dw), complex)
    for p in range(-M, M + 1):
        for q in range(-M, M + 1):
            ktx = kx + 2.0 * np.pi * p / a
            kty = ky + 2.0 * np.pi * q / b
            g = propagation_constant(ktx * ktx + kty * kty, k)
            u = g / (2.0 * E)
            term = (np.exp(g * z) * erfc(u + z * E) + np.exp(-g * z) * erfc(u - z * E)) / g
            K += np.exp(-1j * (ktx * dw[:, 0] + kty * dw[:, 1])) * term
    K /= 4.0 * a * b
    return phase0 * (S + K)


def self_limit_value(k, E):
    """lim_{R->0} [spatial image term - 1/(4 pi R)] for the Ewald split E:
    k erfi(k/2E) / (4 pi) - E exp((k/2E)^2) / (2 pi^(3/2))."""
    y = k / (2.0 * E)
    return k * erfi(y) / FOUR_PI - E * np.exp(y * y) / (2.0 * np.pi ** 1.5)


def pgf_direct(delta, k, kx, ky, a, b, L=300):
    """Direct lattice sum of Eq. 3 truncated at |m|,|n| <= L (only meaningful
    for a lossy k, where the terms decay exponentially)."""
    delta = np.atleast_2d(np.asarray(delta, float))
    m = np.arange(-L, L + 1)
    out = np.zeros(len(delta), complex)
    for i, d in enumerate(delta):
        X = d[0] + m[:, None] * a
        Y = d[1] + m[None, :] * b
        R = np.sqrt(X * X + Y * Y + d[2] ** 2)
        ph = np.exp(1j * (kx * m[:, None] * a + ky * m[None, :] * b))
        out[i] = np.sum(np.exp(-1j * k * R) / (FOUR_PI * R) * ph)
    return out


def pgf_spectral(delta, k, kx, ky, a, b, P=60):
    """Pure spectral (Floquet) series, valid for z != 0:
    (1/ab) sum_pq exp(-j k_t,pq . Delta_t) exp(-gamma |z|) / (2 gamma)."""
    delta = np.atleast_2d(np.asarray(delta, float))
    p = np.arange(-P, P + 1)
    out = np.zeros(len(delta), complex)
    for i, d in enumerate(delta):
        ktx = kx + 2 * np.pi * p[:, None] / a + 0 * p[None, :]
        kty = ky + 2 * np.pi * p[None, :] / b + 0 * p[:, None]
        g = propagation_constant(ktx ** 2 + kty ** 2, k)
        out[i] = np.sum(np.exp(-1j * (ktx * d[0] + kty * d[1])) * np.exp(-g * abs(d[2])) / (2 * g)) / (a * b)
    return out
