"""Transfer-matrix reflectance/transmittance of a homogeneous slab.

Closed-form reference for the homogeneous periodic slab (a periodic structure
whose unit cell is uniform): with vacuum on both sides, a plane wave of angle
theta sees the classical thin-film (Airy) result.  Optics convention
exp(-i w t) with eps Im >= 0 lossy; R, T and A are convention-independent.

  kz_j = k0 sqrt(eps_j - sin^2 theta)  (Im kz >= 0)
  TE: r_ij = (kz_i - kz_j) / (kz_i + kz_j),         t_ij = 2 kz_i / (kz_i + kz_j)
  TM: r_ij = (eps_j kz_i - eps_i kz_j) / (eps_j kz_i + eps_i kz_j),
      t_ij = 2 sqrt(eps_i eps_j) kz_i / (eps_j kz_i + eps_i kz_j)   (field ratio H-based)
  r = (r01 + r12 e^{2 i d kz1}) / (1 + r01 r12 e^{2 i d kz1})
  t = t01 t12 e^{i d kz1} / (1 + r01 r12 e^{2 i d kz1})
  R = |r|^2, T = |t|^2 (same medium on both sides), A = 1 - R - T.

The multilayer form below (characteristic 2x2 matrix per layer) reduces to
the same slab for one layer; the slab itself is pinned against a numerical
integration of the one-dimensional wave equation in the tests.
"""
import numpy as np


def slab_rta(eps, d, lam, theta, pol):
    """pol: 0 = TE (s), 1 = TM (p)."""
    k0 = 2 * np.pi / lam
    s2 = np.sin(theta) ** 2
    e0, e1 = 1.0 + 0j, complex(eps)
    kz0 = k0 * np.sqrt(e0 - s2 + 0j)
    kz1 = k0 * np.sqrt(e1 - s2 + 0j)
    if kz1.imag < 0:
        kz1 = -kz1
    if pol == 0:
        r01 = (kz0 - kz1) / (kz0 + kz1); r12 = (kz1 - kz0) / (kz1 + kz0)
        t01 = 2 * kz0 / (kz0 + kz1); t12 = 2 * kz1 / (kz1 + kz0)
    else:
        r01 = (e1 * kz0 - e0 * kz1) / (e1 * kz0 + e0 * kz1)
        r12 = (e0 * kz1 - e1 * kz0) / (e0 * kz1 + e1 * kz0)
        t01 = 2 * np.sqrt(e0 * e1) * kz0 / (e1 * kz0 + e0 * kz1)
        t12 = 2 * np.sqrt(e1 * e0) * kz1 / (e0 * kz1 + e1 * kz0)
    ph = np.exp(1j * kz1 * d)
    den = 1 + r01 * r12 * ph * ph
    r = (r01 + r12 * ph * ph) / den
    t = t01 * t12 * ph / den
    R = abs(r) ** 2
    T = abs(t) ** 2
    return R, T, 1.0 - R - T


def multilayer_rta(eps_layers, d_layers, lam, theta, pol):
    """Planar stack in vacuum, layers listed in the order the incident wave
    meets them.  Characteristic matrix of each layer (Born & Wolf:
    [[cos b, -i sin b / Y], [-i Y sin b, cos b]], b = kz d, Y the admittance:
    TE kz/k0, TM eps k0/kz),
    r and t from their product; the absorbed fraction of each layer is the
    drop of the normal Poynting flux Re(U V*) across it, with the tangential
    fields (U, V) carried up from the exit side, (U, V) = (t, Y0 t).
    Returns R, T and the list of per-layer absorptions (they add up to
    1 - R - T)."""
    k0 = 2 * np.pi / lam
    s2 = np.sin(theta) ** 2
    kz0 = k0 * np.sqrt(1 - s2 + 0j)
    Y0 = kz0 / k0 if pol == 0 else k0 / kz0
    mats = []
    for eps, d in zip(eps_layers, d_layers):
        kz = k0 * np.sqrt(complex(eps) - s2)
        if kz.imag < 0:
            kz = -kz
        Y = kz / k0 if pol == 0 else complex(eps) * k0 / kz
        bb = kz * d
        mats.append(np.array([[np.cos(bb), -1j * np.sin(bb) / Y], [-1j * Y * np.sin(bb), np.cos(bb)]]))
    M = np.eye(2, dtype=complex)
    for Mj in mats:
        M = M @ Mj
    den = (M[0, 0] + M[0, 1] * Y0) * Y0 + (M[1, 0] + M[1, 1] * Y0)
    r = ((M[0, 0] + M[0, 1] * Y0) * Y0 - (M[1, 0] + M[1, 1] * Y0)) / den
    t = 2 * Y0 / den
    uv = np.array([t, Y0 * t])
    flux = [(uv[0] * np.conj(uv[1])).real]          # below the last layer
    for Mj in reversed(mats):
        uv = Mj @ uv
        flux.append((uv[0] * np.conj(uv[1])).real)  # above layer j
    flux = flux[::-1]                                # above layer 0, ..., below the last
    s_inc = Y0.real
    absorbed = [(flux[j] - flux[j + 1]) / s_inc for j in range(len(mats))]
    return abs(r) ** 2, abs(t) ** 2, absorbed
