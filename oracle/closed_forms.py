"""Analytic results that pin the operators (float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  Uniformly magnetised sphere (Sec. IV.A): with phi_1 = 4 pi M.r (which
  solves Eqs. poisson and bc_poisson exactly for uniform M), the FK
  integral gives phi_2 = -(8 pi/3) M.r on and inside the unit sphere, so
  the stray field is -(4 pi/3) M: demagnetising factor 1/3, the paper's
  analytic value 4 pi/3 along M.
  Demagnetising tensor of any body from surface data:
    N_ba = (1/(4 pi V)) surface-integral of phi^(a) n_b, phi = phi_1 + phi_2,
  for M = e_a. Trace N = 1; a cube gives I/3 (Sec. IV.A, energy 2 pi/3).
  Stray-field energy (Sec. IV.A): E_s = -1/2 vol-integral M.H
    = 1/2 surface-integral phi (M.n) for uniform M: 2 pi/3 for the unit cube,
    8 pi^2/9 for the unit sphere.
  Ellipsoid demagnetising factors (Osborn 1945), by 1-D quadrature:
    N_a = (abc/2) int_0^inf ds / ((a^2+s) sqrt((a^2+s)(b^2+s)(c^2+s))).
  Dielectric sphere in a uniform field E0 (from the operator of Eq. Ax with
  the principal-value field of s cos(theta), which is s cos(theta)/6):
    sigma_b = 3 (eps_i - eps_m)/(eps_i + 2 eps_m) E0 . n.
  Unit-sphere spectra of the single and double layer (1/(4 pi) normalised):
    S[Y_l] = Y_l/(2l+1),  D_pv[Y_l] = -Y_l/(2(2l+1)).
"""

from __future__ import annotations

import numpy as np

SPHERE_DEMAG = 1.0 / 3.0
CUBE_ENERGY = 2.0 * np.pi / 3.0
SPHERE_ENERGY = 8.0 * np.pi ** 2 / 9.0


def sphere_phi2(xyz, m, centre=(0.0, 0.0, 0.0)):
    """phi_2 on/in a uniformly magnetised sphere: -(8 pi/3) M.(r - c)."""
    return -(8.0 * np.pi / 3.0) * ((np.asarray(xyz, dtype=np.float64) - centre) @ np.asarray(m))


def single_layer_eigenvalue(l):
    return 1.0 / (2 * l + 1)


def double_layer_eigenvalue(l):
    return -1.0 / (2 * (2 * l + 1))


def dielectric_sphere_sigma(normals, eps_i, eps_m, e0):
    k = 3.0 * (eps_i - eps_m) / (eps_i + 2.0 * eps_m)
    return k * (np.asarray(normals, dtype=np.float64) @ np.asarray(e0, dtype=np.float64))


def ellipsoid_demag(axes):
    """Osborn's demagnetising factors (N_a, N_b, N_c) of an ellipsoid."""
    from scipy.integrate import quad

    a, b, c = (float(v) for v in axes)
    out = []
    for s0 in (a, b, c):
        f = lambda s, s0=s0: 1.0 / ((s0 * s0 + s) * np.sqrt((a * a + s) * (b * b + s) * (c * c + s)))
        val, _ = quad(f, 0.0, np.inf, limit=200, epsabs=0.0, epsrel=1e-12)
        out.append(0.5 * a * b * c * val)
    return np.array(out)


def demag_tensor_from_surface(phi_total, normals, weights, volume):
    """N[b, a] = (1/(4 pi V)) sum_j phi^(a)_j n_{j,b} w_j; phi_total is [3, n]."""
    phi = np.asarray(phi_total, dtype=np.float64)
    nw = np.asarray(normals, dtype=np.float64) * np.asarray(weights, dtype=np.float64)[:, None]
    return (nw.T @ phi.T) / (4.0 * np.pi * volume)
