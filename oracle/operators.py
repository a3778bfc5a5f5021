"""Boundary operators of the paper's two model problems, on the direct sum (float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Both are written as y = a * x + K[w * x] with per-point coefficients, the
form the GPU library's GMRES operator takes:

  FK (magnetostatic, Sec. II.B Eq. fk_integral, Sec. III.A.1 Eq.
  fk_integral_discrete): phi_2 = D[phi_1 w] + (Omega/(4 pi) - 1) phi_1,
  D the double layer with kernel (x - y).n_y / (4 pi |x - y|^3). So
  a = Omega/(4 pi) - 1 and the double-layer density is w * x.

  Dielectric (Sec. II.C Eqs. linear_system, Ax, Eb; Sec. III.A.2 Eq.
  pol_discret), with epsilon_0 = 1:
    (A s)_j = ebar_j s_j + deps_j [ n_j . E_j + s_j sqrt(pi a_j) H_j / (4 pi) ]
    E_j = sum_{k != j} (r_j - r_k) s_k a_k / (4 pi |r_j - r_k|^3)
  ebar = (eps_i + eps_m)/2, deps = eps_m - eps_i. The self-patch term is a
  reading: the printed term sqrt(a_j/pi) H_j n_j lacks the density s_j and a
  factor pi; the principal-value field of a uniformly charged spherical cap of
  area a is s sqrt(pi a) H / (4 pi). So a = ebar + deps sqrt(pi a) H/(4 pi),
  c = deps, w = area. Right-hand side (Eq. rhs, no free charges, uniform
  field E0): b = -deps E0 . n.

Pins: tests/test_oracle_operators.py (sphere closed forms in closed_forms).
"""

from __future__ import annotations

import numpy as np

from .direct import direct_sum


def fk_apply(x, xyz, normals, weights, a, delta=1e-5, matvec_dl=None):
    """y = a * x + D[w * x] on the same points (targets = sources)."""
    x = np.asarray(x, dtype=np.float64)
    dens = x * np.asarray(weights, dtype=np.float64)
    if matvec_dl is None:
        pot, _ = direct_sum(xyz, xyz, None, dens[:, None] * np.asarray(normals, dtype=np.float64), delta)
    else:
        pot = matvec_dl(dens)
    return np.asarray(a, dtype=np.float64) * x + pot


def dielectric_coeffs(areas, curvature, eps_i, eps_m):
    """(a, c, w) of the dielectric operator y = a*x + c*(n . E[w*x])."""
    areas = np.asarray(areas, dtype=np.float64)
    eps_i = np.asarray(eps_i, dtype=np.float64)
    ebar = 0.5 * (eps_i + eps_m)
    deps = eps_m - eps_i
    self_term = np.sqrt(np.pi * areas) * np.asarray(curvature, dtype=np.float64) / (4.0 * np.pi)
    return ebar + deps * self_term, deps, areas


def dielectric_rhs(normals, eps_i, eps_m, e0):
    """b = -deps * E0 . n (Eq. rhs with sigma_f = 0, rho_f = 0, uniform external field)."""
    deps = eps_m - np.asarray(eps_i, dtype=np.float64)
    return -deps * (np.asarray(normals, dtype=np.float64) @ np.asarray(e0, dtype=np.float64))


def dielectric_apply(x, xyz, normals, a, c, w, delta=1e-5, matvec_field=None):
    """y = a * x + c * (n . E[w * x]) on the same points."""
    x = np.asarray(x, dtype=np.float64)
    dens = x * np.asarray(w, dtype=np.float64)
    if matvec_field is None:
        _, fld = direct_sum(xyz, xyz, dens, None, delta, potential=False, field=True)
    else:
        fld = matvec_field(dens)
    en = np.einsum("ij,ij->i", fld, np.asarray(normals, dtype=np.float64))
    return np.asarray(a, dtype=np.float64) * x + np.asarray(c, dtype=np.float64) * en
