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

  Free charges and body forces (Sec. II.C, Eqs. rhs, Ef and the force
  integral): with free surface charge sigma_f on the bodies (a charge Q_i on
  sphere i of radius r_i is sigma_f = Q_i / (4 pi r_i^2)) and an optional
  uniform external field E0,
    b = (1 - ebar) sigma_f - deps (n . E_f) - deps (n . E0),
  E_f the field of sigma_f discretised as Eq. pol_discret (the same self
  term). The force on body i is the sum over its elements of
  eps_m sigma_j E_j a_j with sigma = sigma_f + sigma_b and E the field of
  sigma (with its self term) plus E0.

  Quadrature variant of FK (Sec. IV.A): sources at the points of a
  fifth-order rule on every flat triangle, targets at the mesh nodes
  (fk_phi2_at_nodes), and the stray-field energy of the nodal potential
  (stray_energy_on_mesh).

Pins: tests/test_oracle_operators.py (sphere closed forms in closed_forms,
Gauss's law for a charged sphere, Coulomb's law for distant spheres, the
paper's force sign change between two charged dielectric spheres) and
tests/test_oracle_fk_quadrature.py (the rule's exactness, second-order
convergence of phi_2 and the energy to the sphere's closed forms).
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


def surface_field(xyz, normals, areas, curvature, sigma, delta=1e-5, matvec_field=None):
    """E_j = sum_{k != j} (r_j - r_k) s_k a_k / (4 pi r^3) + s_j sqrt(pi a_j) H_j / (4 pi) n_j."""
    areas = np.asarray(areas, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    dens = s * areas
    if matvec_field is None:
        _, fld = direct_sum(xyz, xyz, dens, None, delta, potential=False, field=True)
    else:
        fld = matvec_field(dens)
    self_term = s * np.sqrt(np.pi * areas) * np.asarray(curvature, dtype=np.float64) / (4.0 * np.pi)
    return fld + self_term[:, None] * np.asarray(normals, dtype=np.float64)


def dielectric_rhs_free(xyz, normals, areas, curvature, sigma_f, eps_i, eps_m, e0=None, delta=1e-5):
    """b = (1 - ebar) sigma_f - deps n . (E_f + E0)  (Eq. rhs with Eq. Ef, no volume charge)."""
    eps_i = np.asarray(eps_i, dtype=np.float64)
    ebar = 0.5 * (eps_i + eps_m)
    deps = eps_m - eps_i
    nrm = np.asarray(normals, dtype=np.float64)
    ef = surface_field(xyz, nrm, areas, curvature, sigma_f, delta)
    if e0 is not None:
        ef = ef + np.asarray(e0, dtype=np.float64)
    return (1.0 - ebar) * np.asarray(sigma_f, dtype=np.float64) - deps * np.einsum("ij,ij->i", ef, nrm)


def body_forces(xyz, normals, areas, curvature, sigma, eps_m, body_off, e0=None, delta=1e-5):
    """F_i = sum_{j in body i} eps_m sigma_j E_j a_j; bodies are the index ranges body_off[i]..body_off[i+1]."""
    e = surface_field(xyz, normals, areas, curvature, sigma, delta)
    if e0 is not None:
        e = e + np.asarray(e0, dtype=np.float64)
    f = eps_m * (np.asarray(sigma, dtype=np.float64) * np.asarray(areas, dtype=np.float64))[:, None] * e
    return np.array([f[body_off[i]:body_off[i + 1]].sum(axis=0) for i in range(len(body_off) - 1)])


def fk_phi2_at_nodes(phi1, verts, tris, bary, weights, delta=1e-5):
    """phi_2 at the mesh nodes with the double layer integrated by a quadrature
    rule on every flat triangle (Sec. II.B Eq. fk_integral; Sec. IV.A: a
    fifth-order rule, quadrature points as sources and nodes as targets).

    phi_1 is linear on each triangle (nodal values phi1). The solid-angle term
    is taken from the same quadrature: Gauss's identity gives
    Omega(x)/(4 pi) = -D[1](x) at a boundary node, so
      phi_2(x) = D[phi_1](x) + (Omega(x)/(4 pi) - 1) phi_1(x)
               = D[phi_1](x) - phi_1(x) D[1](x) - phi_1(x),
    which integrates the density phi_1 - phi_1(x), zero at the target, where
    the rule is least accurate.
    """
    from workloads import mesh_quadrature

    pts, nrm, w = mesh_quadrature(verts, tris, bary, weights)
    phi1 = np.asarray(phi1, dtype=np.float64)
    phi1_q = (phi1[tris] @ np.asarray(bary).T).reshape(-1)
    d_phi1, _ = direct_sum(verts, pts, None, (phi1_q * w)[:, None] * nrm, delta)
    d_one, _ = direct_sum(verts, pts, None, w[:, None] * nrm, delta)
    return d_phi1 - phi1 * d_one - phi1


def stray_energy_on_mesh(phi, m, verts, tris, bary, weights):
    """E = 1/2 surface-integral phi (M . n) dA (Sec. IV.A) with phi linear on
    each flat triangle (nodal values) and the same quadrature rule."""
    from workloads import mesh_quadrature

    _, nrm, w = mesh_quadrature(verts, tris, bary, weights)
    phi_q = (np.asarray(phi, dtype=np.float64)[tris] @ np.asarray(bary).T).reshape(-1)
    return 0.5 * float(np.sum(phi_q * (nrm @ np.asarray(m, dtype=np.float64)) * w))
