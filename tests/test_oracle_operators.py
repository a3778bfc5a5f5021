"""Closed-form pins of the two model problems' operators on the direct sum
(see oracle/operators.py and oracle/closed_forms.py)."""

import os

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import direct as D
from oracle import operators as OP
from oracle.gmres import gmres

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper(name):
    for line in open(os.path.join(GOLD, "paper_constants.txt")):
        if line.startswith(name + " "):
            return float(line.split()[1])
    raise KeyError(name)


@pytest.fixture(scope="module")
def sphere():
    return W.sphere_quadrature(24, np.zeros(3), 1.0)


def test_uniformly_magnetised_sphere_demag_factor(sphere):
    """Sec. IV.A: stray field 4 pi/3 along M inside the unit sphere.

    With targets equal to sources each point's own patch (a disc of radius
    rho = sqrt(a/pi)) is left out of the double layer; on the unit sphere it
    would contribute -(rho/4) phi_1, so the discrete phi = phi_1 + phi_2 is
    (4 pi/3 + pi rho) x to first order in rho."""
    xyz, nrm, w = sphere
    rho = np.sqrt(w / np.pi)
    m = np.array([1.0, 0.0, 0.0])
    phi1 = 4 * np.pi * xyz @ m
    a = np.full(len(w), 2 * np.pi / (4 * np.pi) - 1.0)  # Omega = 2 pi on a sphere
    phi2 = OP.fk_apply(phi1, xyz, nrm, w, a)
    np.testing.assert_allclose(phi2, CF.sphere_phi2(xyz, m) + np.pi * rho * xyz[:, 0], atol=6e-3)
    # H = -grad(phi1 + phi2): least-squares gradient of the surface values
    g = np.linalg.lstsq(np.c_[xyz, np.ones(len(xyz))], phi1 + phi2, rcond=None)[0][:3]
    rbar = rho.mean()
    assert g[0] == pytest.approx(_paper("sphere_stray_field_along_M") + np.pi * rbar, rel=1e-3)
    assert abs(g[1]) < 1e-9 and abs(g[2]) < 1e-9
    n = CF.demag_tensor_from_surface(np.stack([phi1 + phi2] + [np.zeros_like(phi1)] * 2), nrm, w, 4 * np.pi / 3)
    assert n[0, 0] == pytest.approx(CF.SPHERE_DEMAG + rbar / 4, rel=2e-3)
    e = 0.5 * np.sum((phi1 + phi2) * (nrm @ m) * w)
    assert e == pytest.approx(CF.SPHERE_ENERGY + (2 * np.pi ** 2 / 3) * rbar, rel=2e-3)


def _cube_fk(n_nodes):
    _, cen, nrm, area, _ = W.cube_surface(1.0, n_nodes)
    phis = []
    for c in range(3):
        phi1 = 4 * np.pi * cen[:, c]
        a = np.full(len(cen), 2 * np.pi / (4 * np.pi) - 1.0)
        phis.append(phi1 + OP.fk_apply(phi1, cen, nrm, area, a))
    n = CF.demag_tensor_from_surface(np.stack(phis), nrm, area, 1.0)
    e = 0.5 * np.sum(phis[0] * nrm[:, 0] * area)
    return n, e


def test_unit_cube_demag_tensor_and_energy():
    """Sec. IV.A: unit cube, unit M: N = I/3 and stray-field energy 2 pi/3.
    Targets are the triangle centroids (solid angle 2 pi on a face). The
    flat-element centroid rule converges at first order in the mesh size."""
    n1, e1 = _cube_fk(1500)
    n2, e2 = _cube_fk(6000)
    assert np.trace(n2) == pytest.approx(1.0, abs=1e-2)
    np.testing.assert_allclose(n2, np.eye(3) / 3, atol=3e-3)
    target = _paper("cube_stray_field_energy")
    assert e2 == pytest.approx(target, rel=1e-2)
    assert abs(e2 - target) < 0.6 * abs(e1 - target)
    assert abs(np.trace(n2) - 1) < 0.6 * abs(np.trace(n1) - 1)


def test_dielectric_sphere_in_uniform_field(sphere):
    xyz, nrm, w = sphere
    eps_i, eps_m, e0 = 5.0, 1.0, np.array([0.0, 0.0, 1.0])
    ei = np.full(len(w), eps_i)
    a, c, ww = OP.dielectric_coeffs(w, np.ones(len(w)), ei, eps_m)
    b = OP.dielectric_rhs(nrm, ei, eps_m, e0)
    x, it, rr, ok = gmres(lambda s: OP.dielectric_apply(s, xyz, nrm, a, c, ww), b, rtol=1e-8)
    assert ok
    expect = CF.dielectric_sphere_sigma(nrm, eps_i, eps_m, e0)
    assert D.rel_l2(x, expect) < 2e-3


def test_interior_dirichlet_on_sphere(sphere):
    """(D_pv - I/2) mu = x on the unit sphere has mu = -(3/2) x. The omitted
    self patch shifts the discrete eigenvalue -2/3 by rho/4."""
    xyz, nrm, w = sphere
    a = np.full(len(w), -0.5)
    g = xyz[:, 0]
    x, it, rr, ok = gmres(lambda v: OP.fk_apply(v, xyz, nrm, w, a), g, rtol=1e-10)
    assert ok
    rbar = np.mean(np.sqrt(w / np.pi))
    assert D.rel_l2(x, g / (-2.0 / 3.0 + rbar / 4)) < 1e-3


def test_ellipsoid_demag_factors():
    n = CF.ellipsoid_demag((1.0, 1.0, 1.0))
    np.testing.assert_allclose(n, 1 / 3, rtol=1e-10)
    n = CF.ellipsoid_demag((2.0, 1.0, 0.5))
    assert n.sum() == pytest.approx(1.0, abs=1e-10)
    assert n[0] < n[1] < n[2]


def _two_spheres(d, freq, eps=15.0, eps_m=1.0, charges=(1.0, 10.0)):
    """Two unit spheres on the x axis, centres -d/2 and +d/2, free charges
    charges[i] spread uniformly (sigma_f = Q / (4 pi r^2), Sec. II.C)."""
    parts = [W.sphere_quadrature(freq, np.array([sx, 0.0, 0.0]), 1.0) for sx in (-d / 2, d / 2)]
    xyz = np.concatenate([p[0] for p in parts]).astype(np.float64)
    nrm = np.concatenate([p[1] for p in parts]).astype(np.float64)
    a = np.concatenate([p[2] for p in parts]).astype(np.float64)
    n1 = len(parts[0][2])
    sf = np.concatenate([np.full(n1, charges[0] / (4 * np.pi)), np.full(len(a) - n1, charges[1] / (4 * np.pi))])
    return xyz, nrm, a, np.ones(len(a)), sf, np.full(len(a), eps), eps_m, [0, n1, len(a)]


def _forces(system, rtol=1e-9):
    xyz, nrm, a, curv, sf, ei, eps_m, off = system
    A, c, w = OP.dielectric_coeffs(a, curv, ei, eps_m)
    b = OP.dielectric_rhs_free(xyz, nrm, a, curv, sf, ei, eps_m)
    sb, it, rr, ok = gmres(lambda s: OP.dielectric_apply(s, xyz, nrm, A, c, w), b, rtol=rtol)
    assert ok
    return OP.body_forces(xyz, nrm, a, curv, sf + sb, eps_m, off), sb


def test_charged_sphere_gauss_law(sphere):
    """An isolated sphere with free charge Q in a medium eps_m carries total
    charge Q / eps_m: sigma_b = (1/eps_m - 1) sigma_f, uniform."""
    xyz, nrm, w = sphere
    n = len(w)
    eps_i, eps_m = 5.0, 2.0
    sf = np.full(n, 3.0 / (4 * np.pi))
    ei = np.full(n, eps_i)
    a, c, ww = OP.dielectric_coeffs(w, np.ones(n), ei, eps_m)
    b = OP.dielectric_rhs_free(xyz, nrm, w, np.ones(n), sf, ei, eps_m)
    sb, it, rr, ok = gmres(lambda s: OP.dielectric_apply(s, xyz, nrm, a, c, ww), b, rtol=1e-10)
    assert ok
    assert D.rel_l2(sb, (1.0 / eps_m - 1.0) * sf) < 5e-3


def test_distant_charged_spheres_coulomb():
    """Far apart, the force is Coulomb's in the medium, Q1 Q2 / (4 pi eps_m d^2),
    and the two forces balance."""
    q1, q2, eps_m, d = 2.0, 3.0, 1.5, 12.0
    (f1, f2), _ = _forces(_two_spheres(d, 8, eps=4.0, eps_m=eps_m, charges=(q1, q2)))
    coulomb = q1 * q2 / (4 * np.pi * eps_m * d * d)
    assert abs(f2[0] / coulomb - 1.0) < 1e-2
    assert np.linalg.norm(f1 + f2) < 1e-3 * coulomb
    assert abs(f2[1]) + abs(f2[2]) < 1e-3 * coulomb


def test_two_dielectric_spheres_force_sign_change():
    """Like-charged polarisable spheres (eps 15, charges q and 10q, eps_m 1)
    attract when close: the force changes sign at the separation the paper
    prints (Sec. IV.B), located by linear interpolation of the force."""
    d_paper = _paper("force_sign_change_separation")
    ds = [2.6, 2.7, 2.8, 2.9]
    fx = [_forces(_two_spheres(d, 8))[0][1][0] for d in ds]
    assert fx[0] < 0 and fx[-1] > 0
    k = next(i for i in range(len(ds) - 1) if fx[i] < 0 <= fx[i + 1])
    root = ds[k] + (ds[k + 1] - ds[k]) * (-fx[k]) / (fx[k + 1] - fx[k])
    assert abs(root - d_paper) < 0.03, root
