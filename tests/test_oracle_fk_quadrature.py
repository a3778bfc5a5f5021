"""Pins of the quadrature variant of the magnetostatic (FK) boundary
integral (Sec. IV.A): a fifth-order rule on every flat triangle, quadrature
points as sources and mesh nodes as targets.

The rule is pinned to exact integrals of monomials on the reference
triangle, int x^i y^j = i! j! / (i + j + 2)!, for every degree up to 5 and
shown to miss at degree 6 (so it is the degree-5 rule and not a lucky
subset). The oracle's phi_2 at the nodes and the stray-field energy are
pinned to the uniformly magnetised sphere: phi_2 = -(2/3) phi_1 on the
surface (phi_1 = 4 pi M.r) and E = 8 pi^2 / 9, with the error of the
inscribed polyhedron falling by about 4 per halving of the mesh size
(linear elements, second order)."""

from math import factorial

import numpy as np

import workloads as W
from oracle import closed_forms as CF
from oracle import operators as OP


def _tri_integral(bary, w, i, j):
    # reference triangle (0,0), (1,0), (0,1): area 1/2; x = b1, y = b2
    x, y = bary[:, 1], bary[:, 2]
    return 0.5 * np.sum(w * x ** i * y ** j)


def test_rule_is_exact_to_degree_five():
    bary, w = W.triangle_rule_deg5()
    assert bary.shape == (7, 3) and np.allclose(bary.sum(axis=1), 1.0)
    assert np.all(bary > 0) and np.all(w > 0)
    assert abs(w.sum() - 1.0) < 1e-15
    for deg in range(6):
        for i in range(deg + 1):
            exact = factorial(i) * factorial(deg - i) / factorial(deg + 2)
            assert abs(_tri_integral(bary, w, i, deg - i) - exact) < 1e-15, (i, deg - i)
    miss = max(abs(_tri_integral(bary, w, i, 6 - i) - factorial(i) * factorial(6 - i) / factorial(8))
               for i in range(7))
    assert miss > 1e-6


def test_mesh_quadrature_integrates_the_polyhedron():
    v, t = W.icosphere(6)
    bary, w = W.triangle_rule_deg5()
    pts, nrm, wq = W.mesh_quadrature(v, t, bary, w)
    assert pts.shape == (7 * len(t), 3) and nrm.shape == pts.shape
    # divergence theorem on the polyhedron: int x.n dA = 3 V, int n dA = 0
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    vol = np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0
    assert abs(np.sum(np.einsum("ij,ij->i", pts, nrm) * wq) - 3.0 * vol) < 1e-12
    assert np.abs((nrm * wq[:, None]).sum(axis=0)).max() < 1e-13
    # points lie in their triangle's plane, normals outward
    assert np.abs(np.einsum("ij,ij->i", pts - np.repeat(a, 7, axis=0), nrm)).max() < 1e-14
    assert np.all(np.einsum("ij,ij->i", pts, nrm) > 0)


def test_phi2_and_energy_converge_at_second_order():
    bary, w = W.triangle_rule_deg5()
    m = np.array([0.6, 0.0, 0.8])
    errs, eerrs = [], []
    for freq in (4, 8, 16):
        v, t = W.icosphere(freq)
        phi1 = 4.0 * np.pi * (v @ m)
        phi2 = OP.fk_phi2_at_nodes(phi1, v, t, bary, w)
        exact = CF.sphere_phi2(v, m)
        errs.append(np.linalg.norm(phi2 - exact) / np.linalg.norm(exact))
        e = OP.stray_energy_on_mesh(phi1 + phi2, m, v, t, bary, w)
        eerrs.append(abs(e - CF.SPHERE_ENERGY) / CF.SPHERE_ENERGY)
    assert errs[-1] < 1e-3 and eerrs[-1] < 5e-3
    for k in range(2):
        assert 3.5 < errs[k] / errs[k + 1] < 4.6, errs
        assert 3.5 < eerrs[k] / eerrs[k + 1] < 4.6, eerrs


def test_without_the_subtraction_the_solid_angle_is_first_order():
    """The plain sum D[phi_1] - phi_1 / 2 (Omega = 2 pi at a smooth point)
    is far worse at the nodes: the rule resolves the kernel poorly on the
    triangles next to the target, which the subtraction cancels."""
    bary, w = W.triangle_rule_deg5()
    m = np.array([1.0, 0.0, 0.0])
    v, t = W.icosphere(8)
    phi1 = 4.0 * np.pi * (v @ m)
    good = OP.fk_phi2_at_nodes(phi1, v, t, bary, w)
    from oracle import direct as D
    pts, nrm, wq = W.mesh_quadrature(v, t, bary, w)
    d1, _ = D.direct_sum(v, pts, None, ((phi1[t] @ bary.T).reshape(-1) * wq)[:, None] * nrm)
    plain = d1 - 0.5 * phi1
    exact = CF.sphere_phi2(v, m)
    e_good = np.linalg.norm(good - exact) / np.linalg.norm(exact)
    e_plain = np.linalg.norm(plain - exact) / np.linalg.norm(exact)
    assert e_plain > 5 * e_good
