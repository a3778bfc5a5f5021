"""Pins of the oracle's direct sum against hand-worked values, Gauss's law and
the unit-sphere spectra (see oracle/direct.py)."""

import os

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import direct as D

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _cases():
    out = []
    for line in open(os.path.join(GOLD, "point_sums.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, trg, srcs, pot, fld = [s.strip() for s in line.split("|")]
        s = np.array([[float(v) for v in blk.split()] for blk in srcs.split(";")])
        out.append((name, np.array([[float(v) for v in trg.split()]]), s, float(pot),
                    np.array([float(v) for v in fld.split()])))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_hand_worked_point_sums(case):
    name, trg, s, pot4pi, fld4pi = case
    pot, fld = D.direct_sum(trg, s[:, :3], s[:, 3], s[:, 4:7], delta=1e-5, field=True)
    assert pot[0] * 4 * np.pi == pytest.approx(pot4pi, abs=1e-14)
    np.testing.assert_allclose(fld[0] * 4 * np.pi, fld4pi, atol=1e-14)
    p2, f2 = D.direct_sum_numpy(trg, s[:, :3], s[:, 3], s[:, 4:7], delta=1e-5)
    assert p2[0] * 4 * np.pi == pytest.approx(pot4pi, abs=1e-14)
    np.testing.assert_allclose(f2[0] * 4 * np.pi, fld4pi, atol=1e-14)


def test_c_sum_matches_numpy_twin():
    rng = np.random.default_rng(11)
    t = rng.random((257, 3))
    s = rng.random((301, 3))
    s[:5] = t[:5]  # coincident pairs are excluded on both sides
    q = rng.standard_normal(301)
    m = rng.standard_normal((301, 3))
    p, f = D.direct_sum(t, s, q, m, field=True)
    p2, f2 = D.direct_sum_numpy(t, s, q, m)
    np.testing.assert_allclose(p, p2, rtol=1e-12, atol=1e-12)
    _, fq = D.direct_sum(t, s, q, None, field=True)
    np.testing.assert_allclose(fq, f2, rtol=1e-12, atol=1e-12)


@pytest.fixture(scope="module")
def sphere():
    xyz, nrm, w = W.sphere_quadrature(20, np.zeros(3), 1.0)
    return xyz, nrm, w


def test_gauss_law_double_layer(sphere):
    """Constant double layer on a closed surface: -1 inside, 0 outside,
    principal value -1/2 on the surface (kernel d/dn_y of 1/(4 pi r))."""
    xyz, nrm, w = sphere
    inside = np.array([[0.2, -0.1, 0.3], [0.0, 0.0, 0.0]])
    outside = np.array([[3.0, 0.0, 0.0], [0.0, -2.5, 1.0]])
    pi, _ = D.direct_sum(inside, xyz, None, nrm * w[:, None])
    po, _ = D.direct_sum(outside, xyz, None, nrm * w[:, None])
    np.testing.assert_allclose(pi, -1.0, atol=2e-4)
    np.testing.assert_allclose(po, 0.0, atol=2e-4)
    pv, _ = D.direct_sum(xyz, xyz, None, nrm * w[:, None])
    # the sum omits each point's own patch; on a sphere of radius R a disc of
    # area a contributes sqrt(a/pi) / (4R) to the double layer of 1
    patch = np.sqrt(w / np.pi) / 4.0
    np.testing.assert_allclose(pv, -0.5 + patch, atol=1.5e-3)


def test_uniformly_charged_sphere_field(sphere):
    xyz, nrm, w = sphere
    x = np.array([[2.0, 0.0, 0.0], [0.0, 1.5, 1.5], [0.1, 0.2, -0.3]])
    _, f = D.direct_sum(x, xyz, w, None, field=True)
    r = np.linalg.norm(x, axis=1)
    expect = (4 * np.pi / (4 * np.pi * r ** 3))[:, None] * x
    expect[2] = 0.0
    np.testing.assert_allclose(f, expect, atol=2e-4)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_unit_sphere_spectra(sphere, l):
    xyz, nrm, w = sphere
    z = xyz[:, 2]
    y = {0: np.ones_like(z), 1: z, 2: 3 * z * z - 1}[l]
    s, _ = D.direct_sum(xyz, xyz, y * w, None)
    d, _ = D.direct_sum(xyz, xyz, None, (y * w)[:, None] * nrm)
    lam_s = np.dot(s, y) / np.dot(y, y)
    lam_d = np.dot(d, y) / np.dot(y, y)
    # each point's own patch (a disc of radius rho = sqrt(a/pi)) is left out:
    # it carries rho/2 of the single layer and -rho/(4R) of the double layer
    rho = np.mean(np.sqrt(w / np.pi))
    assert lam_s == pytest.approx(CF.single_layer_eigenvalue(l) - rho / 2, abs=1.5e-3)
    assert lam_d == pytest.approx(CF.double_layer_eigenvalue(l) + rho / 4, abs=1.5e-3)


def test_double_layer_splits_into_three_fields():
    """Eq. sum_split: the double layer equals the sum over c of the field's
    c-component with density sigma * n_c."""
    rng = np.random.default_rng(3)
    t = rng.random((200, 3))
    s = rng.random((300, 3)) + 0.02
    n = rng.standard_normal((300, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    sig = rng.standard_normal(300)
    d, _ = D.direct_sum(t, s, None, sig[:, None] * n)
    acc = np.zeros(200)
    for c in range(3):
        _, f = D.direct_sum(t, s, sig * n[:, c], None, potential=False, field=True)
        acc += f[:, c]
    np.testing.assert_allclose(d, acc, rtol=1e-11, atol=1e-12)
