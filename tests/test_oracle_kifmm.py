"""Pins of the oracle's float64 KIFMM (see oracle/kifmm.py)."""

import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle import kifmm as K
from oracle import tree as T


def test_pinv_is_a_generalised_inverse():
    Y = K.surface(6)
    k = K.slp(K.RAD_OUT * Y, K.RAD_IN * Y)
    kp = K.pinv(k, 1e-12)
    np.testing.assert_allclose(k @ kp @ k, k, atol=1e-9 * np.abs(k).max())


def test_surface_counts():
    for p in (4, 6, 8, 10):
        assert len(K.surface(p)) == 6 * (p - 1) ** 2 + 2


def test_c2e_scales_linearly_with_box_size():
    """Homogeneity of 1/r: the check-to-equivalent map of a box of half-width r
    is r times the unit box's map."""
    Y = K.surface(5)
    r = 0.125
    k1 = K.pinv(K.slp(K.RAD_OUT * Y, K.RAD_IN * Y), 1e-10)
    kr = K.pinv(K.slp(K.RAD_OUT * r * Y, K.RAD_IN * r * Y), 1e-10)
    np.testing.assert_allclose(kr, r * k1, rtol=1e-6, atol=1e-8 * np.abs(kr).max())


def test_upward_equivalent_density_reproduces_far_potential():
    rng = np.random.default_rng(2)
    src = rng.uniform(-1, 1, (60, 3))
    q = rng.standard_normal(60)
    ops = K.Operators(8, 1e-10)
    u, _ = D.direct_sum_numpy(K.RAD_OUT * ops.Y, src, q, None, 0.0)
    phi = ops.uc2e @ u
    far = rng.standard_normal((40, 3))
    far = 4.5 * far / np.linalg.norm(far, axis=1, keepdims=True)
    approx = K.slp(far, K.RAD_IN * ops.Y) @ phi
    exact, _ = D.direct_sum_numpy(far, src, q, None, 0.0)
    assert D.rel_l2(approx, exact) < 1e-6


@pytest.fixture(scope="module")
def cube():
    d = W.cube_uniform()
    t = T.build_tree(d["xyz"], uniform_depth=3, root=d["root"])
    return d, t, T.all_lists(t), D.direct_sum(d["xyz"], d["xyz"], d["q"])[0]


def test_error_decreases_with_order(cube):
    d, t, L, ref = cube
    errs = []
    for p, eps in ((4, 1e-10), (6, 1e-10), (8, 1e-10)):
        pot, _ = K.kifmm_apply(t, L, K.Operators(p, eps), d["xyz"], q=d["q"])
        errs.append(D.rel_l2(pot, ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 5e-6 and errs[2] < 1e-7


def _adaptive_case(seed=7, n=2500):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.random((n // 2, 3)), 0.6 + 0.03 * rng.standard_normal((n - n // 2, 3))])
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return x.astype(np.float32), nrm.astype(np.float32), rng.standard_normal(n), rng.standard_normal(n)


def test_adaptive_single_and_double_layer():
    x, nrm, q, mu = _adaptive_case()
    t = T.build_tree(x, leaf_size=24)
    L = T.all_lists(t)
    assert sum(len(v) for v in L["W"].values()) > 0
    ref, _ = D.direct_sum(x, x, q, mu[:, None] * nrm.astype(np.float64))
    pot, _ = K.kifmm_apply(t, L, K.Operators(6, 1e-10), x, q=q, mu=mu, normals=nrm)
    assert D.rel_l2(pot, ref) < 3e-5
    pot, _ = K.kifmm_apply(t, L, K.Operators(8, 1e-10), x, q=q, mu=mu, normals=nrm)
    assert D.rel_l2(pot, ref) < 1e-6
    ref, _ = D.direct_sum(x, x, q)
    pot, _ = K.kifmm_apply(t, L, K.Operators(6, 1e-10), x, q=q)
    assert D.rel_l2(pot, ref) < 5e-6


def test_field_output_and_method1_split():
    """Double layer through P2M (method 2) equals the sum of the three field
    components with densities mu n_c (method 1, Eq. sum_split)."""
    x, nrm, q, mu = _adaptive_case(8, 1500)
    t = T.build_tree(x, leaf_size=20)
    L = T.all_lists(t)
    ops = K.Operators(6, 1e-10)
    _, fref = D.direct_sum(x, x, q, None, field=True)
    _, f = K.kifmm_apply(t, L, ops, x, q=q, field=True)
    assert D.rel_l2(f, fref) < 2e-4
    dl, _ = K.kifmm_apply(t, L, ops, x, mu=mu, normals=nrm)
    acc = np.zeros(len(x))
    for c in range(3):
        _, fc = K.kifmm_apply(t, L, ops, x, q=mu * nrm[:, c], field=True)
        acc += fc[:, c]
    assert D.rel_l2(dl, acc) < 1e-4


def test_separate_targets_and_sources():
    rng = np.random.default_rng(5)
    trg = rng.random((700, 3)).astype(np.float32)
    src = (0.5 + 0.15 * rng.standard_normal((1200, 3))).astype(np.float32)
    q = rng.standard_normal(1200)
    t = T.build_tree(src, trg=trg, leaf_size=30)
    L = T.all_lists(t)
    pot, _ = K.kifmm_apply(t, L, K.Operators(6, 1e-10), src, q=q, trg_xyz=trg)
    ref, _ = D.direct_sum(trg, src, q)
    assert D.rel_l2(pot, ref) < 1e-5
