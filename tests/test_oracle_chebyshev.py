"""Pins of the Chebyshev-interpolation oracle (Sec. III.A.1 Eq. p2m) against
facts that do not come from the oracle itself: numpy's Chebyshev series, the
textbook Lagrange product formula, polynomial reproduction, exactness of the
nested interpolation in M2M/L2L, homogeneity of the kernel and convergence
to the direct sum."""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import polynomial as nppoly

from oracle import chebyshev as C
from oracle import direct as D
from oracle import tree as T
from oracle.kifmm import octant_sign, slp


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_nodes_are_the_zeros_of_t_n(n):
    x = C.nodes_1d(n)
    assert np.all(np.abs(x) < 1) and len(np.unique(x)) == n
    assert np.max(np.abs(npcheb.chebval(x, [0] * n + [1]))) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 5, 7])
def test_interpolant_is_the_lagrange_polynomial(n):
    """S_n(xbar_i, t) = prod_{j != i} (t - xbar_j) / (xbar_i - xbar_j), and
    its derivative, from numpy's power-series polynomials."""
    x = C.nodes_1d(n)
    t = np.linspace(-1.0, 1.0, 37)
    s = C.interp_1d(n, t)
    ds = C.interp_1d(n, t, deriv=True)
    for i in range(n):
        others = np.delete(x, i)
        c = nppoly.polyfromroots(others) / np.prod(x[i] - others)
        assert np.allclose(s[i], nppoly.polyval(t, c), atol=1e-12)
        assert np.allclose(ds[i], nppoly.polyval(t, nppoly.polyder(c)), atol=1e-10)
    # cardinal property at the nodes
    assert np.allclose(C.interp_1d(n, x), np.eye(n), atol=1e-13)


def test_interpolation_reproduces_polynomials_in_3d():
    n = 5
    rng = np.random.default_rng(3)
    coef = rng.standard_normal((n, n, n))  # degree <= n - 1 per axis

    def p(t):
        return np.einsum("abc,pa,pb,pc->p", coef, *(np.vander(t[:, k], n, increasing=True) for k in range(3)))

    def grad(t):
        v = [np.vander(t[:, k], n, increasing=True) for k in range(3)]
        dv = [np.hstack([np.zeros((len(t), 1)), v[k][:, :-1] * np.arange(1, n)]) for k in range(3)]
        return np.stack([np.einsum("abc,pa,pb,pc->p", coef, dv[0], v[1], v[2]),
                         np.einsum("abc,pa,pb,pc->p", coef, v[0], dv[1], v[2]),
                         np.einsum("abc,pa,pb,pc->p", coef, v[0], v[1], dv[2])])

    X = C.nodes_3d(n)
    t = rng.uniform(-1, 1, (50, 3))
    assert np.allclose(C.interp_3d(n, t).T @ p(X), p(t), rtol=1e-11, atol=1e-11)
    g = C.interp_3d_grad(n, t)
    for c in range(3):
        assert np.allclose(g[c].T @ p(X), grad(t)[c], rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("o", range(8))
def test_m2m_and_l2l_are_exact(o):
    """P2M of sources in child o, moved up by M2M, equals P2M at the parent;
    a parent expansion moved down by L2L gives the same values in the child."""
    n = 4
    ops = C.ChebOperators(n)
    rng = np.random.default_rng(o)
    y = 0.5 * octant_sign(o) + rng.uniform(-0.5, 0.5, (40, 3))  # in child o of the unit box
    q = rng.standard_normal(40)
    m = rng.standard_normal((40, 3))
    w_child = C.interp_3d(n, (y - 0.5 * octant_sign(o)) / 0.5) @ q
    g = C.interp_3d_grad(n, (y - 0.5 * octant_sign(o)) / 0.5)
    w_child += sum(g[c] @ m[:, c] for c in range(3)) / 0.5
    w_parent = C.interp_3d(n, y) @ q + sum(C.interp_3d_grad(n, y)[c] @ m[:, c] for c in range(3))
    assert np.allclose(ops.m2m[o] @ w_child, w_parent, rtol=1e-11, atol=1e-11)
    lp = rng.standard_normal(n ** 3)
    lc = ops.m2m[o].T @ lp
    x = 0.5 * octant_sign(o) + rng.uniform(-0.5, 0.5, (30, 3))
    assert np.allclose(C.interp_3d(n, (x - 0.5 * octant_sign(o)) / 0.5).T @ lc, C.interp_3d(n, x).T @ lp,
                       rtol=1e-11, atol=1e-11)


def test_m2l_translation_scales_with_half_width():
    """K between the nodes of two boxes of half-width h, centres 2 h d apart,
    is the unit-box matrix divided by h (homogeneity of 1/r)."""
    n = 3
    ops = C.ChebOperators(n)
    k = 77
    d = ops.dirs[k].astype(np.float64)
    h, c = 0.037, np.array([0.3, -0.2, 0.9])
    direct = slp(c + h * ops.X, c + 2 * h * d + h * ops.X)
    assert np.allclose(direct, ops.dense(k) / h, rtol=1e-13)


def test_compression_without_truncation_is_the_dense_translation():
    n = 3
    ops = C.ChebOperators(n, eps=1e-300)
    assert ops.rank == n ** 3
    w = np.random.default_rng(1).standard_normal((n ** 3, 4))
    for k in (0, 100, 315):
        assert np.allclose(ops.translate(k, w), ops.dense(k) @ w, rtol=1e-10, atol=1e-12)


def _cloud(npts, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((npts, 3))
    blob = rng.normal(0.3, 0.04, (npts // 2, 3))
    x[: npts // 2] = np.clip(blob, 0, 1)
    nrm = rng.standard_normal((npts, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return x, nrm, rng.standard_normal(npts), rng.standard_normal(npts)


def test_fmm_converges_to_the_direct_sum():
    """Single layer, double layer (method-2 P2M), both, and the field: the
    error against the direct sum falls with the order."""
    x, nrm, q, mu = _cloud(2500, 4)
    t = T.build_tree(x, leaf_size=30)
    L = T.all_lists(t)
    dip = mu[:, None] * nrm
    ref_sl, ref_f = D.direct_sum_numpy(x, x, q, None)
    ref_dl, _ = D.direct_sum_numpy(x, x, None, dip)
    errs = []
    for n in (3, 4, 6):
        ops = C.ChebOperators(n)
        sl, fld = C.cheb_apply(t, L, ops, x, q=q, field=True)
        dl, _ = C.cheb_apply(t, L, ops, x, mu=mu, normals=nrm)
        both, _ = C.cheb_apply(t, L, ops, x, q=q, mu=mu, normals=nrm)
        assert np.allclose(both, sl + dl, rtol=1e-12, atol=1e-12)
        errs.append((D.rel_l2(sl, ref_sl), D.rel_l2(dl, ref_dl), D.rel_l2(fld, ref_f)))
    errs = np.array(errs)
    assert np.all(errs[1:] < 0.5 * errs[:-1])
    assert errs[-1, 0] < 2e-5 and errs[-1, 1] < 2e-4 and errs[-1, 2] < 2e-4


def test_fmm_with_compressed_translations_and_separate_targets():
    x, nrm, q, _ = _cloud(1800, 5)
    trg = np.random.default_rng(9).random((700, 3))
    t = T.build_tree(x, trg=trg, leaf_size=25)
    L = T.all_lists(t)
    ref, _ = D.direct_sum_numpy(trg, x, q, None)
    dense, _ = C.cheb_apply(t, L, C.ChebOperators(5), x, q=q, trg_xyz=trg)
    comp, _ = C.cheb_apply(t, L, C.ChebOperators(5, eps=1e-6), x, q=q, trg_xyz=trg)
    e_dense, e_comp = D.rel_l2(dense, ref), D.rel_l2(comp, ref)
    assert e_dense < 1e-4
    assert e_comp < 1.2 * e_dense
