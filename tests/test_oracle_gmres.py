"""Pins of the oracle's GMRES(m) (see oracle/gmres.py)."""

import numpy as np

from oracle.gmres import gmres


def _system(n, seed):
    rng = np.random.default_rng(seed)
    a = np.eye(n) * 3.0 + rng.standard_normal((n, n)) / np.sqrt(n)
    return a, rng.standard_normal(n)


def test_matches_dense_lu():
    a, b = _system(200, 1)
    x, it, rr, ok = gmres(lambda v: a @ v, b, rtol=1e-12, restart=30, max_iter=500)
    assert ok and rr <= 1e-12
    np.testing.assert_allclose(x, np.linalg.solve(a, b), rtol=1e-9, atol=1e-10)


def test_exact_within_n_steps_without_restart():
    a, b = _system(25, 2)
    a = a + 5.0 * np.diag(np.arange(25))  # widely spread spectrum
    x, it, rr, ok = gmres(lambda v: a @ v, b, rtol=1e-13, restart=25, max_iter=25)
    assert ok and it <= 25
    np.testing.assert_allclose(a @ x, b, atol=1e-9)


def test_eigenvector_rhs_converges_in_one_step():
    a = np.diag(np.arange(1.0, 11.0))
    b = np.zeros(10)
    b[3] = 2.0
    x, it, rr, ok = gmres(lambda v: a @ v, b, rtol=1e-14)
    assert ok and it == 1
    assert abs(x[3] - 0.5) < 1e-14


def test_not_converged_is_reported():
    a, b = _system(100, 3)
    x, it, rr, ok = gmres(lambda v: a @ v, b, rtol=1e-14, restart=5, max_iter=3)
    assert not ok and it == 3 and rr > 1e-14
    assert np.linalg.norm(b - a @ x) / np.linalg.norm(b) < 1.0
