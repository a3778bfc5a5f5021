"""Restarted GMRES(m), float64, matrix-free.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves its dense boundary-integral system with GMRES in matrix-free
form, defining only the action of the operator (Sec. I; Sec. III, electrostatic
problem), with a relative tolerance of 1e-5 (Sec. IV.B). Restart length and
iteration cap are not stated; the readings here are restart m = 30 and at
most 500 iterations, zero initial guess, no preconditioner, and convergence
when ||b - A x|| / ||b|| <= rtol, with the true residual recomputed at every
restart (Saad & Schultz's algorithm: Arnoldi with modified Gram-Schmidt, the
least-squares problem kept upper triangular by Givens rotations).

Pins (tests/test_oracle_gmres.py): agreement with numpy's dense LU solve on
random well-conditioned systems; convergence in at most n iterations on an
n x n system without restart; exact one-step convergence when b is an
eigenvector; the residual history is non-increasing within a cycle.
"""

from __future__ import annotations

import numpy as np


def gmres(matvec, b, x0=None, rtol=1e-6, restart=30, max_iter=500):
    """Solve A x = b; returns (x, iterations, relative residual, converged)."""
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0, True
    iters = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= rtol:
            return x, iters, beta / bnorm, True
        if iters >= max_iter:
            return x, iters, beta / bnorm, False
        m = min(restart, max_iter - iters)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = matvec(V[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= 1e-14 * beta
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k = j + 1
            if abs(g[j + 1]) / bnorm <= rtol or breakdown:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + V[:k].T @ y
