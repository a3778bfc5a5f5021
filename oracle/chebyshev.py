"""Chebyshev-interpolation FMM in float64 (the paper's own far-field form).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. III.A.1, Eq. p2m: the far field between two well-separated boxes is
interpolated on Chebyshev nodes at both ends, with the plain 1/r kernel
between the nodes; the double layer's normal derivative is applied to the
source-side interpolating polynomial (the paper's second method). The
steps, for order n (n nodes per axis, n^3 per box):

  nodes      1D: xbar_i = cos((2i - 1) pi / (2n)), i = 1..n, on [-1, 1];
             3D: tensor products, index m = (i n + j) n + k with i along x.
             A box with centre c and half-width h maps x to t = (x - c) / h.
  S_n        S_n(xbar_i, t) = 1/n + (2/n) sum_{k=1}^{n-1} T_k(xbar_i) T_k(t),
             the Lagrange polynomial of node i written in the Chebyshev
             basis; in 3D the product over the axes.
  P2M        W_m = sum_j q_j S(ybar_m, y_j) + mu_j n_j . grad_y S(ybar_m, y_j)
  M2M        W_parent = sum_o S_o W_child_o, S_o[m, m'] = S(ybar_m, child
             node m' in the parent's coordinates): exact, since S(ybar_m, .)
             is a polynomial the child's nodes interpolate without error.
  M2L        for A in V(B): L_B += K(xbar_B, ybar_A) W_A with K = 1/(4 pi r);
             optionally through SVD-compressed translations (below).
  P2L        for A in X(B): A's sources evaluated at B's nodes (or directly
             at B's targets when B holds <= n^3 targets).
  L2L        L_child_o += S_o^T L_parent (the same matrices, transposed).
  L2P        f(x) = sum_l S(xbar_l, x) L_l; the field is -grad f.
  M2P        for A in W(B): sum_m K(x, ybar_m) W_m (or A's sources directly
             when A holds <= n^3 sources).
  P2P        for A in U(B): the direct sum, with the singular exclusion.

M2L matrices are built between unit boxes (half-width 1, centres 2d apart
for direction d) and divided by the half-width h of the level, which is
exact for the homogeneous kernel. Compression: with Kfat = [K_1 ... K_316]
and Kthin = [K_1; ...; K_316], U_k and V_k are their leading left and right
singular vectors (k = the larger of the two counts of singular values above
eps * sigma_max), and K_d is applied as U_k (U_k^T K_d V_k) V_k^T. The paper
does not state the compression; this unweighted form is a reading.

Pins (tests/test_oracle_chebyshev.py): the nodes are the zeros of T_n
(numpy's Chebyshev series); S_n equals the textbook Lagrange product
formula and its derivative; interpolation reproduces polynomials of degree
n - 1 and their derivatives; M2M and L2L are exact (P2M of a parent equals
M2M of its child's P2M); compression at eps = 0 reproduces the dense
translations; the full FMM error against the direct sum decreases with n, for
the single layer, the double layer through the method-2 P2M and the field.
Parity unpinned: the exact truncation error at a given n (no closed form).
"""

from __future__ import annotations

import numpy as np

from . import tree as T
from .direct import direct_sum_numpy
from .kifmm import _octant, octant_sign, slp, slp_grad


def nodes_1d(n):
    """Chebyshev nodes of the first kind, cos((2i - 1) pi / (2n)), i = 1..n."""
    i = np.arange(1, n + 1)
    return np.cos((2 * i - 1) * np.pi / (2 * n))


def cheb_t(n, t):
    """T_k(t), k = 0..n-1, by the three-term recurrence; shape [n, len(t)]."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros((n, t.size))
    out[0] = 1.0
    if n > 1:
        out[1] = t
    for k in range(2, n):
        out[k] = 2.0 * t * out[k - 1] - out[k - 2]
    return out


def cheb_dt(n, t):
    """T_k'(t) = k U_{k-1}(t), k = 0..n-1; shape [n, len(t)]."""
    t = np.asarray(t, dtype=np.float64)
    u = np.zeros((max(n - 1, 1), t.size))  # U_0 .. U_{n-2}
    u[0] = 1.0
    if n > 2:
        u[1] = 2.0 * t
    for k in range(2, n - 1):
        u[k] = 2.0 * t * u[k - 1] - u[k - 2]
    out = np.zeros((n, t.size))
    for k in range(1, n):
        out[k] = k * u[k - 1]
    return out


def interp_1d(n, t, deriv=False):
    """S_n(xbar_i, t) (or d/dt) for every node i; shape [n, len(t)]."""
    tn = cheb_t(n, nodes_1d(n))                       # T_k(xbar_i), [k, i]
    tt = cheb_dt(n, t) if deriv else cheb_t(n, t)     # T_k(t) or T_k'(t), [k, point]
    s = (2.0 / n) * (tn[1:].T @ tt[1:])
    if not deriv:
        s += 1.0 / n
    return s


def nodes_3d(n):
    x = nodes_1d(n)
    return np.array([(x[i], x[j], x[k]) for i in range(n) for j in range(n) for k in range(n)])


def interp_3d(n, t):
    """S(xbar_m, t_p) for 3D nodes m and points t (reference coordinates); [n^3, P]."""
    t = np.atleast_2d(t)
    sx, sy, sz = (interp_1d(n, t[:, c]) for c in range(3))
    return np.einsum("ip,jp,kp->ijkp", sx, sy, sz).reshape(n ** 3, -1)


def interp_3d_grad(n, t):
    """d/dt_c S(xbar_m, t_p), c = x, y, z; [3, n^3, P]."""
    t = np.atleast_2d(t)
    s = [interp_1d(n, t[:, c]) for c in range(3)]
    d = [interp_1d(n, t[:, c], deriv=True) for c in range(3)]
    gx = np.einsum("ip,jp,kp->ijkp", d[0], s[1], s[2])
    gy = np.einsum("ip,jp,kp->ijkp", s[0], d[1], s[2])
    gz = np.einsum("ip,jp,kp->ijkp", s[0], s[1], d[2])
    return np.stack([g.reshape(n ** 3, -1) for g in (gx, gy, gz)])


class ChebOperators:
    """Unit-box nodes, M2M/L2L interpolation matrices and M2L translations."""

    def __init__(self, n, eps=0.0, rank=None):
        """eps > 0: compressed translations truncated at eps * sigma_max;
        rank: compressed, keeping exactly that many singular vectors."""
        self.n = n
        self.eps = eps
        self.X = nodes_3d(n)
        self.nn = len(self.X)
        # parent (origin, half-width 1) <- child o (centre s_o / 2, half-width 1/2)
        self.m2m = [interp_3d(n, 0.5 * octant_sign(o) + 0.5 * self.X) for o in range(8)]
        self.dirs = T.directions()
        self._dense = {}
        self.rank = self.nn
        self.U = self.V = None
        if eps > 0 or rank is not None:
            ks = [self.dense(k) for k in range(len(self.dirs))]
            uf, sf, _ = np.linalg.svd(np.hstack(ks), full_matrices=False)
            _, st, vt = np.linalg.svd(np.vstack(ks), full_matrices=False)
            self.sigma = sf
            r = max(int(np.sum(sf > eps * sf[0])), int(np.sum(st > eps * st[0]))) if rank is None else rank
            self.rank = r
            self.U = uf[:, :r]
            self.V = vt[:r].T

    def dense(self, k):
        """K(xbar, 2 d_k + ybar) between unit boxes, [n^3 targets, n^3 sources]."""
        m = self._dense.get(k)
        if m is None:
            d = self.dirs[k].astype(np.float64)
            m = slp(self.X, 2.0 * d + self.X)
            self._dense[k] = m
        return m

    def translate(self, k, w):
        """Apply direction k's translation (unit boxes) to columns w [n^3, ...]."""
        if self.U is None:
            return self.dense(k) @ w
        c = self.U.T @ self.dense(k) @ self.V
        return self.U @ (c @ (self.V.T @ w))


def cheb_apply(t, lists, ops, src_xyz, q=None, mu=None, normals=None, trg_xyz=None,
               delta=1e-5, field=False, direct_rule=True, return_stages=False):
    """Float64 Chebyshev FMM of pot_i = sum_j q_j G + mu_j dG/dn_j (and the SL field).

    Same calling convention as `oracle.kifmm.kifmm_apply`: a tree from
    `oracle.tree.build_tree` over the same points and its `all_lists`;
    inputs and outputs in the caller's order.
    """
    if field and mu is not None:
        raise ValueError("field output is defined for the single layer only")
    n, nn, X = ops.n, ops.nn, ops.X
    nb = len(t.level)
    src = np.asarray(src_xyz, dtype=np.float64)
    ys = src[t.src_perm]
    qs = None if q is None else np.asarray(q, dtype=np.float64)[t.src_perm]
    ms = None
    if mu is not None:
        ms = (np.asarray(mu, dtype=np.float64)[:, None] * np.asarray(normals, dtype=np.float64))[t.src_perm]
    trg = src if trg_xyz is None else np.asarray(trg_xyz, dtype=np.float64)
    xt = trg[t.trg_perm]
    nsrc = t.send - t.sbeg
    ntrg = t.tend - t.tbeg
    W = np.zeros((nb, nn))
    L = np.zeros((nb, nn))
    pot = np.zeros(len(xt))
    fld = np.zeros((len(xt), 3))

    def src_of(a):
        s0, s1 = t.sbeg[a], t.send[a]
        return ys[s0:s1], None if qs is None else qs[s0:s1], None if ms is None else ms[s0:s1]

    def points_at(x, a, dl):
        y, qq, mm = src_of(a)
        return direct_sum_numpy(x, y, qq, mm, dl)

    def add_targets(b, p, f):
        t0, t1 = t.tbeg[b], t.tend[b]
        pot[t0:t1] += p
        if field:
            fld[t0:t1] += f

    # P2M (leaves): interpolation at the sources, the double layer through
    # the gradient of the interpolating polynomial (d/dy = (1/h) d/dt)
    for b in np.flatnonzero(t.leaf & (t.level >= 2) & (nsrc > 0)):
        y, qq, mm = src_of(b)
        tref = (y - t.centre[b]) / t.half[b]
        if qq is not None:
            W[b] += interp_3d(n, tref) @ qq
        if mm is not None:
            g = interp_3d_grad(n, tref)
            W[b] += sum(g[c] @ mm[:, c] for c in range(3)) / t.half[b]
    # M2M (levels L-1 .. 2)
    for lv in range(t.nlevels - 2, 1, -1):
        for b in np.flatnonzero((t.level == lv) & ~t.leaf & (nsrc > 0)):
            for o in range(8):
                c = t.children[b, o]
                if c >= 0 and nsrc[c] > 0:
                    W[b] += ops.m2m[o] @ W[c]

    # M2L, grouped by (level, direction)
    tb, sa = [], []
    for b in range(nb):
        if t.level[b] >= 2 and ntrg[b] > 0:
            v = lists["V"][b]
            v = v[nsrc[v] > 0]
            tb.append(np.full(len(v), b))
            sa.append(v)
    if tb:
        tb = np.concatenate(tb).astype(np.int64)
        sa = np.concatenate(sa).astype(np.int64)
        dk = T.direction_index(t.anchor[sa] - t.anchor[tb])
        assert np.all(dk >= 0)
        for lv in range(2, t.nlevels):
            sel_l = t.level[tb] == lv
            if not sel_l.any():
                continue
            h = t.w / 2.0 ** (lv + 1)
            for k in np.unique(dk[sel_l]):
                sel = sel_l & (dk == k)
                contrib = ops.translate(int(k), W[sa[sel]].T).T / h
                np.add.at(L, tb[sel], contrib)
    m2l_only = L.copy()

    # P2L (X list), or direct evaluation at a small target box
    for b in range(nb):
        if ntrg[b] == 0:
            continue
        for a in lists["X"][b]:
            if nsrc[a] == 0:
                continue
            if direct_rule and ntrg[b] <= nn:
                add_targets(b, *points_at(xt[t.tbeg[b]:t.tend[b]], a, delta))
            else:
                u, _ = points_at(t.centre[b] + t.half[b] * X, a, 0.0)
                L[b] += u

    # L2L (levels 3 .. L), parents before children
    for lv in range(3, t.nlevels):
        for b in np.flatnonzero((t.level == lv) & (ntrg > 0)):
            pb = t.parent[b]
            L[b] += ops.m2m[_octant(t.anchor[b])].T @ L[pb]

    # L2P, M2P (W list), P2P (U list)
    for b in np.flatnonzero(t.leaf & (ntrg > 0)):
        x = xt[t.tbeg[b]:t.tend[b]]
        if t.level[b] >= 2:
            tref = (x - t.centre[b]) / t.half[b]
            p = interp_3d(n, tref).T @ L[b]
            f = -np.einsum("cmp,m->pc", interp_3d_grad(n, tref), L[b]) / t.half[b] if field else None
            add_targets(b, p, f)
        for a in lists["W"][b]:
            if nsrc[a] == 0:
                continue
            if direct_rule and nsrc[a] <= nn:
                add_targets(b, *points_at(x, a, delta))
            else:
                y = t.centre[a] + t.half[a] * X
                p = slp(x, y) @ W[a]
                f = np.einsum("cij,j->ic", slp_grad(x, y), W[a]) if field else None
                add_targets(b, p, f)
        u = lists["U"][b]
        u = u[nsrc[u] > 0]
        if len(u):
            idx = np.concatenate([np.arange(t.sbeg[a], t.send[a]) for a in u])
            p, f = direct_sum_numpy(x, ys[idx], None if qs is None else qs[idx],
                                    None if ms is None else ms[idx], delta)
            add_targets(b, p, f)

    out_pot = np.zeros(len(xt))
    out_pot[t.trg_perm] = pot
    out_fld = None
    if field:
        out_fld = np.zeros((len(xt), 3))
        out_fld[t.trg_perm] = fld
    if return_stages:
        return out_pot, out_fld, {"W": W, "L": L, "L_m2l": m2l_only}
    return out_pot, out_fld
