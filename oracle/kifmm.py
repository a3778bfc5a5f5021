"""Kernel-independent FMM in float64, step by step (equivalent-surface form).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper accelerates the quadrature sum of Sec. II.A (Eq. sum_fmm) with a
kernel-independent FMM (Sec. I, Sec. III.A): far-field interactions pass
through an upward approximation of each box's sources, a box-to-box
translation, and a downward approximation evaluated at the targets
(Eq. p2m: interpolate at the sources, translate with the plain 1/r kernel,
interpolate at the targets). The paper's variant interpolates on Chebyshev
nodes; this oracle follows the equivalent-surface variant, which builds the
same three steps from the kernel itself:

  surfaces   Y(p): the boundary nodes of the p^3 grid on [-1,1]^3, ordered
             lexicographically (i over x outermost). A box with centre c and
             half-width r has an upward equivalent surface c + 1.05 r Y, an
             upward check surface c + 2.95 r Y, a downward equivalent surface
             c + 2.95 r Y and a downward check surface c + 1.05 r Y.
  C2E        check-to-equivalent maps are truncated-SVD pseudo-inverses of the
             single-layer matrix between the two surfaces, dropping singular
             values below eps * sigma_max. The Laplace kernel is homogeneous
             of degree -1, so the map of a box of half-width r is r times the
             map of the unit box.
  P2M        check potential of a leaf's sources (single layer q and double
             layer mu d/dn_y, the paper's method-2 normal derivative at P2M),
             then the upward C2E map.
  M2M        children's upward equivalent densities evaluated on the parent's
             upward check surface, then the parent's upward C2E.
  M2L        for A in V(B): A's upward equivalent density evaluated on B's
             downward check surface.
  P2L        for A in X(B): A's sources evaluated on B's downward check
             surface (or directly at B's targets when B holds <= n_s targets).
  L2L        the parent's downward equivalent density evaluated on the child's
             downward check surface, added to the child's M2L/P2L check
             potential, then the child's downward C2E.
  L2P        a leaf's downward equivalent density evaluated at its targets.
  M2P        for A in W(B): A's upward equivalent density evaluated at B's
             targets (or A's sources directly when A holds <= n_s sources).
  P2P        for A in U(B): the direct sum, with the singular exclusion.

Translation matrices between surfaces (one per octant for M2M/L2L, one per
M2L direction) are built once on unit boxes and scaled by 1/r per level,
which is exact for the homogeneous kernel.

Pins (tests/test_oracle_kifmm.py): the pseudo-inverse satisfies
K K+ K = K; an upward equivalent density reproduces its sources' potential
at well-separated points; scaling of the C2E map with r matches a direct
pseudo-inverse at that r; the full FMM error against the direct sum decreases
with p and is below 1e-5 at p = 8 on uniform and clustered clouds; the double
layer through P2M agrees with the three-kernel split (Eq. sum_split).
Parity unpinned: the exact truncation error at a given p (no closed form).
"""

from __future__ import annotations

import numpy as np

from . import tree as T
from .direct import direct_sum_numpy

RAD_IN = 1.05
RAD_OUT = 2.95
FOUR_PI = 4.0 * np.pi


def surface(p):
    """Y(p): boundary nodes of the p^3 grid on [-1,1]^3, lexicographic (i,j,k)."""
    g = -1.0 + 2.0 * np.arange(p) / (p - 1)
    pts = [(g[i], g[j], g[k]) for i in range(p) for j in range(p) for k in range(p)
           if i in (0, p - 1) or j in (0, p - 1) or k in (0, p - 1)]
    return np.array(pts, dtype=np.float64)


def slp(x, y):
    """Single-layer matrix 1 / (4 pi |x_i - y_j|)."""
    d = x[:, None, :] - y[None, :, :]
    return 1.0 / (FOUR_PI * np.sqrt(np.einsum("ijk,ijk->ij", d, d)))


def slp_grad(x, y):
    """Field matrices (x_i - y_j) / (4 pi |x_i - y_j|^3), shape [3, nx, ny]."""
    d = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    inv3 = 1.0 / (FOUR_PI * r ** 3)
    return np.moveaxis(d * inv3[..., None], -1, 0)


def pinv(k, eps):
    """Truncated-SVD pseudo-inverse: singular values below eps*sigma_max dropped."""
    u, s, vt = np.linalg.svd(k)
    keep = s > eps * s[0]
    return (vt[keep].T * (1.0 / s[keep])) @ u[:, keep].T


def octant_sign(o):
    return np.array([2 * ((o >> 2) & 1) - 1, 2 * ((o >> 1) & 1) - 1, 2 * (o & 1) - 1], dtype=np.float64)


class Operators:
    """Unit-box surfaces, C2E maps and translation matrices for order p."""

    def __init__(self, p, eps=1e-12):
        self.p = p
        self.eps = eps
        self.Y = surface(p)
        self.ns = len(self.Y)
        Y = self.Y
        self.uc2e = pinv(slp(RAD_OUT * Y, RAD_IN * Y), eps)
        self.dc2e = pinv(slp(RAD_IN * Y, RAD_OUT * Y), eps)
        # parent (unit half-width, origin) <- child o (half-width 1/2)
        self.m2m_g = [slp(RAD_OUT * Y, 0.5 * octant_sign(o) + 0.5 * RAD_IN * Y) for o in range(8)]
        self.l2l_g = [slp(0.5 * octant_sign(o) + 0.5 * RAD_IN * Y, RAD_OUT * Y) for o in range(8)]
        self._m2l = {}
        self.dirs = T.directions()

    def m2l_g(self, k):
        """Downward check of a unit box <- upward equivalent of the box at offset 2*d_k."""
        m = self._m2l.get(k)
        if m is None:
            d = self.dirs[k].astype(np.float64)
            m = slp(RAD_IN * self.Y, 2.0 * d + RAD_IN * self.Y)
            self._m2l[k] = m
        return m


def _octant(anchor):
    return int((anchor[0] & 1) << 2 | (anchor[1] & 1) << 1 | (anchor[2] & 1))


def kifmm_apply(t, lists, ops, src_xyz, q=None, mu=None, normals=None, trg_xyz=None,
                delta=1e-5, field=False, direct_rule=True, return_stages=False):
    """Float64 KIFMM of pot_i = sum_j q_j G + mu_j dG/dn_j (and the SL field).

    `t` is a tree from `oracle.tree.build_tree` over the same points and
    `lists` its `all_lists`. Inputs are in the caller's order; outputs too.
    """
    if field and mu is not None:
        raise ValueError("field output is defined for the single layer only")
    ns = ops.ns
    Y = ops.Y
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
    phi_u = np.zeros((nb, ns))
    u_chk = np.zeros((nb, ns))
    d_chk = np.zeros((nb, ns))
    e_chk = np.zeros((nb, ns))
    phi_d = np.zeros((nb, ns))
    pot = np.zeros(len(xt))
    fld = np.zeros((len(xt), 3))

    def src_of(a):
        s0, s1 = t.sbeg[a], t.send[a]
        return ys[s0:s1], None if qs is None else qs[s0:s1], None if ms is None else ms[s0:s1]

    def points_at(x, a, dl):
        y, qq, mm = src_of(a)
        return direct_sum_numpy(x, y, qq, mm, dl)

    def surface_at(x, centre, radius, dens):
        y = centre + radius * Y
        p = slp(x, y) @ dens
        f = np.einsum("cij,j->ic", slp_grad(x, y), dens) if field else None
        return p, f

    def add_targets(b, p, f):
        t0, t1 = t.tbeg[b], t.tend[b]
        pot[t0:t1] += p
        if field:
            fld[t0:t1] += f

    # P2M (leaves) and M2M (levels L-1 .. 2)
    for b in np.flatnonzero(t.leaf & (t.level >= 2) & (nsrc > 0)):
        xu = t.centre[b] + RAD_OUT * t.half[b] * Y
        u, _ = points_at(xu, b, 0.0)
        u_chk[b] = u
        phi_u[b] = t.half[b] * (ops.uc2e @ u)
    for lv in range(t.nlevels - 2, 1, -1):
        for b in np.flatnonzero((t.level == lv) & ~t.leaf & (nsrc > 0)):
            u = np.zeros(ns)
            for o in range(8):
                c = t.children[b, o]
                if c >= 0 and nsrc[c] > 0:
                    u += ops.m2m_g[o] @ phi_u[c]
            u_chk[b] = u / t.half[b]
            phi_u[b] = t.half[b] * (ops.uc2e @ u_chk[b])

    # M2L: group the V pairs by (level, direction) and apply each matrix once
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
            r = t.w / 2.0 ** (lv + 1)
            for k in np.unique(dk[sel_l]):
                sel = sel_l & (dk == k)
                contrib = (ops.m2l_g(int(k)) @ phi_u[sa[sel]].T).T / r
                np.add.at(d_chk, tb[sel], contrib)

    # P2L (X list), or direct evaluation at a small target box
    for b in range(nb):
        if ntrg[b] == 0:
            continue
        for a in lists["X"][b]:
            if nsrc[a] == 0:
                continue
            if direct_rule and ntrg[b] <= ns:
                p, f = points_at(xt[t.tbeg[b]:t.tend[b]], a, delta)
                add_targets(b, p, f)
            else:
                xd = t.centre[b] + RAD_IN * t.half[b] * Y
                u, _ = points_at(xd, a, 0.0)
                d_chk[b] += u

    # L2L + downward C2E (levels 2 .. L)
    for lv in range(2, t.nlevels):
        for b in np.flatnonzero((t.level == lv) & (ntrg > 0)):
            d = d_chk[b].copy()
            if lv >= 3:
                pb = t.parent[b]
                d += ops.l2l_g[_octant(t.anchor[b])] @ phi_d[pb] / t.half[pb]
            e_chk[b] = d
            phi_d[b] = t.half[b] * (ops.dc2e @ d)

    # L2P, M2P (W list), P2P (U list)
    for b in np.flatnonzero(t.leaf & (ntrg > 0)):
        x = xt[t.tbeg[b]:t.tend[b]]
        if t.level[b] >= 2:
            add_targets(b, *surface_at(x, t.centre[b], RAD_OUT * t.half[b], phi_d[b]))
        for a in lists["W"][b]:
            if nsrc[a] == 0:
                continue
            if direct_rule and nsrc[a] <= ns:
                add_targets(b, *points_at(x, a, delta))
            else:
                add_targets(b, *surface_at(x, t.centre[a], RAD_IN * t.half[a], phi_u[a]))
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
        return out_pot, out_fld, {"phi_u": phi_u, "u_chk": u_chk, "d_chk": d_chk,
                                  "e_chk": e_chk, "phi_d": phi_d}
    return out_pot, out_fld
