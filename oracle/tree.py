"""Morton keys, octree and U/V/W/X interaction lists, from their plain definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper inserts targets and sources into an octree (Sec. III.A.1, target
source model) whose height sets the near/far balance, and maps points to a
1-D array by their z-value (Morton order, Sec. III.B). It does not define the
tree or the lists further; the readings used here are:

  Root cube     given, or the float64 bounding box of the (float32) points,
                width w = max extent * (1 + 2^-20), centred on the box; w = 1
                when every point coincides.
  Quantisation  q = floor((double(x) - x0) * (2^21 / w)) clamped to
                [0, 2^21 - 1] per axis: two float64 operations, no FMA.
  Key           63-bit interleave, bit b of (qx, qy, qz) at bit (3b+2, 3b+1, 3b).
  Order         stable sort by key, ties by original index. With separate
                targets the combined index is [targets..., sources...].
  Boxes         level 0 is the root. Uniform mode: every box above the given
                depth is split. Adaptive mode: a box is split while it holds
                more than s points (targets + sources) and its level is below
                max_depth. Empty boxes do not exist; no 2:1 balance. Boxes are
                numbered level by level, in Morton order within a level.
  Adjacent      the closed cubes touch (checked on integer finest-level
                coordinates); a box is adjacent to itself and its ancestors.
  Lists         (textbook KIFMM definitions)
                U(B), leaf B:    leaves adjacent to B, B included
                V(B), level>=2:  same-level boxes whose parent is adjacent to
                                 parent(B), that are not adjacent to B
                W(B), leaf B:    finer boxes D not adjacent to B whose parent is
                                 adjacent to B
                X(B):            leaves A with B in W(A)

Pins (tests/test_oracle_tree.py): brute-force per-point box assignment,
invariance of boxes under input permutation, the interaction-coverage
invariant (every ordered leaf pair counted exactly once over U, V, W, X), list
counts of a uniform depth-3 tree derived by hand, and symmetries of U and V.
"""

from __future__ import annotations

import numpy as np

MAXLEV = 21
NDIR = 316


def root_box(xyz, root=None):
    """Root cube (x0[3], w) in float64; see the module docstring."""
    if root is not None and float(root[3]) > 0.0:
        return np.array(root[:3], dtype=np.float64), float(root[3])
    p = np.asarray(xyz, dtype=np.float64)
    if len(p) == 0:
        return np.zeros(3), 1.0
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    ext = float((hi - lo).max())
    w = ext * (1.0 + 2.0 ** -20) if ext > 0.0 else 1.0
    centre = (lo + hi) * 0.5
    return centre - 0.5 * w, w


def quantise(xyz, x0, w):
    """Integer finest-level coordinates in [0, 2^21 - 1]."""
    scale = float(2 ** MAXLEV) / w
    p = np.asarray(xyz, dtype=np.float64)
    q = np.floor((p - x0) * scale)
    return np.clip(q, 0, 2 ** MAXLEV - 1).astype(np.int64)


def interleave(q):
    """63-bit Morton key from [n,3] integer coordinates."""
    q = np.asarray(q, dtype=np.uint64)
    key = np.zeros(len(q), dtype=np.uint64)
    for b in range(MAXLEV):
        bit = np.uint64(b)
        one = np.uint64(1)
        key |= ((q[:, 0] >> bit) & one) << np.uint64(3 * b + 2)
        key |= ((q[:, 1] >> bit) & one) << np.uint64(3 * b + 1)
        key |= ((q[:, 2] >> bit) & one) << np.uint64(3 * b)
    return key


def deinterleave(prefix, level):
    """Anchor (ix, iy, iz) of a level-`level` box from its 3*level-bit prefix."""
    prefix = np.asarray(prefix, dtype=np.uint64)
    a = np.zeros((len(prefix), 3), dtype=np.int64)
    for b in range(level):
        for ax in range(3):
            a[:, ax] |= (((prefix >> np.uint64(3 * b + 2 - ax)) & np.uint64(1)).astype(np.int64) << b)
    return a


class Tree:
    """Octree over targets and sources (plain arrays, box-indexed)."""


def build_tree(src, trg=None, leaf_size=64, uniform_depth=0, max_depth=MAXLEV, root=None):
    src = np.asarray(src, dtype=np.float32)
    tsm = trg is not None
    pts = np.concatenate([np.asarray(trg, dtype=np.float32), src]) if tsm else src
    n = len(pts)
    n_trg = len(trg) if tsm else n
    is_trg = np.zeros(n, dtype=bool)
    is_src = np.zeros(n, dtype=bool)
    if tsm:
        is_trg[:n_trg] = True
        is_src[n_trg:] = True
    else:
        is_trg[:] = True
        is_src[:] = True
    x0, w = root_box(pts, root)
    keys = interleave(quantise(pts, x0, w))
    order = np.argsort(keys, kind="stable")
    ks = keys[order]

    level, anchor, begin, end, parent = [], [], [], [], []
    if n:
        level.append(0)
        anchor.append((0, 0, 0))
        begin.append(0)
        end.append(n)
        parent.append(-1)
    cur = list(range(len(level)))
    lv = 0
    while cur:
        nxt = []
        for b in cur:
            cnt = end[b] - begin[b]
            if uniform_depth > 0:
                split = lv < uniform_depth
            else:
                split = cnt > leaf_size and lv < max_depth
            if not split:
                continue
            shift = np.uint64(3 * (MAXLEV - (lv + 1)))
            pre = ks[begin[b]:end[b]] >> shift
            starts = np.concatenate([[0], np.flatnonzero(np.diff(pre)) + 1, [cnt]])
            anc = deinterleave(pre[starts[:-1]], lv + 1)
            for k in range(len(starts) - 1):
                nxt.append(len(level))
                level.append(lv + 1)
                anchor.append(tuple(anc[k]))
                begin.append(begin[b] + int(starts[k]))
                end.append(begin[b] + int(starts[k + 1]))
                parent.append(b)
        cur = nxt
        lv += 1

    t = Tree()
    nb = len(level)
    t.n = n
    t.tsm = tsm
    t.n_trg = n_trg
    t.n_src = len(src)
    t.x0, t.w = x0, w
    t.keys = ks
    t.order = order
    t.level = np.array(level, dtype=np.int64)
    t.anchor = np.array(anchor, dtype=np.int64).reshape(nb, 3)
    t.begin = np.array(begin, dtype=np.int64)
    t.end = np.array(end, dtype=np.int64)
    t.parent = np.array(parent, dtype=np.int64)
    t.children = -np.ones((nb, 8), dtype=np.int64)
    for b in range(nb):
        p = t.parent[b]
        if p >= 0:
            o = (t.anchor[b, 0] & 1) << 2 | (t.anchor[b, 1] & 1) << 1 | (t.anchor[b, 2] & 1)
            t.children[p, o] = b
    t.leaf = np.all(t.children < 0, axis=1)
    t.nlevels = int(t.level.max()) + 1 if nb else 0
    ct = np.concatenate([[0], np.cumsum(is_trg[order])])
    cs = np.concatenate([[0], np.cumsum(is_src[order])])
    t.tbeg, t.tend = ct[t.begin], ct[t.end]
    t.sbeg, t.send = cs[t.begin], cs[t.end]
    # user index of the k-th sorted target / source
    t.trg_perm = order[is_trg[order]]
    t.src_perm = order[is_src[order]] - (n_trg if tsm else 0)
    size = np.int64(1) << (MAXLEV - t.level)
    t.lo = t.anchor * size[:, None]
    t.size = size
    t.half = w / (2.0 ** (t.level + 1))
    t.centre = x0 + (t.anchor + 0.5) * (w / (2.0 ** t.level))[:, None]
    return t


def adjacent(t, a, b):
    """Closed cubes of boxes a and b touch (vectorised over a or b)."""
    lo_a, lo_b = t.lo[a], t.lo[b]
    sa = np.asarray(t.size[a])[..., None]
    sb = np.asarray(t.size[b])[..., None]
    return np.all((lo_a <= lo_b + sb) & (lo_b <= lo_a + sa), axis=-1)


def lists_of_box(t, b):
    """(U, V, W, X) of box b as sorted int arrays, by brute force over all boxes."""
    nb = len(t.level)
    allb = np.arange(nb)
    adj_b = adjacent(t, allb, b)
    par = t.parent
    U = V = W = X = np.zeros(0, dtype=np.int64)
    if t.leaf[b]:
        U = allb[t.leaf & adj_b]
        finer = t.level > t.level[b]
        has_par = par >= 0
        adj_par = np.zeros(nb, dtype=bool)
        adj_par[has_par] = adjacent(t, par[has_par], b)
        W = allb[finer & ~adj_b & adj_par]
    if t.level[b] >= 2:
        same = (t.level == t.level[b]) & (par >= 0)
        cand = allb[same]
        adj_pp = adjacent(t, par[cand], par[b])
        V = cand[adj_pp & ~adj_b[cand]]
    if par[b] >= 0:
        coarser_leaf = t.leaf & (t.level < t.level[b])
        cand = allb[coarser_leaf]
        adj_pb = adjacent(t, cand, par[b])
        X = cand[adj_pb & ~adj_b[cand]]
    return U, V, W, X


def all_lists(t, boxes=None):
    """Dict of CSR-like python lists: {'U': [arr per box], ...} for `boxes` (default all)."""
    if boxes is None:
        boxes = range(len(t.level))
    out = {"U": {}, "V": {}, "W": {}, "X": {}}
    for b in boxes:
        U, V, W, X = lists_of_box(t, int(b))
        out["U"][int(b)] = U
        out["V"][int(b)] = V
        out["W"][int(b)] = W
        out["X"][int(b)] = X
    return out


def directions():
    """The 316 M2L directions d in {-3..3}^3 with max|d| >= 2, lexicographic (dx, dy, dz)."""
    d = [(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)
         if max(abs(i), abs(j), abs(k)) >= 2]
    return np.array(d, dtype=np.int64)


def direction_index(d):
    """Index of offset(s) d (source anchor minus target anchor) in `directions()`."""
    d = np.atleast_2d(np.asarray(d, dtype=np.int64))
    table = -np.ones(343, dtype=np.int64)
    dirs = directions()
    table[(dirs[:, 0] + 3) * 49 + (dirs[:, 1] + 3) * 7 + (dirs[:, 2] + 3)] = np.arange(NDIR)
    return table[(d[:, 0] + 3) * 49 + (d[:, 1] + 3) * 7 + (d[:, 2] + 3)]


def coverage(t, lists):
    """Count, for every ordered (target leaf, source leaf) pair, how often the
    U, V, W and X lists account for it. The KIFMM is exact in structure only
    if every entry is 1."""
    leaves = np.flatnonzero(t.leaf)
    pos = -np.ones(len(t.level), dtype=np.int64)
    pos[leaves] = np.arange(len(leaves))
    nl = len(leaves)
    cnt = np.zeros((nl, nl), dtype=np.int64)
    # leaves under each box
    under = [[] for _ in range(len(t.level))]
    for lf in leaves:
        b = lf
        while b >= 0:
            under[b].append(pos[lf])
            b = t.parent[b]
    under = [np.array(u, dtype=np.int64) for u in under]
    for b in range(len(t.level)):
        tb = under[b]
        for a in lists["U"][b]:
            cnt[pos[b], pos[a]] += 1
        for a in lists["V"][b]:
            cnt[np.ix_(tb, under[a])] += 1
        for a in lists["W"][b]:
            cnt[pos[b], under[a]] += 1
        for a in lists["X"][b]:
            cnt[tb, pos[a]] += 1
    return cnt
