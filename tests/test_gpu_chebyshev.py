"""Parity of the HIP Chebyshev path (the paper's interpolation form,
Sec. III.A.1 Eq. p2m) with the float64 oracle, through the C ABI.

Against the oracle's Chebyshev FMM on the same tree, with M2L compressed to
the same rank, the bound is the float32 floor (no ill-conditioned step in
this form: P2M, M2M, L2L and L2P are interpolations with bounded weights).
Against the direct sum the bound is the oracle's own interpolation error at
that order plus the same floor.
"""

import numpy as np
import pytest

import workloads as W
from oracle import chebyshev as C
from oracle import direct as D
from oracle import tree as T

from gpu_common import fmm_run, say

pytestmark = pytest.mark.gpu

CHEB = 1


def _cloud(n, seed, frac_blob=0.6, sigma=0.03):
    rng = np.random.default_rng(seed)
    nb = int(n * frac_blob)
    x = np.concatenate([rng.random((n - nb, 3)), np.clip(0.55 + sigma * rng.standard_normal((nb, 3)), 0, 0.999)])
    x = x[rng.permutation(n)]
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return x.astype(np.float32), nrm.astype(np.float32), rng.standard_normal(n).astype(np.float32), \
        rng.standard_normal(n).astype(np.float32)


@pytest.mark.parametrize("precision", [0, 1])
def test_chebyshev_matches_oracle_and_its_stages(precision):
    """Same tree and lists, M2L compressed to the GPU's rank: potentials, the
    multipole weights W and the local node values L against the oracle."""
    import paper_1605_01715_amd as F

    say(f"test_chebyshev_matches_oracle_and_its_stages: n=6000 s=30 order 5 precision {precision}")
    x, nrm, q, mu = _cloud(6000, 6)
    r = fmm_run(x, q=q, mu=mu, nrm=nrm, order=5, leaf=30, pinv_eps=1e-6, basis=CHEB, precision=precision,
                keep_plan=True)
    info = F.fmm_plan_info(r["plan"])
    assert info["basis"] == CHEB and info["n_surface"] == 125
    t = T.build_tree(x, leaf_size=30)
    L = T.all_lists(t)
    ops = C.ChebOperators(5, rank=info["rank"])
    # the GPU's rank comes from the same threshold on the same singular values,
    # the count rounded up to the 32 the M2L kernel pads it to anyway
    kept = int(np.sum(ops.sigma > 1e-6 * ops.sigma[0]))
    assert info["rank"] == min((kept + 31) // 32 * 32, 125)
    pot, _, st = C.cheb_apply(t, L, ops, x, q=q, mu=mu, normals=nrm, return_stages=True)
    err = D.rel_l2(r["pot"][0], pot)
    say(f"  GPU vs oracle Chebyshev FMM rel L2 = {err:.3e} (rank {info['rank']})")
    assert err < 2e-6
    w = F.fmm_export_stage(r["plan"], 0)
    l = F.fmm_export_stage(r["plan"], 1)
    F.fmm_destroy(r["plan"])
    has_src = (t.send - t.sbeg) > 0
    sel = (t.level >= 2) & has_src
    e_w = D.rel_l2(w[sel], st["W"][sel])
    sel_d = (t.level >= 2) & ((t.tend - t.tbeg) > 0)
    e_l = D.rel_l2(l[sel_d], st["L"][sel_d])
    say(f"  node weights W rel L2 = {e_w:.3e}, node values L = {e_l:.3e}")
    for lv in range(2, t.nlevels):
        s_l = sel_d & (t.level == lv)
        if s_l.any():
            say(f"    level {lv}: {int(s_l.sum())} boxes, L rel L2 = {D.rel_l2(l[s_l], st['L'][s_l]):.3e}")
    assert e_w < 1e-6
    # node values are more sensitive than the potentials interpolated from
    # them (float64 compression alone moves L 10x more than the potential);
    # the same bound as the surface form's downward state
    assert e_l < 1e-5


def test_chebyshev_field_with_separate_targets():
    say("test_chebyshev_field_with_separate_targets: 5000 sources, 3000 targets, order 6")
    x, _, q, _ = _cloud(5000, 8)
    trg = np.random.default_rng(11).random((3000, 3)).astype(np.float32)
    r = fmm_run(x, q=q, trg=trg, field=True, order=6, leaf=40, pinv_eps=1e-7, basis=CHEB)
    import paper_1605_01715_amd as F  # noqa: F401

    t = T.build_tree(x, trg=trg, leaf_size=40)
    ops = C.ChebOperators(6, rank=r["info"]["rank"])
    _, fld, _ = C.cheb_apply(t, T.all_lists(t), ops, x, q=q, trg_xyz=trg, field=True, return_stages=True)
    err = D.rel_l2(r["field"][0], fld)
    ref_p, ref_f = D.direct_sum(trg, x, q, None, field=True)
    e_dir = D.rel_l2(r["field"][0], ref_f)
    say(f"  field vs oracle Chebyshev {err:.3e}, vs direct sum {e_dir:.3e}")
    assert err < 5e-6
    assert e_dir < 1e-4


def test_chebyshev_converges_with_order():
    """Error against the float64 direct sum falls with the order, as the
    oracle's does, down to the float32 floor."""
    say("test_chebyshev_converges_with_order: n=20000 s=64")
    x, nrm, q, mu = _cloud(20000, 12)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(len(x), 1500, replace=False))
    ref, _ = D.direct_sum(x[sample], x, q, mu[:, None].astype(np.float64) * nrm)
    errs = []
    for n in (3, 5, 7):
        r = fmm_run(x, q=q, mu=mu, nrm=nrm, order=n, leaf=64, basis=CHEB)
        errs.append(D.rel_l2(r["pot"][0][sample], ref))
        say(f"  order {n}: rel L2 vs direct = {errs[-1]:.3e} (rank {r['info']['rank']})")
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1]
    assert errs[2] < 1e-5


def test_chebyshev_uniform_tree_and_three_right_hand_sides():
    say("test_chebyshev_uniform_tree_and_three_right_hand_sides: n=4096 depth 3 order 4")
    d = W.cube_uniform(4096, seed=3)
    x = d["xyz"]
    q3 = np.random.default_rng(5).standard_normal((3, len(x))).astype(np.float32)
    r3 = fmm_run(x, q=q3, nrhs=3, order=4, depth=3, root=d["root"], basis=CHEB, pinv_eps=1e-5)
    for k in range(3):
        r1 = fmm_run(x, q=q3[k], order=4, depth=3, root=d["root"], basis=CHEB, pinv_eps=1e-5)
        assert D.rel_l2(r3["pot"][k], r1["pot"][0]) < 1e-6
    t = T.build_tree(x, uniform_depth=3, root=d["root"])
    ops = C.ChebOperators(4, rank=r3["info"]["rank"])
    pot, _ = C.cheb_apply(t, T.all_lists(t), ops, x, q=q3[1])
    err = D.rel_l2(r3["pot"][1], pot)
    say(f"  rhs 1 vs oracle Chebyshev {err:.3e}")
    assert err < 2e-6


def test_chebyshev_m2l_pieces_and_pair_tiles_agree():
    """The M2L schedule (pieces per tile, pair tiles) does not change the
    result beyond float32 summation order."""
    say("test_chebyshev_m2l_pieces_and_pair_tiles_agree: n=30000 s=24 order 5")
    x, nrm, q, mu = _cloud(30000, 21, frac_blob=0.8, sigma=0.02)
    base = fmm_run(x, q=q, mu=mu, nrm=nrm, order=5, leaf=24, basis=CHEB, m2l_pieces=1)
    for k in (3, 8):
        r = fmm_run(x, q=q, mu=mu, nrm=nrm, order=5, leaf=24, basis=CHEB, m2l_pieces=k)
        assert D.rel_l2(r["pot"][0], base["pot"][0]) < 1e-6
    assert base["info"]["m2l_pair_tiles"] > 0


def test_chebyshev_edge_cases():
    say("test_chebyshev_edge_cases")
    r = fmm_run(np.array([[0.3, 0.4, 0.5]], np.float32), q=np.array([2.0], np.float32), basis=CHEB, order=5)
    assert r["pot"][0, 0] == 0.0
    for n in (2, 63, 65, 1001):
        xx, nrm, qq, mu = _cloud(n, n)
        r = fmm_run(xx, q=qq, mu=mu, nrm=nrm, leaf=9, order=6, basis=CHEB)
        ref, _ = D.direct_sum(xx, xx, qq, mu[:, None].astype(np.float64) * nrm)
        assert D.rel_l2(r["pot"][0], ref) < 1e-4, n
    for n in (2, 8):  # lowest and highest order
        xx, nrm, qq, mu = _cloud(3000, 40 + n)
        r = fmm_run(xx, q=qq, leaf=20, order=n, basis=CHEB)
        t = T.build_tree(xx, leaf_size=20)
        pot, _ = C.cheb_apply(t, T.all_lists(t), C.ChebOperators(n, rank=r["info"]["rank"]), xx, q=qq)
        err = D.rel_l2(r["pot"][0], pot)
        say(f"  order {n}: vs oracle Chebyshev {err:.3e}")
        assert err < 3e-6


def test_chebyshev_field_with_two_right_hand_sides():
    """Field output with two right-hand sides in one plan: each equals its
    single-rhs run, and the second matches the oracle's Chebyshev field."""
    say("test_chebyshev_field_with_two_right_hand_sides: n=8000 order 6, split-BF16")
    x, _, q, _ = _cloud(8000, 31)
    q2 = np.stack([q, np.random.default_rng(32).standard_normal(len(q)).astype(np.float32)])
    r2 = fmm_run(x, q=q2, nrhs=2, field=True, order=6, leaf=40, basis=CHEB, precision=1, pinv_eps=1e-7)
    for k in range(2):
        r1 = fmm_run(x, q=q2[k], field=True, order=6, leaf=40, basis=CHEB, precision=1, pinv_eps=1e-7)
        assert D.rel_l2(r2["field"][k], r1["field"][0]) < 1e-6
    t = T.build_tree(x, leaf_size=40)
    ops = C.ChebOperators(6, rank=r2["info"]["rank"])
    _, fld = C.cheb_apply(t, T.all_lists(t), ops, x, q=q2[1], field=True)
    err = D.rel_l2(r2["field"][1], fld)
    say(f"  rhs 1 field vs oracle Chebyshev {err:.3e}")
    assert err < 5e-6
