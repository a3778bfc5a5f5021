"""Leaf-size autotuning (fmm_autotune) and its cache, through the C ABI: the
trial runs report every candidate and keep the fastest; a plan built with
leaf_size = 0 reads the choice back (single and batched plans) and gives the
same result as a plan built with that leaf size; a configuration without an
entry falls back to the default cap."""

import os

import numpy as np
import pytest

import workloads as W

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def test_autotune_chooses_the_fastest_and_plans_read_it_back(tmp_path, monkeypatch):
    import torch

    import paper_1605_01715_amd as F

    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("FMM_TUNE_CACHE", str(cache))
    d = W.clustered(60000, seed=9)
    x, nrm, q, mu = dev(d["xyz"]), dev(d["normals"]), dev(d["q"]), dev(d["mu"])
    say("test_autotune_chooses_the_fastest_and_plans_read_it_back: clustered n=60000, Chebyshev n=6")
    opts = F.fmm_default_options(order=6, leaf_size=0, basis=F.FMM_BASIS_CHEBYSHEV, precision=1,
                                 src_kernels=F.FMM_SRC_SINGLE | F.FMM_SRC_DOUBLE, root=d["root"])
    r = F.fmm_autotune(x, nrm, options=opts, leaf_sizes=(32, 64, 128), pieces=(0, 2), reps=2)
    say(f"  trials {[(t['leaf'], t['m2l_pieces'], round(t['ms'], 3)) for t in r['tried']]} -> leaf {r['leaf_size']}")
    assert len(r["tried"]) == 6
    best = min(r["tried"], key=lambda t: t["ms"])
    assert (r["leaf_size"], r["ms"]) == (best["leaf"], best["ms"])
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and f'"leaf_size": {r["leaf_size"]}' in lines[0]
    # a plan with leaf_size 0 reads the entry back and matches an explicit plan
    outs = []
    for leaf in (0, r["leaf_size"]):
        o = F.fmm_default_options(order=6, leaf_size=leaf, basis=F.FMM_BASIS_CHEBYSHEV, precision=1,
                                  src_kernels=F.FMM_SRC_SINGLE | F.FMM_SRC_DOUBLE, root=d["root"],
                                  m2l_pieces=r["m2l_pieces"])
        plan = F.fmm_setup(x, nrm, options=o)
        info = F.fmm_plan_info(plan)
        assert info["leaf_size"] == r["leaf_size"] and info["leaf_from_cache"] == (1 if leaf == 0 else 0)
        pot = torch.empty(len(d["q"]), device="cuda:0")
        F.fmm_apply(plan, q=q, mu=mu, pot=pot)
        torch.cuda.synchronize()
        outs.append(pot.cpu().numpy())
        F.fmm_destroy(plan)
    assert np.array_equal(outs[0], outs[1])
    # retuning the same configuration replaces its entry
    F.fmm_autotune(x, nrm, options=opts, leaf_sizes=(48,), reps=1)
    assert len(cache.read_text().strip().splitlines()) == 1 and '"leaf_size": 48' in cache.read_text()
    # another configuration (two right-hand sides) has no entry: the default cap
    o2 = F.fmm_default_options(order=6, leaf_size=0, basis=F.FMM_BASIS_CHEBYSHEV, nrhs=2, root=d["root"])
    plan = F.fmm_setup(x, options=o2)
    info = F.fmm_plan_info(plan)
    F.fmm_destroy(plan)
    assert info["leaf_from_cache"] == 0 and info["leaf_size"] == 128


def test_autotune_of_a_batch(tmp_path, monkeypatch):
    import paper_1605_01715_amd as F

    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("FMM_TUNE_CACHE", str(cache))
    insts = W.ferro_batch(n_inst=8, seed=12, nmin=1000, nmax=6000)
    so = np.concatenate([[0], np.cumsum([len(i["src"]) for i in insts])])
    to = np.concatenate([[0], np.cumsum([len(i["trg"]) for i in insts])])
    say(f"test_autotune_of_a_batch: 8 instances, {so[-1]} sources, {to[-1]} targets")
    src = dev(np.concatenate([i["src"] for i in insts]))
    nrm = dev(np.concatenate([i["normals"] for i in insts]))
    trg = dev(np.concatenate([i["trg"] for i in insts]))
    opts = F.fmm_default_options(order=6, leaf_size=0, src_kernels=F.FMM_SRC_DOUBLE, nrhs=3)
    r = F.fmm_autotune(src, nrm, trg_xyz=trg, options=opts, leaf_sizes=(32, 96), reps=2, src_off=so, trg_off=to)
    say(f"  trials {[(t['leaf'], round(t['ms'], 3)) for t in r['tried']]} -> leaf {r['leaf_size']}")
    plan = F.fmm_setup_batch(so, src, nrm, to, trg, options=opts)
    info = F.fmm_plan_info(plan)
    F.fmm_destroy(plan)
    assert info["leaf_from_cache"] == 1 and info["leaf_size"] == r["leaf_size"]
    # no cache written when asked not to
    F.fmm_autotune(src, nrm, trg_xyz=trg, options=opts, leaf_sizes=(64,), reps=1, src_off=so, trg_off=to,
                   cache_path=None)
    assert '"leaf_size": 64' not in cache.read_text()
