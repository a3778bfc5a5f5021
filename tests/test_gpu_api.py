"""Plan handles through the C ABI: a destroyed plan answers every later call
with FMM_ERR_STATE (the handle is kept as a tombstone, never freed or reused),
including a second fmm_destroy."""

import ctypes

import numpy as np
import pytest

import workloads as W

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def test_destroyed_plan_returns_state_error():
    import torch

    import paper_1605_01715_amd as F

    lib = F._lib.load()
    d = W.cube_uniform(1024, seed=0)
    say("test_destroyed_plan_returns_state_error: n=1024 p=4")
    x = dev(d["xyz"])
    nrm = dev(np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (1024, 1)))
    opts = F.fmm_default_options(order=4, leaf_size=64, src_kernels=F.FMM_SRC_DOUBLE, root=d["root"])
    plan = F.fmm_setup(x, nrm, options=opts)
    h = ctypes.c_void_p(plan.handle)
    mu = dev(d["q"])
    pot = torch.empty(1024, device="cuda:0")
    assert lib.fmm_apply(h, None, mu.data_ptr(), pot.data_ptr(), None, None) == F.FMM_OK
    torch.cuda.synchronize()
    F.fmm_destroy(plan)
    assert plan.handle is None
    # every entry point that takes the plan
    assert lib.fmm_apply(h, None, mu.data_ptr(), pot.data_ptr(), None, None) == F.FMM_ERR_STATE
    assert "destroyed" in F.fmm_last_error()
    info = F._lib.FmmInfo()
    assert lib.fmm_plan_info(h, ctypes.byref(info)) == F.FMM_ERR_STATE
    w = dev(np.ones(1024, np.float32))
    b = dev(np.ones(1024))
    xs = dev(np.zeros(1024))
    op = F._lib.FmmOperator(F.FMM_OP_FK, w.data_ptr(), None, w.data_ptr())
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    assert lib.gmres_solve(h, ctypes.byref(op), b.data_ptr(), xs.data_ptr(), 1e-6, 10, 10, ctypes.byref(it),
                           ctypes.byref(rr), None) == F.FMM_ERR_STATE
    assert lib.fmm_set_graph(h, 1) == F.FMM_ERR_STATE
    assert lib.fmm_set_timing(h, 1) == F.FMM_ERR_STATE
    times = (ctypes.c_double * 7)()
    assert lib.fmm_stage_times(h, times) == F.FMM_ERR_STATE
    assert lib.fmm_destroy(h) == F.FMM_ERR_STATE
    # a new plan gets a new handle and works
    plan2 = F.fmm_setup(x, nrm, options=opts)
    assert plan2.handle != h.value
    F.fmm_apply(plan2, mu=mu, pot=pot)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(pot.cpu().numpy()))
    F.fmm_destroy(plan2)


def test_setup_phase_times_add_up():
    """fmm_info.setup_phase_ms: every phase timed, none negative, their sum
    within the setup's wall time; a second plan of the same form finds its
    operators cached (phase 3 near zero), a batch merges nothing (phase 7)."""
    import paper_1605_01715_amd as F

    d = W.clustered(60_000, seed=21)
    opts = F.fmm_default_options(order=6, leaf_size=64, basis=F.FMM_BASIS_CHEBYSHEV)
    infos = []
    for _ in range(2):
        plan = F.fmm_setup(dev(d["xyz"]), options=opts)
        infos.append(F.fmm_plan_info(plan))
        F.fmm_destroy(plan)
    for info in infos:
        ph = info["setup_phase_ms"]
        say(f"  setup {info['setup_ms']:.1f} ms, phases {ph}")
        assert all(v >= 0.0 for v in ph.values())
        assert sum(ph.values()) <= info["setup_ms"] * 1.001 + 0.1
        assert ph["sort"] > 0 and ph["lists"] > 0 and ph["m2l_schedule"] > 0 and ph["worklists"] > 0
        assert ph["unused"] == 0.0
    assert infos[1]["setup_phase_ms"]["operators"] < 1.0


@pytest.mark.parametrize("basis", [0, 1])
def test_stage_times_are_means_over_timed_applies(basis):
    """fmm_stage_times reads the events of the timed applies made since the
    previous call (the applies do not wait for them): -1 before any timed
    apply, the means after, the same means again when nothing new was timed,
    and more timed applies than the plan keeps event sets for (16) are still
    all counted. Timed applies give the same potentials as untimed ones."""
    import torch

    import paper_1605_01715_amd as F

    d = W.clustered(40_000, seed=22)
    say(f"test_stage_times_are_means_over_timed_applies: n=40000 basis={basis}")
    opts = F.fmm_default_options(order=6, leaf_size=64, basis=basis,
                                 src_kernels=F.FMM_SRC_SINGLE | F.FMM_SRC_DOUBLE)
    x, q, mu = dev(d["xyz"]), dev(d["q"]), dev(d["mu"])
    plan = F.fmm_setup(x, dev(d["normals"]), options=opts)
    ref = torch.empty(len(d["q"]), device="cuda:0")
    F.fmm_apply(plan, q=q, mu=mu, pot=ref)
    st0 = F.fmm_stage_times(plan)
    assert all(v == -1.0 for v in st0.values())
    F.fmm_set_timing(plan, True)
    pot = torch.empty_like(ref)
    for _ in range(3):
        F.fmm_apply(plan, q=q, mu=mu, pot=pot)
    st1 = F.fmm_stage_times(plan)
    say(f"  3 timed applies: {st1}")
    assert all(v >= 0.0 for v in st1.values()) and st1["EVAL"] > 0.0 and st1["M2L"] > 0.0
    assert F.fmm_stage_times(plan) == st1
    for _ in range(20):
        F.fmm_apply(plan, q=q, mu=mu, pot=pot)
    st2 = F.fmm_stage_times(plan)
    say(f"  20 timed applies: {st2}")
    assert all(v >= 0.0 for v in st2.values())
    # the same work: the means agree to within the run-to-run spread
    assert 0.3 < st2["EVAL"] / st1["EVAL"] < 3.0
    torch.cuda.synchronize()
    assert torch.equal(pot, ref)
    F.fmm_set_timing(plan, False)
    F.fmm_destroy(plan)


def test_injected_allocation_failure_is_reported_and_recovered():
    """FMM_FAULT_INJECT=alloc:<k> makes the k-th device allocation fail: setup,
    apply and gmres_solve return FMM_ERR_NOMEM with a message, release what
    they had allocated, and work again once the variable is unset (the
    results equal those of a run without injection)."""
    import os

    import torch

    import paper_1605_01715_amd as F

    d = W.clustered(20_000, seed=23)
    say("test_injected_allocation_failure_is_reported_and_recovered: n=20000")
    x, q = dev(d["xyz"]), dev(d["q"])
    opts = F.fmm_default_options(order=6, leaf_size=64)
    plan = F.fmm_setup(x, options=opts)
    ref = torch.empty(len(d["q"]), device="cuda:0")
    F.fmm_apply(plan, q=q, pot=ref)
    plan_dl = F.fmm_setup(x, dev(d["normals"]),
                          options=F.fmm_default_options(order=6, leaf_size=64, src_kernels=F.FMM_SRC_DOUBLE))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    try:
        for k in (1, 3, 17):
            os.environ["FMM_FAULT_INJECT"] = f"alloc:{k}"
            with pytest.raises(F.FmmError) as e:
                F.fmm_setup(x, options=opts)
            say(f"  setup, allocation {k}: {e.value}")
            assert e.value.code == F.FMM_ERR_NOMEM and "FMM_FAULT_INJECT" in str(e.value)
        # a solve allocates its work vectors: the first of its allocations fails
        n = len(d["q"])
        os.environ["FMM_FAULT_INJECT"] = "alloc:1"
        a, w = dev(np.ones(n, np.float32)), dev(np.full(n, 1e-3, np.float32))
        b, xs = dev(np.ones(n)), dev(np.zeros(n))
        with pytest.raises(F.FmmError) as e:
            F.gmres_solve(plan_dl, F.FMM_OP_FK, a, None, w, b, xs, rtol=1e-6, max_iter=3)
        assert e.value.code == F.FMM_ERR_NOMEM
    finally:
        del os.environ["FMM_FAULT_INJECT"]
    rc = F.gmres_solve(plan_dl, F.FMM_OP_FK, a, None, w, b, xs, rtol=1e-6, max_iter=3)
    assert rc[0] in (F.FMM_OK, F.FMM_ERR_NOT_CONVERGED)
    F.fmm_destroy(plan_dl)
    torch.cuda.synchronize()
    # nothing leaked by the failed calls (the torch allocations above are small)
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
    plan2 = F.fmm_setup(x, options=opts)
    pot = torch.empty_like(ref)
    F.fmm_apply(plan2, q=q, pot=pot)
    F.fmm_apply(plan, q=q, pot=ref.clone())
    torch.cuda.synchronize()
    assert torch.equal(pot, ref)
    F.fmm_destroy(plan2)
    F.fmm_destroy(plan)


_OPS_SCRIPT = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, {root!r})
import workloads as W
import paper_1605_01715_amd as F
d = W.clustered(20000, seed=24)
x, q = torch.from_numpy(d["xyz"]).cuda(), torch.from_numpy(d["q"]).cuda()
for basis, order in ((0, 6), (1, 5)):
    plan = F.fmm_setup(x, options=F.fmm_default_options(order=order, leaf_size=64, basis=basis))
    pot = torch.empty(20000, device="cuda")
    F.fmm_apply(plan, q=q, pot=pot)
    np.save({out!r} + "_%d.npy" % basis, pot.cpu().numpy())
    F.fmm_destroy(plan)
"""


def test_operator_factors_cached_on_disk(tmp_path):
    """The float64 factorisations the operators are built from are written to
    FMM_OP_CACHE by the first process and read by the next (same potentials
    bit for bit); a damaged file is detected, ignored and rewritten."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ops = tmp_path / "ops"
    env = dict(os.environ, FMM_OP_CACHE=str(ops), FMM_LOG="1")

    def run(tag):
        out = str(tmp_path / tag)
        say(f"test_operator_factors_cached_on_disk: process {tag}")
        r = subprocess.run([sys.executable, "-c", _OPS_SCRIPT.format(root=root, out=out)], env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        lines = [l for l in r.stderr.splitlines() if "operators: factors" in l]
        say("  " + " | ".join(lines))
        return lines, [np.load(out + "_%d.npy" % b) for b in (0, 1)]

    first, pots1 = run("a")
    assert sum("written to" in l for l in first) == 2
    files = sorted(p.name for p in ops.iterdir())
    assert files == ["cheb_5.f64", "surface_6.f64"]
    second, pots2 = run("b")
    assert sum(l.endswith("read") for l in second) == 2 and not any("written" in l for l in second)
    for a, b in zip(pots1, pots2):
        assert np.array_equal(a, b)
    # flip one byte of the data: detected by the checksum, rebuilt and rewritten
    f = ops / "surface_6.f64"
    raw = bytearray(f.read_bytes())
    raw[-100] ^= 0x40
    f.write_bytes(bytes(raw))
    third, pots3 = run("c")
    assert any("do not match" in l for l in third) and any("written to" in l for l in third)
    for a, b in zip(pots1, pots3):
        assert np.array_equal(a, b)
