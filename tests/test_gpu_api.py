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
