"""fmm_dielectric_rhs_noalloc (the right-hand side for callers that cannot
allocate device memory) against fmm_dielectric_rhs, through the C ABI: two
calls in a row on two plans, the second smaller, each checked against the
allocating entry point and against the oracle's right-hand side (Eq. rhs with
Eq. Ef, Sec. II.C); and the point limit of the fixed scratch."""

import numpy as np
import pytest

import workloads as W
from oracle import operators as OP

from gpu_common import dev, errors, say

pytestmark = pytest.mark.gpu


def _spheres(n_spheres, freq, seed):
    d = W.dielectric(n_spheres=n_spheres, freq=freq, box=4.0 * n_spheres ** (1 / 3) + 4.0, seed=seed)
    n = len(d["xyz"])
    rng = np.random.default_rng(seed)
    sf = (rng.standard_normal(n) * 0.1).astype(np.float32)  # free charge per element
    return d, sf


def _plan(d):
    import paper_1605_01715_amd as F

    opts = F.fmm_default_options(order=8, leaf_size=64, src_kernels=F.FMM_SRC_SINGLE, outputs=F.FMM_OUT_FIELD)
    return F.fmm_setup(dev(d["xyz"]), dev(d["normals"]), None, dev(d["normals"]), options=opts)


@pytest.mark.parametrize("order_of_calls", ["large_then_small"])
def test_noalloc_rhs_matches_the_allocating_entry_point(order_of_calls):
    import torch

    import paper_1605_01715_amd as F

    cases = [_spheres(10, 8, 41), _spheres(3, 6, 42)]  # the second call has fewer points
    for k, (d, sf) in enumerate(cases):
        n = len(d["xyz"])
        say(f"test_noalloc_rhs_matches_the_allocating_entry_point: call {k}, n={n}")
        plan = _plan(d)
        args = (dev(sf), dev(d["areas"]), dev(d["curvature"]), dev(d["eps_i"]))
        e0 = np.array([0.0, 0.3, 1.0])
        ref = F.fmm_dielectric_rhs(plan, *args, d["eps_m"], e0=e0).cpu().numpy()
        b = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        F.fmm_dielectric_rhs_noalloc(plan, *args, d["eps_m"], b, e0=e0)
        torch.cuda.synchronize()
        got = b.cpu().numpy()
        F.fmm_destroy(plan)
        assert np.all(np.isfinite(got))
        # same kernels on the same plan: identical results
        assert np.array_equal(got, ref)
        x64, n64 = d["xyz"].astype(np.float64), d["normals"].astype(np.float64)
        orc = OP.dielectric_rhs_free(x64, n64, d["areas"], d["curvature"], sf, d["eps_i"], d["eps_m"], e0=e0)
        l2, worst = errors(got, orc)
        say(f"  identical to fmm_dielectric_rhs; against the oracle rel L2 {l2:.2e}, worst {worst:.2e}")
        assert l2 < 1e-5 and worst < 1e-3


def test_noalloc_rhs_rejects_more_points_than_its_scratch():
    import torch

    import paper_1605_01715_amd as F

    n = 2_000_001
    say(f"test_noalloc_rhs_rejects_more_points_than_its_scratch: n={n}")
    rng = np.random.default_rng(5)
    x = rng.random((n, 3)).astype(np.float32)
    nrm = np.tile(np.float32([[0.0, 0.0, 1.0]]), (n, 1))
    opts = F.fmm_default_options(order=4, leaf_size=256, src_kernels=F.FMM_SRC_SINGLE, outputs=F.FMM_OUT_FIELD)
    plan = F.fmm_setup(dev(x), dev(nrm), None, dev(nrm), options=opts)
    ones = dev(np.ones(n, np.float32))
    b = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(F.FmmError) as e:
        F.fmm_dielectric_rhs_noalloc(plan, ones, ones, ones, ones, 1.0, b)
    assert e.value.code == F.FMM_ERR_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(b.abs().max()) == 0.0  # nothing was written
    F.fmm_destroy(plan)
