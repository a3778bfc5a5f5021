"""Graph replay of the apply (fmm_set_graph): every replay must equal the
ordinary apply bit for bit, with eager work and synchronisations between
replays, after in-place changes of the densities, and after a change of
output pointer (which records a new graph)."""

import numpy as np
import pytest

import workloads as W

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def _plan(x, nrm, F, prec=0, basis=0):
    opts = F.fmm_default_options(order=6, leaf_size=48, precision=prec, basis=basis,
                                 src_kernels=F.FMM_SRC_SINGLE | F.FMM_SRC_DOUBLE, outputs=F.FMM_OUT_POT)
    return F.fmm_setup(x, nrm, options=opts)


@pytest.mark.parametrize("prec,basis", [(0, 0), (1, 0), (1, 1)])
def test_graph_replays_equal_eager(prec, basis):
    import torch

    import paper_1605_01715_amd as F

    d = W.clustered(30000, seed=7)
    say(f"test_graph_replays_equal_eager: n=30000 precision={prec} basis={basis}")
    x, nrm = dev(d["xyz"]), dev(d["normals"])
    q, mu = dev(d["q"]), dev(d["mu"])
    plan = _plan(x, nrm, F, prec, basis)
    ref = torch.empty(len(d["q"]), device="cuda:0")
    F.fmm_apply(plan, q=q, mu=mu, pot=ref)
    torch.cuda.synchronize()
    ref = ref.clone()

    F.fmm_set_graph(plan, True)
    pot = torch.empty_like(ref)
    for k in range(4):
        pot.fill_(np.nan)
        F.fmm_apply(plan, q=q, mu=mu, pot=pot)  # k = 0 records, then replays
        junk = (x * 2.0).sum()  # eager work and a synchronisation between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(pot, ref), f"replay {k} differs"
    # new density values in the same tensors: the replay reads them
    q2 = q * -0.5
    mu2 = mu * 2.0
    F.fmm_set_graph(plan, False)
    ref2 = torch.empty_like(ref)
    F.fmm_apply(plan, q=q2, mu=mu2, pot=ref2)
    torch.cuda.synchronize()
    F.fmm_set_graph(plan, True)
    F.fmm_apply(plan, q=q, mu=mu, pot=pot)
    q.copy_(q2)
    mu.copy_(mu2)
    F.fmm_apply(plan, q=q, mu=mu, pot=pot)
    torch.cuda.synchronize()
    assert torch.equal(pot, ref2)
    # another output pointer records a new graph
    pot3 = torch.full_like(ref, np.nan)
    F.fmm_apply(plan, q=q, mu=mu, pot=pot3)
    torch.cuda.synchronize()
    assert torch.equal(pot3, ref2)
    # stage timing runs the ordinary apply; turning it off resumes replay
    F.fmm_set_timing(plan, True)
    F.fmm_apply(plan, q=q, mu=mu, pot=pot3)
    F.fmm_apply(plan, q=q, mu=mu, pot=pot3)
    torch.cuda.synchronize()
    st = F.fmm_stage_times(plan)
    say(f"  stage times: {st}")
    assert all(v >= 0.0 for v in st.values()) and sum(st.values()) > 0.0
    assert torch.equal(pot3, ref2)
    F.fmm_set_timing(plan, False)
    pot3.fill_(np.nan)
    F.fmm_apply(plan, q=q, mu=mu, pot=pot3)
    torch.cuda.synchronize()
    assert torch.equal(pot3, ref2)
    F.fmm_destroy(plan)


def test_gmres_with_graph_replay_matches():
    import torch

    import paper_1605_01715_amd as F

    d = W.spheres_8(freq=6)
    xyz, nrm, w, g = d["xyz"], d["normals"], d["weights"], d["g"]
    n = len(w)
    say(f"test_gmres_with_graph_replay_matches: n={n}")
    opts = F.fmm_default_options(order=6, leaf_size=48, src_kernels=F.FMM_SRC_DOUBLE, outputs=F.FMM_OUT_POT)
    plan = F.fmm_setup(dev(xyz), dev(nrm), options=opts)
    a, wd, bd = dev(np.full(n, -0.5, np.float32)), dev(w), dev(g)
    x1 = dev(np.zeros(n))
    r1 = F.gmres_solve(plan, F.FMM_OP_FK, a, None, wd, bd, x1, rtol=1e-7)
    F.fmm_set_graph(plan, True)
    x2 = dev(np.zeros(n))
    r2 = F.gmres_solve(plan, F.FMM_OP_FK, a, None, wd, bd, x2, rtol=1e-7)
    torch.cuda.synchronize()
    say(f"  eager {r1}, graph {r2}")
    assert r1[0] == F.FMM_OK and r2[0] == F.FMM_OK and r1[1] == r2[1]
    assert torch.equal(x1, x2)
    # short restarts: the recorded matvec is replayed across restarts (the
    # restart's residual and every Arnoldi step), with eager work and
    # synchronisations between solves; every solve must equal the ordinary one
    # bit for bit
    F.fmm_set_graph(plan, False)
    x3 = dev(np.zeros(n))
    r3 = F.gmres_solve(plan, F.FMM_OP_FK, a, None, wd, bd, x3, rtol=1e-7, restart=4)
    F.fmm_set_graph(plan, True)
    for k in range(2):
        x4 = dev(np.zeros(n))
        r4 = F.gmres_solve(plan, F.FMM_OP_FK, a, None, wd, bd, x4, rtol=1e-7, restart=4)
        junk = (x4 * 2.0).sum()
        torch.cuda.synchronize()
        say(f"  restart 4: eager {r3}, graph {r4}")
        assert torch.isfinite(junk)
        assert r4[0] == r3[0] and r4[1] == r3[1] and r4[1] > 4
        assert torch.equal(x3, x4), f"solve {k} differs"
    # stage timing on (its events are created by the solve's first apply): the
    # ordinary path, same result
    F.fmm_set_timing(plan, True)
    x5 = dev(np.zeros(n))
    r5 = F.gmres_solve(plan, F.FMM_OP_FK, a, None, wd, bd, x5, rtol=1e-7, restart=4)
    F.fmm_set_timing(plan, False)
    torch.cuda.synchronize()
    assert r5[1] == r3[1] and torch.equal(x3, x5)
    F.fmm_destroy(plan)


def test_gmres_dielectric_with_graph_replay_matches():
    """Graph-replayed matvecs with the dielectric operator (field output,
    single layer) and short restarts: the same iterates as the ordinary solve."""
    import torch

    import paper_1605_01715_amd as F

    d = W.dielectric(12, 4)
    n = len(d["areas"])
    say(f"test_gmres_dielectric_with_graph_replay_matches: n={n}")
    opts = F.fmm_default_options(order=6, leaf_size=48, src_kernels=F.FMM_SRC_SINGLE, outputs=F.FMM_OUT_FIELD)
    nrm = dev(d["normals"])
    plan = F.fmm_setup(dev(d["xyz"]), nrm, None, nrm, options=opts)
    eps_i = np.asarray(d["eps_i"], np.float64)
    lam = (eps_i - 1.0) / (eps_i + 1.0)
    a = dev(np.ones(n, np.float32))
    c = dev((-2.0 * lam).astype(np.float32))
    w = dev(d["areas"])
    b = dev((2.0 * lam * d["normals"][:, 2]).astype(np.float64))
    x1 = dev(np.zeros(n))
    r1 = F.gmres_solve(plan, F.FMM_OP_DIELECTRIC, a, c, w, b, x1, rtol=1e-7, restart=4)
    F.fmm_set_graph(plan, True)
    x2 = dev(np.zeros(n))
    r2 = F.gmres_solve(plan, F.FMM_OP_DIELECTRIC, a, c, w, b, x2, rtol=1e-7, restart=4)
    torch.cuda.synchronize()
    say(f"  eager {r1}, graph {r2}")
    assert r1[0] == F.FMM_OK and r2[0] == F.FMM_OK and r1[1] == r2[1] and r1[1] > 4
    assert torch.equal(x1, x2)
    F.fmm_destroy(plan)
