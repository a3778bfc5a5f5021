"""The benchmark's configuration and the paper-shaped workloads at their full
sizes, through the C ABI, against the float64 oracle.

* The headline path (the paper's Chebyshev form, Sec. III.A.1 Eq. p2m, with 8
  nodes per axis, leaf 192, bf16x3 M2L, M2L basis threshold 1e-7 or 1e-8:
  the benchmark takes the faster of the two): at 20,000 points against the
  oracle's Chebyshev FMM compressed to the GPU's rank (every target), and on
  the 4M-point clustered cloud in the launch configuration the benchmark
  times (with the other arithmetics and the surface form beside it) against
  the direct sum on the benchmark's second set of 10,000 targets.
* Eight spheres, 196,000 quadrature points, double layer: one apply against
  the direct sum, then the interior Dirichlet problem (Eq. fk_integral with
  Omega = 2 pi) by matrix-free GMRES (Sec. III) to 1e-6, with the true
  residual of the exact operator at sampled rows.
* 1000 dielectric spheres, about 980,000 points, single-layer field: one
  apply of E.n against the direct sum, then Eq. Ax by GMRES to 1e-6, with the
  sampled true residual.
* 256 ferromagnet surfaces (cubes and ellipsoids), three right-hand sides,
  targets at the nodes and sources at the triangle centroids, one batched plan
  replayed as a HIP graph: against 256 separate plans and, on six sampled
  instances, against the direct sum.

Every comparison bounds both the relative L2 error and the worst target's
error relative to the rms output, the latter at 100 times the former (on
clustered clouds the potential near a blob centre is far above the rms, and
so is its rounding error; a wrong leaf or target group would show as an
error of order one).
"""

import numpy as np
import pytest

import workloads as W
from oracle import chebyshev as C
from oracle import direct as D
from oracle import operators as OP
from oracle import tree as T

from gpu_common import dev, errors, fmm_run, say

pytestmark = pytest.mark.gpu

CHEB = 1


@pytest.mark.parametrize("eps", [1e-7, 1e-8])
def test_headline_path_against_the_oracle_chebyshev_fmm(eps):
    """The benchmark's two finalists (Chebyshev, 8 nodes per axis, threshold
    1e-7 or 1e-8, leaf 192, bf16x3 M2L) at 20,000 points against the
    oracle's Chebyshev FMM compressed to the GPU's rank, every target."""
    d = W.clustered(20000, seed=31)
    x, nrm, q, mu = d["xyz"], d["normals"], d["q"], d["mu"]
    say(f"test_headline_path_against_the_oracle_chebyshev_fmm: clustered n=20000, Chebyshev n=8, leaf 192, "
        f"eps {eps:g}, bf16x3, 3 M2L pieces")
    r = fmm_run(x, q=q, mu=mu, nrm=nrm, order=8, leaf=192, root=d["root"], pinv_eps=eps, basis=CHEB, precision=2,
                m2l_pieces=3)
    info = r["info"]
    assert info["m2l_pieces"] == 3 and info["basis"] == CHEB
    t = T.build_tree(x, leaf_size=192, root=d["root"])
    ops = C.ChebOperators(8, rank=info["rank"])
    say(f"  GPU rank {info['rank']}; oracle operators built")
    pot, _, _ = C.cheb_apply(t, T.all_lists(t), ops, x, q=q, mu=mu, normals=nrm, return_stages=True)
    l2, worst = errors(r["pot"][0], pot)
    say(f"  GPU vs oracle Chebyshev FMM: rel L2 {l2:.2e}, worst target {worst:.2e}")
    assert l2 < 5e-7 and worst < 5e-5
    ref, _ = D.direct_sum(x, x, q, mu[:, None].astype(np.float64) * nrm)
    l2d, worstd = errors(r["pot"][0], ref)
    say(f"  GPU vs direct sum: rel L2 {l2d:.2e}, worst target {worstd:.2e}")
    assert l2d < 1e-6 and worstd < 1e-4


_FULL = {}


def _full_size_reference():
    """The 4M-point cloud and the float64 direct sum at the benchmark's second
    error set (10,000 targets drawn with seed 7), computed once."""
    if not _FULL:
        d = W.clustered(4_000_000)
        sample = np.sort(np.random.default_rng(7).choice(len(d["xyz"]), 10000, replace=False))
        ref, _ = D.direct_sum(d["xyz"][sample], d["xyz"], d["q"], d["mu"][:, None].astype(np.float64) * d["normals"])
        _FULL.update(d=d, sample=sample, ref=ref)
    return _FULL["d"], _FULL["sample"], _FULL["ref"]


@pytest.mark.parametrize("basis,precision,eps,bound", [(CHEB, 2, 1e-7, 1e-6), (CHEB, 2, 1e-8, 1e-6),
                                                       (CHEB, 1, 1e-8, 1e-6), (CHEB, 0, 1e-8, 1e-6),
                                                       (0, 2, 1e-7, 1e-6), (CHEB, 1, 1e-7, 1.5e-6)])
def test_headline_configuration_at_full_size(basis, precision, eps, bound):
    """The 4M-point clustered cloud as the benchmark runs it (order 8, leaf
    192, pieces chosen at setup) on the benchmark's seed-7 error set: its two
    finalists (Chebyshev, bf16x3, thresholds 1e-7 and 1e-8), the Chebyshev
    form at 1e-8 with bf16x6 and float32, the surface form, all below 1e-6.
    The Chebyshev form at 1e-7 is closest to the bound on this set (9.7e-7
    with bf16x3 in the benchmark; its error is dominated by the few targets
    near blob centres whose potential is up to 80 times the rms); with bf16x6
    it is held to 1.5e-6."""
    d, sample, ref = _full_size_reference()
    x, nrm, q, mu = d["xyz"], d["normals"], d["q"], d["mu"]
    say(f"test_headline_configuration_at_full_size: clustered n=4M, basis {basis}, order 8, leaf 192, "
        f"precision {precision}, eps {eps:g}")
    r = fmm_run(x, q=q, mu=mu, nrm=nrm, order=8, leaf=192, root=d["root"], pinv_eps=eps, basis=basis,
                precision=precision)
    l2, worst = errors(r["pot"][0][sample], ref)
    say(f"  {r['info']['n_boxes']} boxes, rank {r['info']['rank']}, {r['info']['m2l_pieces']} pieces: "
        f"rel L2 {l2:.2e}, worst target {worst:.2e}")
    assert l2 < bound and worst < 100 * bound


def _sampled_fk_residual(xyz, nrm, w, a, b, x, rows):
    """b - (a x + D[w x]) at the sampled rows, exact operator (float64 direct sum)."""
    x64, n64 = xyz.astype(np.float64), nrm.astype(np.float64)
    dens = x * w.astype(np.float64)
    dl, _ = D.direct_sum(x64[rows], x64, None, dens[:, None] * n64)
    return b[rows] - (a[rows] * x[rows] + dl)


def _sampled_dielectric_residual(xyz, nrm, a, c, w, b, s, rows):
    x64, n64 = xyz.astype(np.float64), nrm.astype(np.float64)
    _, fld = D.direct_sum(x64[rows], x64, s * w, None, potential=False, field=True)
    en = np.einsum("ij,ij->i", fld, n64[rows])
    return b[rows] - (a[rows] * s[rows] + c[rows] * en)


def test_eight_spheres_at_full_size():
    import torch

    import paper_1605_01715_amd as F

    d = W.spheres_8(freq=35)
    xyz, nrm, w, g, mu = d["xyz"], d["normals"], d["weights"], d["g"], d["mu"]
    n = len(w)
    say(f"test_eight_spheres_at_full_size: n={n}, double layer, surface order 8, leaf 128")
    rows = np.sort(np.random.default_rng(1).choice(n, 3000, replace=False))
    dens = (mu.astype(np.float64) * w).astype(np.float32)
    ref, _ = D.direct_sum(xyz[rows], xyz, None, dens[:, None].astype(np.float64) * nrm)
    for prec in (0, 1):
        r = fmm_run(xyz, mu=dens, nrm=nrm, order=8, leaf=128, precision=prec)
        l2, worst = errors(r["pot"][0][rows], ref)
        say(f"  one apply, precision {prec}: rel L2 {l2:.2e}, worst target {worst:.2e} "
            f"({r['info']['n_boxes']} boxes)")
        assert l2 < 1e-5 and worst < 1e-3
    # (D_pv - I/2) x = g, the FK operator with Omega = 2 pi at every centroid
    opts = F.fmm_default_options(order=8, leaf_size=128, src_kernels=F.FMM_SRC_DOUBLE, outputs=F.FMM_OUT_POT,
                                 precision=1)
    plan = F.fmm_setup(dev(xyz), dev(nrm), options=opts)
    a = np.full(n, -0.5)
    xd = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    rc, it, rr = F.gmres_solve(plan, F.FMM_OP_FK, dev(a.astype(np.float32)), None, dev(w), dev(g.astype(np.float64)),
                               xd, rtol=1e-6, restart=30, max_iter=200)
    torch.cuda.synchronize()
    F.fmm_destroy(plan)
    x = xd.cpu().numpy()
    say(f"  GMRES: rc={rc} iterations={it} relative residual {rr:.2e}")
    assert rc == F.FMM_OK and rr <= 1e-6 and it <= 40
    res = _sampled_fk_residual(xyz, nrm, w, a, g.astype(np.float64), x, rows)
    tr = np.linalg.norm(res) / np.linalg.norm(g[rows])
    say(f"  true residual of the exact operator at {len(rows)} rows: {tr:.2e}")
    assert tr < 2e-5


def test_dielectric_spheres_at_full_size():
    import torch

    import paper_1605_01715_amd as F

    d = W.dielectric(1000, 7)
    xyz, nrm = d["xyz"], d["normals"]
    n = len(xyz)
    say(f"test_dielectric_spheres_at_full_size: 1000 spheres, n={n}, single-layer field, surface order 8")
    a, c, w = OP.dielectric_coeffs(d["areas"], d["curvature"], d["eps_i"], d["eps_m"])
    b = OP.dielectric_rhs(nrm, d["eps_i"], d["eps_m"], d["e0"])
    rows = np.sort(np.random.default_rng(1).choice(n, 3000, replace=False))
    # one apply of E . n for the density b w (float32 path)
    s0 = (b * w).astype(np.float32)
    r = fmm_run(xyz, q=s0, field=True, order=8, leaf=128, precision=0)
    _, ref = D.direct_sum(xyz[rows], xyz, s0, None, potential=False, field=True)
    en_gpu = np.einsum("ij,ij->i", r["field"][0][rows], nrm[rows].astype(np.float64))
    en_ref = np.einsum("ij,ij->i", ref, nrm[rows].astype(np.float64))
    l2f, worstf = errors(r["field"][0][rows], ref)
    l2, worst = errors(en_gpu, en_ref)
    say(f"  one apply ({r['info']['n_boxes']} boxes): field rel L2 {l2f:.2e} (worst {worstf:.2e}); "
        f"E.n rel L2 {l2:.2e} (worst {worst:.2e})")
    assert l2f < 1e-5 and worstf < 1e-3 and l2 < 1e-5
    opts = F.fmm_default_options(order=8, leaf_size=128, src_kernels=F.FMM_SRC_SINGLE, outputs=F.FMM_OUT_FIELD)
    plan = F.fmm_setup(dev(xyz), None, None, dev(nrm), options=opts)
    sd = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    rc, it, rr = F.gmres_solve(plan, F.FMM_OP_DIELECTRIC, dev(a.astype(np.float32)), dev(np.float32(c)),
                               dev(w.astype(np.float32)), dev(b), sd, rtol=1e-6, restart=30, max_iter=200)
    torch.cuda.synchronize()
    F.fmm_destroy(plan)
    s = sd.cpu().numpy()
    say(f"  GMRES: rc={rc} iterations={it} relative residual {rr:.2e}")
    assert rc == F.FMM_OK and rr <= 1e-6 and it <= 40
    res = _sampled_dielectric_residual(xyz, nrm, a, np.broadcast_to(c, (n,)), w, b, s, rows)
    tr = np.linalg.norm(res) / np.linalg.norm(b[rows])
    say(f"  true residual of the exact operator at {len(rows)} rows: {tr:.2e}")
    assert tr < 2e-5


def test_ferromagnet_batch_at_full_size():
    import torch

    import paper_1605_01715_amd as F

    insts = W.ferro_batch(256)
    so = np.concatenate([[0], np.cumsum([len(i["src"]) for i in insts])])
    to = np.concatenate([[0], np.cumsum([len(i["trg"]) for i in insts])])
    say(f"test_ferromagnet_batch_at_full_size: 256 instances, {to[-1]} targets, {so[-1]} sources, 3 rhs")
    # mu_c = 4 pi M_c y_c w: phi_1 of the instance's magnetisation, one component per rhs
    mus = []
    for d in insts:
        y, wt = d["src"].astype(np.float64), d["weights"].astype(np.float64)
        mus.append(np.stack([4 * np.pi * d["M"][c] * y[:, c] * wt for c in range(3)]).astype(np.float32))
    src = np.concatenate([d["src"] for d in insts])
    nrm = np.concatenate([d["normals"] for d in insts])
    trg = np.concatenate([d["trg"] for d in insts])
    mu = np.ascontiguousarray(np.concatenate(mus, axis=1))
    opts = F.fmm_default_options(order=8, leaf_size=128, src_kernels=F.FMM_SRC_DOUBLE, outputs=F.FMM_OUT_POT,
                                 nrhs=3, precision=1)
    plan = F.fmm_setup_batch(so, dev(src), dev(nrm), to, dev(trg), options=opts)
    F.fmm_set_graph(plan, True)
    mud = dev(mu)
    pot = torch.empty(3 * int(to[-1]), device="cuda:0")
    outs = []
    for _ in range(3):  # capture, then two replays, with host work in between
        pot.fill_(float("nan"))
        F.fmm_apply(plan, mu=mud, pot=pot)
        torch.cuda.synchronize()
        outs.append(pot.cpu().numpy().astype(np.float64).reshape(3, -1))
    F.fmm_destroy(plan)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    got = outs[0]
    assert np.all(np.isfinite(got))
    # every instance against a plan of its own
    worst_one = 0.0
    for i, d in enumerate(insts):
        one = fmm_run(d["src"], mu=mus[i], nrm=d["normals"], trg=d["trg"], order=8, leaf=128, nrhs=3,
                      precision=1)["pot"]
        l2, wt = errors(got[:, to[i]:to[i + 1]], one)
        worst_one = max(worst_one, l2)
        assert l2 < 1e-6 and wt < 1e-4, (i, l2, wt)
    say(f"  batch vs 256 separate plans: largest rel L2 {worst_one:.2e}")
    for i in np.sort(np.random.default_rng(1).choice(256, 6, replace=False)):
        d = insts[i]
        rows = np.arange(len(d["trg"]))
        if len(rows) > 2000:
            rows = np.sort(np.random.default_rng(int(i)).choice(len(rows), 2000, replace=False))
        dip = [mus[i][c].astype(np.float64)[:, None] * d["normals"].astype(np.float64) for c in range(3)]
        ref = np.stack([D.direct_sum(d["trg"][rows], d["src"], None, dip[c])[0] for c in range(3)])
        l2, wt = errors(got[:, to[i]:to[i + 1]][:, rows], ref)
        say(f"  instance {i} ({d['kind']}, {len(d['trg'])} targets): vs direct rel L2 {l2:.2e}, worst {wt:.2e}")
        assert l2 < 5e-6 and wt < 5e-4
