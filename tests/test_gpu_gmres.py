"""GMRES through the C ABI (gmres_solve) on the paper's two model operators,
against the oracle's GMRES on the float64 direct sum and against closed forms.

The GPU matvec is the FMM in float32; with matvec relative error e and a
well-conditioned second-kind operator (condition number k of a few) the
solutions agree to about k e, far above the GMRES tolerance, so the bounds
below are set at the FMM error level, not at rtol.
"""

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import direct as D
from oracle import operators as OP
from oracle.gmres import gmres

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def _plan(xyz, nrm, kernels, outputs, trg_nrm=None, order=8, leaf=64, precision=0, basis=0):
    import paper_1605_01715_amd as F

    opts = F.fmm_default_options(order=order, leaf_size=leaf, src_kernels=kernels, outputs=outputs,
                                 precision=precision, basis=basis)
    x = dev(np.asarray(xyz, np.float32))
    n = dev(np.asarray(nrm, np.float32))
    tn = dev(np.asarray(trg_nrm, np.float32)) if trg_nrm is not None else None
    return F.fmm_setup(x, n, None, tn, options=opts)


def _solve(plan, kind, a, c, w, b, rtol, restart=30, max_iter=200, x0=None):
    import torch

    import paper_1605_01715_amd as F

    ad, wd = dev(np.asarray(a, np.float32)), dev(np.asarray(w, np.float32))
    cd = dev(np.asarray(c, np.float32)) if c is not None else None
    bd = dev(np.asarray(b, np.float64))
    xd = dev(np.zeros(len(b)) if x0 is None else np.asarray(x0, np.float64))
    rc, it, rr = F.gmres_solve(plan, kind, ad, cd, wd, bd, xd, rtol=rtol, restart=restart, max_iter=max_iter)
    torch.cuda.synchronize()
    return rc, it, rr, xd.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_fk_interior_dirichlet_on_eight_spheres(precision):
    """(D_pv - I/2) mu = 1/|r - r0| on the 8-sphere lattice (Eq. fk_integral with
    Omega = 2 pi): GPU GMRES against the oracle GMRES on the direct sum."""
    import paper_1605_01715_amd as F

    d = W.spheres_8(freq=9)
    xyz, nrm, w, g = d["xyz"], d["normals"], d["weights"], d["g"]
    n = len(w)
    say(f"test_fk_interior_dirichlet_on_eight_spheres: n={n} precision={precision}")
    a = np.full(n, -0.5)
    plan = _plan(xyz, nrm, F.FMM_SRC_DOUBLE, F.FMM_OUT_POT, precision=precision)
    rc, it, rr, x = _solve(plan, F.FMM_OP_FK, a, None, w, g, rtol=1e-7)
    F.fmm_destroy(plan)
    say(f"  GPU GMRES: rc={rc} iterations={it} relative residual={rr:.2e}")
    assert rc == F.FMM_OK and rr <= 1e-7
    x64, w64, n64 = xyz.astype(np.float64), w.astype(np.float64), nrm.astype(np.float64)
    ref, it_o, rr_o, ok = gmres(lambda v: OP.fk_apply(v, x64, n64, w64, a), g, rtol=1e-10)
    assert ok
    err = D.rel_l2(x, ref)
    say(f"  oracle GMRES iterations={it_o}; solution rel L2 = {err:.2e}")
    assert err < 2e-5
    # the solution reproduces the data: (D_pv - I/2) x = g with the direct operator
    res = D.rel_l2(OP.fk_apply(x, x64, n64, w64, a), g)
    assert res < 2e-5


@pytest.mark.parametrize("order,tol", [(5, 1e-3), (7, 5e-5)])
def test_fk_and_dielectric_with_the_chebyshev_form(order, tol):
    """Both model problems solved with the paper's Chebyshev form (order 5 is
    the paper's setting): GPU GMRES against the oracle GMRES on the direct
    sum, at the interpolation error of that order. The solves stop at 1e-6:
    the float32 matvec of this form has a noise floor near 2e-7 (GMRES
    stalls there; the surface form's is just below 1e-7), and at order 5 the
    matvec itself is only accurate to about 1e-4."""
    import paper_1605_01715_amd as F

    d = W.spheres_8(freq=9)
    xyz, nrm, w, g = d["xyz"], d["normals"], d["weights"], d["g"]
    n = len(w)
    say(f"test_fk_and_dielectric_with_the_chebyshev_form: FK n={n} order {order}")
    a = np.full(n, -0.5)
    plan = _plan(xyz, nrm, F.FMM_SRC_DOUBLE, F.FMM_OUT_POT, basis=F.FMM_BASIS_CHEBYSHEV, order=order, precision=1)
    rc, it, rr, x = _solve(plan, F.FMM_OP_FK, a, None, w, g, rtol=1e-6)
    F.fmm_destroy(plan)
    assert rc == F.FMM_OK and it <= 20
    x64, w64, n64 = xyz.astype(np.float64), w.astype(np.float64), nrm.astype(np.float64)
    ref, _, _, ok = gmres(lambda v: OP.fk_apply(v, x64, n64, w64, a), g, rtol=1e-10)
    assert ok
    err = D.rel_l2(x, ref)
    say(f"  FK: iterations={it}; solution rel L2 against the oracle = {err:.2e}")
    assert err < tol
    d = W.dielectric(n_spheres=12, freq=8, box=12.0)
    xyz, nrm = d["xyz"], d["normals"]
    a, c, w = OP.dielectric_coeffs(d["areas"], d["curvature"], d["eps_i"], d["eps_m"])
    b = OP.dielectric_rhs(nrm, d["eps_i"], d["eps_m"], d["e0"])
    plan = _plan(xyz, nrm, F.FMM_SRC_SINGLE, F.FMM_OUT_FIELD, trg_nrm=nrm, basis=F.FMM_BASIS_CHEBYSHEV, order=order)
    rc, it, rr, x = _solve(plan, F.FMM_OP_DIELECTRIC, a, c, w, b, rtol=1e-6)
    F.fmm_destroy(plan)
    assert rc == F.FMM_OK and it <= 20
    x64, n64 = xyz.astype(np.float64), nrm.astype(np.float64)
    ref, _, _, ok = gmres(lambda s: OP.dielectric_apply(s, x64, n64, a, c, w), b, rtol=1e-10)
    assert ok
    err = D.rel_l2(x, ref)
    say(f"  dielectric (field output): iterations={it}; solution rel L2 against the oracle = {err:.2e}")
    assert err < tol


def test_dielectric_spheres_against_oracle():
    """Eq. Ax with Eq. pol_discret on 12 random dielectric spheres in a uniform
    field (Eq. rhs, no free charge): GPU GMRES against the oracle's."""
    import paper_1605_01715_amd as F

    d = W.dielectric(n_spheres=12, freq=8, box=12.0)
    xyz, nrm = d["xyz"], d["normals"]
    n = len(xyz)
    say(f"test_dielectric_spheres_against_oracle: n={n}")
    a, c, w = OP.dielectric_coeffs(d["areas"], d["curvature"], d["eps_i"], d["eps_m"])
    b = OP.dielectric_rhs(nrm, d["eps_i"], d["eps_m"], d["e0"])
    plan = _plan(xyz, nrm, F.FMM_SRC_SINGLE, F.FMM_OUT_FIELD, trg_nrm=nrm)
    rc, it, rr, x = _solve(plan, F.FMM_OP_DIELECTRIC, a, c, w, b, rtol=1e-7)
    F.fmm_destroy(plan)
    say(f"  GPU GMRES: rc={rc} iterations={it} relative residual={rr:.2e}")
    assert rc == F.FMM_OK and rr <= 1e-7
    x64, n64 = xyz.astype(np.float64), nrm.astype(np.float64)
    ref, it_o, rr_o, ok = gmres(lambda s: OP.dielectric_apply(s, x64, n64, a, c, w), b, rtol=1e-10)
    assert ok
    err = D.rel_l2(x, ref)
    say(f"  oracle GMRES iterations={it_o}; solution rel L2 = {err:.2e}")
    assert err < 2e-5


def test_single_dielectric_sphere_closed_form():
    """An isolated dielectric sphere in a uniform field carries
    sigma_b = 3 (e_i - e_m)/(e_i + 2 e_m) E0 . n, to discretisation error."""
    import paper_1605_01715_amd as F

    xyz, nrm, w = W.sphere_quadrature(24, np.zeros(3), 1.0)
    n = len(w)
    say(f"test_single_dielectric_sphere_closed_form: n={n}")
    eps_i, eps_m, e0 = 5.0, 1.0, np.array([0.0, 0.0, 1.0])
    ei = np.full(n, eps_i)
    a, c, ww = OP.dielectric_coeffs(w, np.ones(n), ei, eps_m)
    b = OP.dielectric_rhs(nrm, ei, eps_m, e0)
    plan = _plan(xyz, nrm, F.FMM_SRC_SINGLE, F.FMM_OUT_FIELD, trg_nrm=nrm)
    rc, it, rr, x = _solve(plan, F.FMM_OP_DIELECTRIC, a, c, ww, b, rtol=1e-6)
    F.fmm_destroy(plan)
    assert rc == F.FMM_OK
    expect = CF.dielectric_sphere_sigma(np.asarray(nrm, np.float64), eps_i, eps_m, e0)
    err = D.rel_l2(x, expect)
    say(f"  iterations={it}; rel L2 against the closed form = {err:.2e}")
    assert err < 2e-3


def test_long_restart_cycle_against_oracle():
    """A restart length above 64 (the Krylov basis and the per-step dot
    products sized by it): 70 iterations in one cycle with a tolerance the
    float32 matvec cannot reach, then the iterate against the oracle GMRES on
    the direct sum at the FMM error level."""
    import paper_1605_01715_amd as F

    d = W.spheres_8(freq=6)
    xyz, nrm, w, g = d["xyz"], d["normals"], d["weights"], d["g"]
    n = len(w)
    say(f"test_long_restart_cycle_against_oracle: n={n} restart=80 max_iter=70")
    a = np.full(n, -0.5)
    plan = _plan(xyz, nrm, F.FMM_SRC_DOUBLE, F.FMM_OUT_POT, order=6)
    rc, it, rr, x = _solve(plan, F.FMM_OP_FK, a, None, w, g, rtol=1e-15, restart=80, max_iter=70)
    F.fmm_destroy(plan)
    say(f"  GPU GMRES: rc={rc} iterations={it} relative residual={rr:.2e}")
    assert rc == F.FMM_ERR_NOT_CONVERGED and it == 70
    assert rr < 1e-5 and np.all(np.isfinite(x))
    x64, w64, n64 = xyz.astype(np.float64), w.astype(np.float64), nrm.astype(np.float64)
    ref, _, _, ok = gmres(lambda v: OP.fk_apply(v, x64, n64, w64, a), g, rtol=1e-10)
    assert ok
    err = D.rel_l2(x, ref)
    say(f"  solution rel L2 against the oracle = {err:.2e}")
    assert err < 5e-5


def test_gmres_not_converged_and_argument_errors():
    import paper_1605_01715_amd as F

    d = W.spheres_8(freq=4)
    xyz, nrm, w, g = d["xyz"], d["normals"], d["weights"], d["g"]
    n = len(w)
    say(f"test_gmres_not_converged_and_argument_errors: n={n}")
    plan = _plan(xyz, nrm, F.FMM_SRC_DOUBLE, F.FMM_OUT_POT, order=4)
    a = np.full(n, -0.5)
    rc, it, rr, x = _solve(plan, F.FMM_OP_FK, a, None, w, g, rtol=1e-14, restart=5, max_iter=3)
    assert rc == F.FMM_ERR_NOT_CONVERGED
    assert it == 3 and 0.0 < rr < 1.0 and np.all(np.isfinite(x))
    # zero right-hand side: x = 0 at once
    rc, it, rr, x = _solve(plan, F.FMM_OP_FK, a, None, w, np.zeros(n), rtol=1e-6, x0=np.ones(n))
    assert rc == F.FMM_OK and it == 0 and np.all(x == 0.0)
    # a dielectric operator on a double-layer plan is rejected before any work
    with pytest.raises(F.FmmError):
        _solve(plan, F.FMM_OP_DIELECTRIC, a, a, w, g, rtol=1e-6)
    with pytest.raises(F.FmmError):
        _solve(plan, F.FMM_OP_FK, a, None, w, g, rtol=0.0)
    F.fmm_destroy(plan)
