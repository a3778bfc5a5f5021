"""Helpers shared by the GPU tests: move inputs to the device, run the
library through its C ABI, bring results back as float64 numpy arrays."""

import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def fmm_run(xyz, q=None, mu=None, nrm=None, trg=None, trg_nrm=None, field=False, order=6, leaf=64, depth=0,
            root=None, precision=0, nrhs=1, cutoff=1e-5, pinv_eps=0.0, keep_plan=False, m2l_pieces=0, basis=0):
    """One setup + apply; q/mu are [nrhs, n_src] (or [n_src]). Returns dict."""
    import torch

    import paper_1605_01715_amd as F

    kern = (F.FMM_SRC_SINGLE if q is not None else 0) | (F.FMM_SRC_DOUBLE if mu is not None else 0)
    outs = F.FMM_OUT_FIELD if field else F.FMM_OUT_POT
    kw = dict(order=order, leaf_size=leaf, uniform_depth=depth, precision=precision, src_kernels=kern,
              outputs=outs, nrhs=nrhs, cutoff=cutoff, pinv_eps=pinv_eps, m2l_pieces=m2l_pieces, basis=basis)
    if root is not None:
        kw["root"] = root
    opts = F.fmm_default_options(**kw)
    x = dev(np.asarray(xyz, np.float32))
    n = dev(np.asarray(nrm, np.float32)) if nrm is not None else None
    t = dev(np.asarray(trg, np.float32)) if trg is not None else None
    tn = dev(np.asarray(trg_nrm, np.float32)) if trg_nrm is not None else None
    plan = F.fmm_setup(x, n, t, tn, options=opts)
    nt = len(trg) if trg is not None else len(xyz)
    qq = dev(np.asarray(q, np.float32).reshape(nrhs, -1)) if q is not None else None
    mm = dev(np.asarray(mu, np.float32).reshape(nrhs, -1)) if mu is not None else None
    pot = torch.empty(nrhs * nt, device="cuda:0") if not field else None
    fld = torch.empty(nrhs * nt * 3, device="cuda:0") if field else None
    F.fmm_apply(plan, q=qq, mu=mm, pot=pot, field=fld)
    torch.cuda.synchronize()
    out = {"info": F.fmm_plan_info(plan)}
    if pot is not None:
        out["pot"] = pot.cpu().numpy().astype(np.float64).reshape(nrhs, nt)
    if fld is not None:
        out["field"] = fld.cpu().numpy().astype(np.float64).reshape(nrhs, nt, 3)
    if keep_plan:
        out["plan"] = plan
    else:
        F.fmm_destroy(plan)
    return out


def errors(got, ref):
    """(relative L2 error, worst-target error): the worst target's error
    relative to the root-mean-square output, max_i |got_i - ref_i| / rms(ref),
    with vector outputs (last axis 3) compared per target as vectors. A bound
    on the second catches a few wrong targets that an L2 norm over many would
    average away."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(r)
    l2 = float(np.linalg.norm(g - r) / den) if den > 0 else float(np.linalg.norm(g))
    if r.ndim >= 1 and r.shape[-1] == 3 and r.ndim >= 2:
        d = np.linalg.norm(g - r, axis=-1).ravel()
        m = np.linalg.norm(r, axis=-1).ravel()
    else:
        d = np.abs(g - r).ravel()
        m = np.abs(r).ravel()
    rms = float(np.sqrt(np.mean(m * m))) if m.size else 0.0
    worst = float(d.max() / rms) if rms > 0 and d.size else float(d.max() if d.size else 0.0)
    return l2, worst
