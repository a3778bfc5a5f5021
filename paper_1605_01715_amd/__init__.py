"""MI355X kernel-independent FMM for boundary integrals (arXiv:1605.01715 hot path).

Thin Python binding of the C ABI in include/fmm.h. The functions here carry
the same names as the C entry points and only marshal arguments: torch
tensors (device memory, streams) go in as raw pointers, and every step of the
computation runs in the HIP library. If the library is not built, importing
works but the first call raises ImportError.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from ._lib import (FMM_BASIS_CHEBYSHEV, FMM_BASIS_SURFACE, FMM_ERR_ARG, FMM_ERR_DEVICE, FMM_ERR_NOMEM,
                   FMM_ERR_NOT_CONVERGED, FMM_ERR_STATE, FMM_OK, FMM_OP_DIELECTRIC, FMM_OP_FK, FMM_OUT_FIELD,
                   FMM_OUT_POT, FMM_PREC_FP32, FMM_PREC_SPLIT_BF16, FMM_PREC_SPLIT_BF16X3, FMM_PREC_SPLIT_BF16X4,
                   FMM_SRC_DOUBLE, FMM_SRC_SINGLE, STAGES)

__all__ = ["fmm_setup_batch", "Plan", "FmmError", "fmm_default_options", "fmm_setup", "fmm_apply", "gmres_solve", "fmm_destroy",
           "fmm_last_error", "fmm_direct", "fmm_plan_info", "fmm_export_tree", "fmm_export_stage",
           "fmm_set_timing", "fmm_set_graph", "fmm_dielectric_rhs", "fmm_body_forces", "fmm_stage_times", "fmm_pinv", "fmm_unit_surface", "fmm_split_bf16", "fmm_dielectric_rhs_noalloc", "fmm_autotune", "fmm_issue_probe",
           "library_path"]


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[fmm status {code}] {msg}")
        self.code = code


def library_path():
    return L.LIB_PATH


def _check(rc):
    if rc != FMM_OK:
        raise FmmError(rc, fmm_last_error())
    return rc


def _ptr(t, dtype=None, name="array"):
    """Device pointer of a contiguous torch tensor (or None/int passthrough)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def fmm_last_error():
    return L.load().fmm_last_error().decode()


def fmm_default_options(**kw):
    """FmmOptions with the library defaults, then the given fields set."""
    o = L.FmmOptions()
    L.load().fmm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "root":
            for i in range(4):
                o.root[i] = float(v[i])
        else:
            setattr(o, k, v)
    return o


class Plan:
    """Handle of an fmm_plan (owned by the library until fmm_destroy)."""

    def __init__(self, handle, opts, n_src, n_trg):
        self.handle = handle
        self.opts = opts
        self.n_src = n_src
        self.n_trg = n_trg
        self.nrhs = opts.nrhs

    def __del__(self):
        try:
            if self.handle:
                fmm_destroy(self)
        except Exception:
            pass


def fmm_setup(src_xyz, src_nrm=None, trg_xyz=None, trg_nrm=None, options=None, stream=None):
    import torch

    lib = L.load()
    opts = options if options is not None else fmm_default_options()
    n_src = int(src_xyz.shape[0])
    n_trg = int(trg_xyz.shape[0]) if trg_xyz is not None else n_src
    h = ctypes.c_void_p()
    f32 = torch.float32
    _check(lib.fmm_setup(_ptr(src_xyz, f32, "src_xyz"), _ptr(src_nrm, f32, "src_nrm"), n_src,
                         _ptr(trg_xyz, f32, "trg_xyz"), _ptr(trg_nrm, f32, "trg_nrm"),
                         n_trg if trg_xyz is not None else 0, ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
    return Plan(h.value, opts, n_src, n_trg)


def fmm_setup_batch(src_off, src_xyz, src_nrm=None, trg_off=None, trg_xyz=None, trg_nrm=None, options=None,
                    stream=None):
    """One plan over independent instances; offsets are host sequences of n_inst + 1 prefix sums."""
    import numpy as np
    import torch

    lib = L.load()
    opts = options if options is not None else fmm_default_options()
    so = np.ascontiguousarray(np.asarray(src_off, dtype=np.int64))
    to = np.ascontiguousarray(np.asarray(trg_off, dtype=np.int64)) if trg_off is not None else None
    n_inst = len(so) - 1
    h = ctypes.c_void_p()
    f32 = torch.float32
    _check(lib.fmm_setup_batch(n_inst, so.ctypes.data, to.ctypes.data if to is not None else None,
                               _ptr(src_xyz, f32, "src_xyz"), _ptr(src_nrm, f32, "src_nrm"),
                               _ptr(trg_xyz, f32, "trg_xyz"), _ptr(trg_nrm, f32, "trg_nrm"), ctypes.byref(opts),
                               _stream(stream), ctypes.byref(h)))
    n_src = int(so[-1])
    return Plan(h.value, opts, n_src, int(to[-1]) if to is not None else n_src)


def fmm_apply(plan, q=None, mu=None, pot=None, field=None, stream=None):
    import torch

    f32 = torch.float32
    _check(L.load().fmm_apply(plan.handle, _ptr(q, f32, "q"), _ptr(mu, f32, "mu"), _ptr(pot, f32, "pot"),
                              _ptr(field, f32, "field"), _stream(stream)))


def gmres_solve(plan, kind, a, c, w, b, x, rtol=1e-6, restart=30, max_iter=500, stream=None):
    """Returns (status, iterations, relative residual); x is updated in place."""
    import torch

    op = L.FmmOperator(kind, _ptr(a, torch.float32, "a"), _ptr(c, torch.float32, "c"), _ptr(w, torch.float32, "w"))
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = L.load().gmres_solve(plan.handle, ctypes.byref(op), _ptr(b, torch.float64, "b"), _ptr(x, torch.float64, "x"),
                              float(rtol), int(restart), int(max_iter), ctypes.byref(it), ctypes.byref(rr),
                              _stream(stream))
    if rc not in (FMM_OK, FMM_ERR_NOT_CONVERGED):
        _check(rc)
    return rc, it.value, rr.value


def fmm_destroy(plan):
    if plan is None or not plan.handle:
        return
    h = plan.handle
    plan.handle = None
    _check(L.load().fmm_destroy(h))


def fmm_direct(src_xyz, trg_xyz, q=None, mu=None, src_nrm=None, cutoff=1e-5, pot=None, field=None, stream=None):
    import torch

    f32 = torch.float32
    _check(L.load().fmm_direct(_ptr(src_xyz, f32, "src_xyz"), _ptr(src_nrm, f32, "src_nrm"), int(src_xyz.shape[0]),
                               _ptr(trg_xyz, f32, "trg_xyz"), int(trg_xyz.shape[0]), _ptr(q, f32, "q"),
                               _ptr(mu, f32, "mu"), float(cutoff), _ptr(pot, f32, "pot"), _ptr(field, f32, "field"),
                               _stream(stream)))


SETUP_PHASES = ("sort", "octree", "lists", "operators", "buffers", "m2l_schedule", "worklists", "unused")


def fmm_plan_info(plan):
    info = L.FmmInfo()
    _check(L.load().fmm_plan_info(plan.handle, ctypes.byref(info)))
    d = {name: getattr(info, name) for name, _ in L.FmmInfo._fields_ if name not in ("root", "setup_phase_ms")}
    d["root"] = tuple(info.root)
    d["setup_phase_ms"] = dict(zip(SETUP_PHASES, info.setup_phase_ms))
    return d


def fmm_export_tree(plan):
    """Host copies of the tree and lists as numpy arrays."""
    info = fmm_plan_info(plan)
    nb = info["n_boxes"]
    out = {
        "level": np.zeros(nb, np.int32), "anchor": np.zeros((nb, 3), np.int32), "parent": np.zeros(nb, np.int32),
        "begin": np.zeros(nb, np.int64), "end": np.zeros(nb, np.int64), "tbeg": np.zeros(nb, np.int64),
        "tend": np.zeros(nb, np.int64), "sbeg": np.zeros(nb, np.int64), "send": np.zeros(nb, np.int64),
        "src_perm": np.zeros(info["n_src"], np.int64), "trg_perm": np.zeros(info["n_trg"], np.int64),
        "keys": np.zeros(info["n_points"], np.uint64),
    }
    for k in "uvwx":
        out[k + "_off"] = np.zeros(nb + 1, np.int32)
        out[k + "_idx"] = np.zeros(max(info["n_" + k], 1), np.int32)
    e = L.FmmTreeExport(**{k: v.ctypes.data for k, v in out.items()})
    _check(L.load().fmm_export_tree(plan.handle, ctypes.byref(e)))
    for k in "uvwx":
        out[k + "_idx"] = out[k + "_idx"][: info["n_" + k]]
    return out


def fmm_export_stage(plan, which):
    info = fmm_plan_info(plan)
    out = np.zeros((info["n_boxes"], info["n_surface"]), np.float32)
    _check(L.load().fmm_export_stage(plan.handle, int(which), out.ctypes.data))
    return out


def fmm_dielectric_rhs(plan, sigma_f, areas, curvature, eps_i, eps_m, e0=None, b=None, stream=None):
    """Right-hand side of the dielectric system with free charges; returns b (device float64)."""
    import numpy as np
    import torch

    f32 = torch.float32
    if b is None:
        b = torch.empty(sigma_f.shape[0], dtype=torch.float64, device=sigma_f.device)
    e = np.ascontiguousarray(np.asarray(e0, dtype=np.float64)) if e0 is not None else None
    _check(L.load().fmm_dielectric_rhs(plan.handle, _ptr(sigma_f, f32, "sigma_f"), _ptr(areas, f32, "areas"),
                                       _ptr(curvature, f32, "curvature"), _ptr(eps_i, f32, "eps_i"), float(eps_m),
                                       e.ctypes.data if e is not None else None, _ptr(b, torch.float64, "b"),
                                       _stream(stream)))
    return b


def fmm_body_forces(plan, sigma_f, sigma_b, areas, curvature, eps_m, body_off, e0=None, stream=None):
    """Forces on the bodies (host float64 [n_body, 3])."""
    import numpy as np
    import torch

    f32 = torch.float32
    off = np.ascontiguousarray(np.asarray(body_off, dtype=np.int64))
    out = np.zeros((len(off) - 1, 3))
    e = np.ascontiguousarray(np.asarray(e0, dtype=np.float64)) if e0 is not None else None
    _check(L.load().fmm_body_forces(plan.handle, _ptr(sigma_f, f32, "sigma_f"), _ptr(sigma_b, f32, "sigma_b"),
                                    _ptr(areas, f32, "areas"), _ptr(curvature, f32, "curvature"), float(eps_m),
                                    e.ctypes.data if e is not None else None, len(off) - 1, off.ctypes.data,
                                    out.ctypes.data, _stream(stream)))
    return out


def fmm_set_graph(plan, enable=True):
    _check(L.load().fmm_set_graph(plan.handle, int(bool(enable))))


def fmm_set_timing(plan, enable=True):
    _check(L.load().fmm_set_timing(plan.handle, int(bool(enable))))


def fmm_stage_times(plan):
    ms = (ctypes.c_double * len(STAGES))()
    _check(L.load().fmm_stage_times(plan.handle, ms))
    return dict(zip(STAGES, list(ms)))


def fmm_pinv(K, eps):
    """Host truncated-SVD pseudo-inverse used by the plan's operator precompute."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    n = K.shape[0]
    out = np.zeros((n, n))
    _check(L.load().fmm_pinv(K.ctypes.data, n, float(eps), out.ctypes.data))
    return out


def fmm_unit_surface(p):
    ns = ctypes.c_int(0)
    _check(L.load().fmm_unit_surface(int(p), None, ctypes.byref(ns)))
    out = np.zeros((ns.value, 3))
    _check(L.load().fmm_unit_surface(int(p), out.ctypes.data, ctypes.byref(ns)))
    return out


def fmm_split_bf16(which, r_pad, values, stream=None):
    """The library's three-part bfloat16 split of a float32 device tensor
    (which 0: count vectors of r_pad values; which 1: count r_pad x r_pad
    matrices). Returns a device uint16-bit int16 tensor [3][values.numel()]."""
    import torch

    n = int(values.numel())
    per = r_pad * (r_pad if which == 1 else 1)
    if n % per:
        raise ValueError("fmm_split_bf16: values do not fill whole vectors or matrices")
    parts = torch.empty(3 * n, dtype=torch.int16, device=values.device)
    _check(L.load().fmm_split_bf16(int(which), int(r_pad), n // per, _ptr(values, torch.float32, "values"),
                                    parts.data_ptr(), _stream(stream)))
    return parts.view(3, n)


def fmm_issue_probe(kind, out, iters, stream=None):
    """Queue the library's issue-rate probe of the given kind on the stream
    over out.numel() lanes (out: device float32, a multiple of 256 values).
    Returns the wave64 VALU instructions of its chains per lane."""
    import torch

    instr = ctypes.c_int64(0)
    _check(L.load().fmm_issue_probe(int(kind), int(out.numel()), int(iters), _ptr(out, torch.float32, "out"),
                                    ctypes.byref(instr), _stream(stream)))
    return instr.value


def fmm_dielectric_rhs_noalloc(plan, sigma_f, areas, curvature, eps_i, eps_m, b, e0=None, stream=None):
    """fmm_dielectric_rhs without device allocation: b (device float64 [n]) is
    written in stream order, the charge and its field live in the library's
    fixed per-GPU scratch."""
    import numpy as np
    import torch

    f32 = torch.float32
    e = np.ascontiguousarray(np.asarray(e0, dtype=np.float64)) if e0 is not None else None
    _check(L.load().fmm_dielectric_rhs_noalloc(plan.handle, _ptr(sigma_f, f32, "sigma_f"), _ptr(areas, f32, "areas"),
                                               _ptr(curvature, f32, "curvature"), _ptr(eps_i, f32, "eps_i"),
                                               float(eps_m), e.ctypes.data if e is not None else None,
                                               _ptr(b, torch.float64, "b"), _stream(stream)))
    return b


def fmm_autotune(src_xyz, src_nrm=None, trg_xyz=None, trg_nrm=None, options=None, leaf_sizes=(64, 128, 192, 256),
                 pieces=(), reps=3, cache_path="", src_off=None, trg_off=None, stream=None):
    """Leaf-size tuning by trial runs; returns a dict with the choice and every
    trial. cache_path: "" the default cache file, None no cache, else a path.
    src_off / trg_off (host prefix offsets) make it a batch as in fmm_setup_batch."""
    import torch

    lib = L.load()
    opts = options if options is not None else fmm_default_options()
    sp = L.FmmTuneSpace()
    sp.n_leaf = len(leaf_sizes)
    for i, v in enumerate(leaf_sizes):
        sp.leaf_sizes[i] = int(v)
    sp.n_pieces = len(pieces)
    for i, v in enumerate(pieces):
        sp.pieces[i] = int(v)
    sp.reps = int(reps)
    res = L.FmmTuneResult()
    f32 = torch.float32
    so = np.ascontiguousarray(np.asarray(src_off, dtype=np.int64)) if src_off is not None else None
    to = np.ascontiguousarray(np.asarray(trg_off, dtype=np.int64)) if trg_off is not None else None
    n_inst = len(so) - 1 if so is not None else 0
    n_src = int(src_xyz.shape[0])
    n_trg = int(trg_xyz.shape[0]) if trg_xyz is not None else 0
    cp = None if cache_path is None else str(cache_path).encode()
    _check(lib.fmm_autotune(n_inst, so.ctypes.data if so is not None else None, to.ctypes.data if to is not None else None,
                            _ptr(src_xyz, f32, "src_xyz"), _ptr(src_nrm, f32, "src_nrm"), n_src,
                            _ptr(trg_xyz, f32, "trg_xyz"), _ptr(trg_nrm, f32, "trg_nrm"), n_trg, ctypes.byref(opts),
                            ctypes.byref(sp), cp, ctypes.byref(res), _stream(stream)))
    tried = [{"leaf": res.tried_leaf[i], "m2l_pieces": res.tried_pieces[i], "ms": res.tried_ms[i],
              "setup_ms": res.tried_setup_ms[i]} for i in range(res.n_tried)]
    return {"leaf_size": res.leaf_size, "m2l_pieces": res.m2l_pieces, "ms": res.ms, "tried": tried}
