"""ctypes declarations of the C ABI in include/fmm.h (libfmm_mi355x.so)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FMM_MI355X_LIB selects another build of the same library (for testing builds)
LIB_PATH = os.environ.get("FMM_MI355X_LIB") or os.path.join(HERE, "libfmm_mi355x.so")

c_int, c_int64, c_float, c_double, c_void_p = (ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_double,
                                               ctypes.c_void_p)

FMM_OK, FMM_ERR_ARG, FMM_ERR_NOMEM, FMM_ERR_DEVICE, FMM_ERR_NOT_CONVERGED, FMM_ERR_STATE = range(6)
FMM_SRC_SINGLE, FMM_SRC_DOUBLE = 1, 2
FMM_OUT_POT, FMM_OUT_FIELD = 1, 2
FMM_PREC_FP32, FMM_PREC_SPLIT_BF16, FMM_PREC_SPLIT_BF16X3, FMM_PREC_SPLIT_BF16X4 = 0, 1, 2, 3
FMM_BASIS_SURFACE, FMM_BASIS_CHEBYSHEV = 0, 1
FMM_OP_FK, FMM_OP_DIELECTRIC = 1, 2
STAGES = ("P2M", "M2M", "P2L", "M2L", "L2L", "C2E", "EVAL")


class FmmOptions(ctypes.Structure):
    _fields_ = [("order", c_int), ("leaf_size", c_int), ("uniform_depth", c_int), ("max_depth", c_int),
                ("precision", c_int), ("src_kernels", c_int), ("outputs", c_int), ("nrhs", c_int),
                ("cutoff", c_float), ("root", c_double * 4), ("pinv_eps", c_double), ("m2l_pieces", c_int),
                ("basis", c_int)]


class FmmOperator(ctypes.Structure):
    _fields_ = [("kind", c_int), ("a", c_void_p), ("c", c_void_p), ("w", c_void_p)]


class FmmInfo(ctypes.Structure):
    _fields_ = [(n, c_int64) for n in ("n_src", "n_trg", "n_points", "n_boxes", "n_leaves", "n_levels", "n_u", "n_v",
                                       "n_w", "n_x", "n_surface", "p2p_pairs", "m2l_pairs", "surf_evals",
                                       "p2m_evals", "m2l_columns", "rank", "m2l_pieces", "m2l_pair_tiles", "basis")] + [("root", c_double * 4),
                                                                                 ("setup_ms", c_double),
                                                                                 ("leaf_size", c_int64),
                                                                                 ("leaf_from_cache", c_int64),
                                                                                 ("p2l_evals", c_int64),
                                                                                 ("setup_phase_ms", c_double * 8)]


class FmmTuneSpace(ctypes.Structure):
    _fields_ = [("n_leaf", c_int), ("leaf_sizes", c_int * 8), ("n_pieces", c_int), ("pieces", c_int * 4),
                ("reps", c_int)]


class FmmTuneResult(ctypes.Structure):
    _fields_ = [("leaf_size", c_int), ("m2l_pieces", c_int), ("ms", c_double), ("n_tried", c_int),
                ("tried_leaf", c_int * 32), ("tried_pieces", c_int * 32), ("tried_ms", c_double * 32),
                ("tried_setup_ms", c_double * 32)]


class FmmTreeExport(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ("level", "anchor", "parent", "begin", "end", "tbeg", "tend", "sbeg", "send",
                                        "u_off", "u_idx", "v_off", "v_idx", "w_off", "w_idx", "x_off", "x_idx",
                                        "src_perm", "trg_perm", "keys")]


# name -> (restype, argtypes)
SIGNATURES = {
    "fmm_default_options": (None, [ctypes.POINTER(FmmOptions)]),
    "fmm_setup": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_int64, ctypes.POINTER(FmmOptions),
                          c_void_p, ctypes.POINTER(c_void_p)]),
    "fmm_setup_batch": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                ctypes.POINTER(FmmOptions), c_void_p, ctypes.POINTER(c_void_p)]),
    "fmm_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gmres_solve": (c_int, [c_void_p, ctypes.POINTER(FmmOperator), c_void_p, c_void_p, c_double, c_int, c_int,
                            ctypes.POINTER(c_int), ctypes.POINTER(c_double), c_void_p]),
    "fmm_destroy": (c_int, [c_void_p]),
    "fmm_last_error": (ctypes.c_char_p, []),
    "fmm_direct": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_float, c_void_p,
                           c_void_p, c_void_p]),
    "fmm_plan_info": (c_int, [c_void_p, ctypes.POINTER(FmmInfo)]),
    "fmm_export_tree": (c_int, [c_void_p, ctypes.POINTER(FmmTreeExport)]),
    "fmm_set_graph": (c_int, [c_void_p, c_int]),
    "fmm_dielectric_rhs": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_void_p,
                                   c_void_p]),
    "fmm_dielectric_rhs_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p,
                                           c_void_p, c_void_p]),
    "fmm_body_forces": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_int,
                                c_void_p, c_void_p, c_void_p]),
    "fmm_set_timing": (c_int, [c_void_p, c_int]),
    "fmm_export_stage": (c_int, [c_void_p, c_int, c_void_p]),
    "fmm_stage_times": (c_int, [c_void_p, ctypes.POINTER(c_double)]),
    "fmm_pinv": (c_int, [c_void_p, c_int, c_double, c_void_p]),
    "fmm_autotune": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_int64,
                             ctypes.POINTER(FmmOptions), ctypes.POINTER(FmmTuneSpace), ctypes.c_char_p,
                             ctypes.POINTER(FmmTuneResult), c_void_p]),
    "fmm_split_bf16": (c_int, [c_int, c_int, c_int64, c_void_p, c_void_p, c_void_p]),
    "fmm_issue_probe": (c_int, [c_int, c_int64, c_int, c_void_p, ctypes.POINTER(c_int64), c_void_p]),
    "fmm_unit_surface": (c_int, [c_int, c_void_p, ctypes.POINTER(c_int)]),
}

_lib = None


def load():
    """Load the HIP library; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(or python paper_1605_01715_amd/build.py)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
