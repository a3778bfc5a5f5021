"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point declared in include/fmm.h, validates arguments before any
device work, and its host pseudo-inverse and unit surface match the oracle's
definitions."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")


def _lib():
    import paper_1605_01715_amd as F

    if not os.path.exists(F.library_path()):
        import __graft_entry__

        __graft_entry__.build()
    return F


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fmm_setup", "fmm_apply", "gmres_solve", "fmm_destroy", "fmm_last_error", "fmm_direct"):
        assert n in names


def test_library_exports_every_declared_symbol():
    F = _lib()
    lib = ctypes.CDLL(F.library_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []


def test_default_options():
    F = _lib()
    o = F.fmm_default_options()
    assert (o.order, o.leaf_size, o.uniform_depth, o.max_depth, o.nrhs) == (6, 64, 0, 21, 1)
    assert o.cutoff == pytest.approx(1e-5)
    assert o.src_kernels == F.FMM_SRC_SINGLE and o.outputs == F.FMM_OUT_POT
    assert o.basis == F.FMM_BASIS_SURFACE


def test_binding_structs_match_the_header(tmp_path):
    """Offsets and sizes of the option and info structs as the C compiler
    lays them out, against the ctypes mirrors."""
    import shutil
    import subprocess

    F = _lib()
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    L = F._lib
    fields = {"fmm_options": [n for n, _ in L.FmmOptions._fields_], "fmm_info": [n for n, _ in L.FmmInfo._fields_]}
    body = "".join(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));' for st, fs in fields.items() for f in fs)
    body += 'printf("fmm_options sizeof %zu\\n", sizeof(fmm_options));printf("fmm_info sizeof %zu\\n", sizeof(fmm_info));'
    src = tmp_path / "probe.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "fmm.h"\nint main(void){' + body + "return 0;}\n")
    exe = tmp_path / "probe"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call([cc, "-I", inc, str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    mirror = {"fmm_options": L.FmmOptions, "fmm_info": L.FmmInfo}
    for line in filter(None, out):
        st, f, v = line.split()
        want = ctypes.sizeof(mirror[st]) if f == "sizeof" else getattr(mirror[st], f).offset
        assert int(v) == want, (st, f)


@pytest.mark.parametrize("field,value", [("order", 1), ("order", 11), ("leaf_size", -1), ("max_depth", 22),
                                         ("nrhs", 0), ("nrhs", 5), ("precision", 7), ("src_kernels", 0),
                                         ("outputs", 4), ("basis", 2), ("basis", -1), ("cheb_order", 9),
                                         ("cheb_order", 1)])
def test_setup_rejects_bad_options_before_device_work(field, value):
    F = _lib()
    lib = F._lib.load()
    if field == "cheb_order":
        o = F.fmm_default_options(basis=F.FMM_BASIS_CHEBYSHEV, order=value)
    else:
        o = F.fmm_default_options(**{field: value})
    h = ctypes.c_void_p()
    rc = lib.fmm_setup(None, None, 0, None, None, 0, ctypes.byref(o), None, ctypes.byref(h))
    assert rc == F.FMM_ERR_ARG
    assert F.fmm_last_error() != ""
    assert h.value is None


def test_setup_rejects_null_points_and_field_with_double_layer():
    F = _lib()
    lib = F._lib.load()
    h = ctypes.c_void_p()
    o = F.fmm_default_options()
    assert lib.fmm_setup(None, None, 10, None, None, 0, ctypes.byref(o), None, ctypes.byref(h)) == F.FMM_ERR_ARG
    o = F.fmm_default_options(src_kernels=F.FMM_SRC_DOUBLE, outputs=F.FMM_OUT_FIELD)
    assert lib.fmm_setup(None, None, 0, None, None, 0, ctypes.byref(o), None, ctypes.byref(h)) == F.FMM_ERR_ARG
    assert "single layer" in F.fmm_last_error()
    assert lib.fmm_setup(None, None, -1, None, None, 0, ctypes.byref(o), None, ctypes.byref(h)) == F.FMM_ERR_ARG


def test_null_plan_calls_fail_cleanly():
    F = _lib()
    lib = F._lib.load()
    assert lib.fmm_destroy(None) == F.FMM_OK
    assert lib.fmm_apply(None, None, None, None, None, None) == F.FMM_ERR_ARG
    info = F._lib.FmmInfo()
    assert lib.fmm_plan_info(None, ctypes.byref(info)) == F.FMM_ERR_ARG


def test_unit_surface_matches_the_definition():
    F = _lib()
    from oracle.kifmm import surface

    for p in (2, 4, 6, 8, 10):
        np.testing.assert_array_equal(F.fmm_unit_surface(p), surface(p))


@pytest.mark.parametrize("p", [4, 6, 8])
def test_host_pseudo_inverse_is_a_generalised_inverse(p):
    """The library's one-sided Jacobi SVD against the mathematical definition
    (K K+ K = K) and against numpy's LAPACK SVD away from the truncation edge."""
    F = _lib()
    from oracle.kifmm import RAD_IN, RAD_OUT, pinv, slp, surface

    Y = surface(p)
    K = slp(RAD_OUT * Y, RAD_IN * Y)
    P = F.fmm_pinv(K, 1e-10)
    assert np.linalg.norm(K @ P @ K - K) / np.linalg.norm(K) < 1e-7
    # on a well-conditioned matrix the two SVDs agree to rounding
    rng = np.random.default_rng(p)
    A = np.eye(50) * 2 + rng.standard_normal((50, 50)) / 10
    np.testing.assert_allclose(F.fmm_pinv(A, 1e-12), pinv(A, 1e-12), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(F.fmm_pinv(A, 1e-12), np.linalg.inv(A), rtol=1e-10, atol=1e-12)


def test_pseudo_inverse_truncates_small_singular_values():
    F = _lib()
    u, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((20, 20)))
    v, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((20, 20)))
    s = np.logspace(0, -14, 20)
    K = (u * s) @ v.T
    P = F.fmm_pinv(K, 1e-6)
    keep = s > 1e-6
    expect = (v[:, keep] / s[keep]) @ u[:, keep].T
    np.testing.assert_allclose(P, expect, rtol=1e-6, atol=1e-6 * np.abs(expect).max())


def test_unknown_handles_are_rejected_without_being_read():
    """A pointer the library never issued is an argument error in every entry
    point that takes a plan; the library looks it up instead of reading it."""
    F = _lib()
    lib = F._lib.load()
    bogus = ctypes.c_void_p(0x10)
    assert lib.fmm_apply(bogus, None, None, None, None, None) == F.FMM_ERR_ARG
    assert "not a plan handle" in F.fmm_last_error()
    assert lib.fmm_destroy(bogus) == F.FMM_ERR_ARG
    info = F._lib.FmmInfo()
    assert lib.fmm_plan_info(bogus, ctypes.byref(info)) == F.FMM_ERR_ARG
    assert lib.fmm_set_timing(bogus, 1) == F.FMM_ERR_ARG
    assert lib.fmm_set_graph(bogus, 1) == F.FMM_ERR_ARG
    assert lib.fmm_destroy(None) == F.FMM_OK


@pytest.mark.slow
def test_host_abi_under_address_and_ub_sanitizers(tmp_path):
    """The library's host code built with AddressSanitizer and
    UndefinedBehaviorSanitizer, driven through every C entry point path that
    needs no GPU (argument checks, unknown handles, the host SVD, the unit
    surface)."""
    import shutil
    import subprocess

    from paper_1605_01715_amd import build as B

    cxx = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(cxx):
        pytest.skip("no clang++ for the sanitizer runtime")
    lib = B.build_sanitized(str(tmp_path / "san"))
    blob = open(lib, "rb").read()
    assert b"__asan_report" in blob and b"__ubsan_handle" in blob  # the host code is instrumented
    exe = tmp_path / "abi_host_checks"
    subprocess.check_call([cxx, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "native",
                                                                              "abi_host_checks.cpp"),
                           "-L", str(tmp_path / "san"), "-lfmm_mi355x_san", "-Wl,-rpath," + str(tmp_path / "san"),
                           "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "host ABI checks passed" in out.stdout
