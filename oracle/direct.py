"""Direct O(N^2) quadrature sum (float64): the ground truth of every FMM result.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. II.A Eq. sum_fmm, f(r_i) = sum_j K(r_i, r_j) sigma_j, with the
Laplace kernels of the two model problems:
  single layer   K = 1 / (4 pi |x - y|)
  double layer   K = (x - y) . n_y / (4 pi |x - y|^3)     (Eq. fk_integral)
  field          K = (x - y) / (4 pi |x - y|^3)           (Eq. kernel_pol)
Pairs closer than the tolerance radius delta contribute 0 (Sec. III.A.1).

Pins (tests/test_oracle_direct.py): hand-computed two- and three-point sums;
Gauss's law for the double layer (interior -1, exterior 0, principal value
-1/2 on a closed surface); the field of a uniformly charged sphere; the
unit-sphere eigenvalues of the single and double layer for l = 0, 1, 2;
the split of the double layer into three field components (Eq. sum_split);
agreement of the C sum with the numpy twin.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle_direct.so")
_lib = None

FOUR_PI = 4.0 * np.pi


def build():
    """Compile the C direct sum with gcc (OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        lib.oracle_direct_sum.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, d, d,
                                          d, d, d, d, ctypes.c_double, d, d, d, d]
        lib.oracle_direct_sum.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads():
    return int(_load().oracle_num_threads())


def _col(a, k):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)[:, k])


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def direct_sum(trg, src, q=None, dipole=None, delta=1e-5, potential=True, field=False):
    """Float64 direct sum at targets `trg` [nt,3] from sources `src` [ns,3].

    q: [ns] single-layer densities or None; dipole: [ns,3] double-layer
    dipoles m_j = mu_j n_j (already weighted) or None. Returns
    (pot [nt] or None, field [nt,3] or None).
    """
    lib = _load()
    trg = np.asarray(trg, dtype=np.float64)
    src = np.asarray(src, dtype=np.float64)
    nt, ns = len(trg), len(src)
    tx, ty, tz = (_col(trg, k) for k in range(3))
    sx, sy, sz = (_col(src, k) for k in range(3))
    qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
    if dipole is None:
        mx = my = mz = None
    else:
        mx, my, mz = (_col(dipole, k) for k in range(3))
    pot = np.zeros(nt) if potential else None
    if field:
        fx, fy, fz = np.zeros(nt), np.zeros(nt), np.zeros(nt)
    else:
        fx = fy = fz = None
    if nt and ns:
        lib.oracle_direct_sum(nt, _ptr(tx), _ptr(ty), _ptr(tz), ns, _ptr(sx), _ptr(sy), _ptr(sz),
                              _ptr(qq), _ptr(mx), _ptr(my), _ptr(mz), float(delta),
                              _ptr(pot), _ptr(fx), _ptr(fy), _ptr(fz))
    fld = np.stack([fx, fy, fz], axis=1) if field else None
    return pot, fld


def direct_sum_numpy(trg, src, q=None, dipole=None, delta=1e-5):
    """The same sum written with numpy broadcasting (small inputs only)."""
    trg = np.asarray(trg, dtype=np.float64)
    src = np.asarray(src, dtype=np.float64)
    d = trg[:, None, :] - src[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", d, d)
    keep = (r2 > 0.0) & (r2 >= delta * delta)
    r = np.sqrt(np.where(keep, r2, 1.0))
    inv_r = np.where(keep, 1.0 / r, 0.0)
    inv_r3 = inv_r ** 3
    pot = np.zeros(len(trg))
    fld = np.zeros((len(trg), 3))
    if q is not None:
        q = np.asarray(q, dtype=np.float64)
        pot += inv_r @ q
        fld += np.einsum("ij,ijk->ik", inv_r3 * q[None, :], d)
    if dipole is not None:
        m = np.asarray(dipole, dtype=np.float64)
        pot += np.einsum("ij,ijk,jk->i", inv_r3, d, m)
    return pot / FOUR_PI, fld / FOUR_PI


def rel_l2(approx, exact):
    """Relative L2 error ||a - e|| / ||e|| over all entries."""
    a = np.asarray(approx, dtype=np.float64).ravel()
    e = np.asarray(exact, dtype=np.float64).ravel()
    den = np.linalg.norm(e)
    return float(np.linalg.norm(a - e) / den) if den > 0 else float(np.linalg.norm(a))
