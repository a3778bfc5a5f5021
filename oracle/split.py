"""Split-precision arithmetic: bfloat16 splits, split GEMMs and TwoSum.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes no floating-point precision for its matvec (Sec. III states
the problem and Sec. IV the tolerances only). The GPU path computes the
far-field translations (the M2L step of Sec. III.A.1, Eq. p2m) on bfloat16
matrix cores with both operands split into bfloat16 parts, and folds the
near-field sums (Eq. sum_fmm) into compensated accumulators. This module
restates the published methods those rest on, so that the GPU's parts can be
checked bit for bit and the error of a split product can be bounded:

  bf16_round  float32 -> bfloat16 (1 sign, 8 exponent, 7 stored fraction
              bits: 8 significant bits), IEEE 754 roundTiesToEven. Written
              here as a choice between the two bfloat16 neighbours of x, the
              one toward zero (x with its low 16 bits cleared) and the next
              one away from zero, by exact comparison of the two distances.
  split       x = p_0 + p_1 + ... + p_{k-1} + r_k with p_0 = bf16(x) and
              p_i = bf16(r_i), r_i = x - p_0 - ... - p_{i-1}. Each r_i is exact
              in float32 (p_i is r_i rounded at its 8th significant bit, so
              r_i - p_i needs at most 16 more significant bits), and with the
              bfloat16 unit roundoff u = 2^-8, |r_k| <= u^k |x| and
              |p_i| <= u^i (1 + u) |x| (for x and its parts in the normal
              range). This is the multi-part splitting of Henry, Tang and
              Heinecke, "Leveraging the bfloat16 artificial intelligence
              datatype for higher-precision computations" (ARITH 2019).
  SCHEMES     which part products a split product keeps:
                bf16x3  two parts, hh + hl + lh            (Henry et al.)
                bf16x4  two parts, all four products
                bf16x6  three parts, hh + hm + mh + mm + hl + lh  (Henry et al.)
  split_gemm  C = sum over the kept (i, j) of A_i B_j, the products formed
              exactly (a product of two bfloat16 values has at most 16
              significant bits, exact in float64) and summed in float64.
  gemm_bound  gamma_S with |C_split - A B| <= gamma_S * (|A| |B|) elementwise:
              x y - sum_S p_i q_j = (x s + r y - r s) + sum_{(i,j) not in S}
              p_i q_j, with r, s the split residuals of x, y, so
              gamma_S = 2 u^k + u^(2k) + (1 + u)^2 sum_{(i,j) not in S} u^(i+j).
              bf16x6: about 4 u^3 = 2^-22; bf16x3: about 3 u^2; bf16x4: 2 u^2.
              An accumulation in float32 (as on the matrix cores) adds the
              textbook gamma_n = n u32 / (1 - n u32), u32 = 2^-24, over the
              n = (kept products) x (inner dimension) terms.
  two_sum     Knuth's TwoSum (TAOCP vol. 2, Sec. 4.2.2): s = fl(a + b) and
              t = (a - (s - (s - a))) + (b - (s - a)) satisfy a + b = s + t
              exactly, in float32, for any finite a, b without overflow.
  sum2        the cascaded sum of Ogita, Rump and Oishi ("Accurate sum and
              dot product", SIAM J. Sci. Comput. 26, 2005, Algorithm 4.4):
              TwoSum along the values, the rounding errors summed in float32
              and added at the end; |result - sum| <= u32 |sum| +
              gamma_{n-1}^2 sum |x_i|.

Pins (tests/test_oracle_split.py): bf16_round against brute force over all
finite bfloat16 values (nearest, ties to the even fraction) and against
torch's float32 -> bfloat16 conversion; hand-worked values
(tests/golden/bf16_split.txt); every part bfloat16-representable and the
residual within u^k |x|, checked in exact rational arithmetic; two_sum exact
in rational arithmetic; sum2 within its bound of the exact rational sum;
split_gemm within gemm_bound of a float64 GEMM and, for the two-part schemes,
not far inside it (a dropped or doubled term would show).
"""

from __future__ import annotations

import numpy as np

U_BF16 = 2.0 ** -8   # unit roundoff of bfloat16 (8 significant bits)
U_F32 = 2.0 ** -24   # unit roundoff of float32

SCHEMES = {
    "bf16x3": (2, ((0, 0), (0, 1), (1, 0))),
    "bf16x4": (2, ((0, 0), (0, 1), (1, 0), (1, 1))),
    "bf16x6": (3, ((0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0))),
}


def _bits(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32)


def bf16_round(x):
    """float32 -> bfloat16, round to nearest, ties to even. Returns the
    bfloat16 bit patterns (uint16). Finite inputs whose rounding does not
    overflow."""
    x = np.asarray(x, dtype=np.float32)
    b = _bits(x).astype(np.uint64)
    toward = b & 0xFFFF0000                       # the neighbour toward zero (same sign)
    away = toward + 0x10000                       # the next bfloat16 value away from zero
    lo = toward.astype(np.uint32).view(np.float32).astype(np.float64)
    hi = away.astype(np.uint32).view(np.float32).astype(np.float64)
    xv = x.astype(np.float64)
    d_lo = np.abs(xv - lo)                        # both exact in float64
    d_hi = np.abs(hi - xv)
    lo_even = ((toward >> 16) & 1) == 0
    pick_away = (d_hi < d_lo) | ((d_hi == d_lo) & ~lo_even)
    out = np.where(pick_away, away, toward) >> 16
    return out.astype(np.uint16)


def bf16_to_f32(h):
    """bfloat16 bit patterns -> float32 (exact)."""
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32)


def split(x, parts):
    """The bfloat16 parts of float32 x: list of `parts` uint16 arrays
    (p_0 = bf16(x), p_i = bf16 of the float32 residual)."""
    r = np.asarray(x, dtype=np.float32).copy()
    out = []
    for _ in range(parts):
        p = bf16_round(r)
        out.append(p)
        r = (r - bf16_to_f32(p)).astype(np.float32)  # exact (see the module docstring)
    return out


def split_values(x, parts):
    """The parts as float64 values (exact), shape [parts, ...]."""
    return np.stack([bf16_to_f32(p).astype(np.float64) for p in split(x, parts)])


def split_gemm(a, b, scheme):
    """sum over the scheme's kept part pairs (i, j) of A_i @ B_j, float64.
    a: [m, k] float32, b: [k, n] float32."""
    parts, pairs = SCHEMES[scheme]
    ap = split_values(a, parts)
    bp = split_values(b, parts)
    c = np.zeros((a.shape[0], b.shape[1]))
    for i, j in pairs:
        c += ap[i] @ bp[j]
    return c


def gemm_bound(scheme, inner=0, f32_accumulate=False):
    """gamma with |C_split - A B| <= gamma (|A| |B|), elementwise (module
    docstring); with f32_accumulate, plus gamma_n of a float32 sum of the
    kept products over an inner dimension of `inner`."""
    parts, pairs = SCHEMES[scheme]
    u = U_BF16
    kept = set(pairs)
    dropped = sum(u ** (i + j) for i in range(parts) for j in range(parts) if (i, j) not in kept)
    g = 2 * u ** parts + u ** (2 * parts) + (1 + u) ** 2 * dropped
    if f32_accumulate:
        n = len(pairs) * inner
        g += n * U_F32 / (1 - n * U_F32)
    return g


def two_sum(a, b):
    """Knuth's TwoSum in float32: (s, t) with s = fl(a + b), a + b = s + t."""
    a = np.float32(a)
    b = np.float32(b)
    with np.errstate(over="ignore"):
        s = np.float32(a + b)
        bb = np.float32(s - a)
        aa = np.float32(s - bb)
        t = np.float32(np.float32(a - aa) + np.float32(b - bb))
    return s, t


def sum2(values):
    """Cascaded compensated sum in float32 (Ogita, Rump and Oishi)."""
    s = np.float32(0.0)
    c = np.float32(0.0)
    for v in np.asarray(values, dtype=np.float32):
        s, t = two_sum(s, v)
        c = np.float32(c + t)
    return np.float32(s + c)


def sum2_bound(values):
    """|sum2(values) - exact| <= u32 |exact| + gamma_{n-1}^2 sum |x| (the
    exact sum is not known here: the caller passes it to the comparison)."""
    n = len(values)
    g = (n - 1) * U_F32 / (1 - (n - 1) * U_F32)
    return g * g * float(np.sum(np.abs(np.asarray(values, dtype=np.float64))))
