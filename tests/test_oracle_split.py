"""Pins of oracle/split.py: the bfloat16 split, the split GEMM error bound,
TwoSum and the cascaded compensated sum, each against what the arithmetic
fixes (brute force over every bfloat16 value, exact rational arithmetic,
hand-worked values, an independent library conversion)."""

import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import split as S

HERE = os.path.dirname(os.path.abspath(__file__))


def _f32(bits):
    return np.array([bits], np.uint32).view(np.float32)[0]


def _random_f32(n, seed, lo=-30, hi=30):
    return W.float32_bits(n, seed, lo, hi)


def _all_bf16_finite():
    h = np.arange(1 << 16, dtype=np.uint32)
    v = (h << 16).view(np.float32)
    keep = np.isfinite(v)
    h, v = h[keep], v[keep].astype(np.float64)
    order = np.lexsort((h, v))
    return v[order], h[order]


def test_bf16_round_is_the_nearest_bfloat16_ties_to_even():
    """Brute force: for each input, the nearest of all finite bfloat16 values;
    on a tie, the one whose last fraction bit is 0."""
    vals, pats = _all_bf16_finite()
    x = _random_f32(3000, seed=11)
    # exact ties: x halfway between two neighbouring bfloat16 values
    ties = ((_random_f32(500, seed=12).view(np.uint32) & 0xFFFF0000) | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, np.float32([0.0, -0.0, 1.0, -1.0])])
    got = S.bf16_round(x)
    for xi, gi in zip(x.astype(np.float64), got):
        k = int(np.searchsorted(vals, xi))
        cands = [j for j in (k - 1, k, k + 1) if 0 <= j < len(vals)]
        best = min(abs(vals[j] - xi) for j in cands)
        near = [j for j in cands if abs(vals[j] - xi) == best]
        if xi == 0.0:
            assert (int(gi) & 0x7FFF) == 0
            continue
        if len(near) == 2 and vals[near[0]] != vals[near[1]]:
            want = [pats[j] for j in near if (pats[j] & 1) == 0]
        else:
            want = [pats[j] for j in near]
        assert int(gi) in [int(w) for w in want], (xi, hex(int(gi)), [hex(int(w)) for w in want])


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    x = np.concatenate([_random_f32(20000, seed=13, lo=-120, hi=120),
                        ((_random_f32(2000, seed=14).view(np.uint32) & 0xFFFF0000) | 0x8000).view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(S.bf16_round(x), ref)


def test_hand_worked_splits():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "bf16_split.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 6
    for xs, *ps in rows:
        parts = S.split(np.array([_f32(int(xs, 16))]), 3)
        assert [int(p[0]) for p in parts] == [int(p, 16) for p in ps], xs


@pytest.mark.parametrize("parts", [1, 2, 3])
def test_split_parts_are_bf16_and_reconstruct_within_u_to_the_k(parts):
    x = _random_f32(4000, seed=15, lo=-40, hi=40)
    pv = S.split(x, parts)
    for p in pv:
        # a part is a bfloat16 value: as float32, its low 16 bits are zero
        assert np.all((S.bf16_to_f32(p).view(np.uint32) & 0xFFFF) == 0)
    for i in range(0, len(x), 97):
        xi = Fraction(float(x[i]))
        s = sum(Fraction(float(S.bf16_to_f32(p[i]))) for p in pv)
        assert abs(xi - s) <= Fraction(1, 2 ** (8 * parts)) * abs(xi)
        # each part is bounded by u^i (1 + u) |x|
        for k, p in enumerate(pv):
            assert abs(Fraction(float(S.bf16_to_f32(p[i])))) <= Fraction(257, 256) * Fraction(1, 256 ** k) * abs(xi)
    # three parts hold all 24 significant bits of most float32 values exactly
    exact = np.sum(S.split_values(x, 3), axis=0) == x.astype(np.float64)
    assert exact.mean() > 0.9


def test_two_sum_is_error_free():
    x = _random_f32(3000, seed=16, lo=-20, hi=20)
    y = _random_f32(3000, seed=17, lo=-20, hi=20)
    # hand cases: a tiny addend lost in s and kept in t; a tie in the sum; cancellation
    hand = [(1.0, 2.0 ** -30, 1.0, 2.0 ** -30), (2.0 ** 24, 1.0, 2.0 ** 24, 1.0),
            (1.0 + 2.0 ** -23, -1.0, 2.0 ** -23, 0.0)]
    for a, b, s_want, t_want in hand:
        s, t = S.two_sum(a, b)
        assert (float(s), float(t)) == (s_want, t_want)
    for a, b in zip(x, y):
        s, t = S.two_sum(a, b)
        assert s == np.float32(a + b)
        assert Fraction(float(s)) + Fraction(float(t)) == Fraction(float(a)) + Fraction(float(b))


def test_sum2_within_its_bound():
    rng = np.random.default_rng(18)
    for n in (10, 200, 2000):
        v = (rng.standard_normal(n) * 10.0 ** rng.integers(-3, 4, n)).astype(np.float32)
        exact = sum(Fraction(float(a)) for a in v)
        got = S.sum2(v)
        err = abs(Fraction(float(got)) - exact)
        assert err <= S.U_F32 * abs(exact) + Fraction(S.sum2_bound(v))
        # plain float32 accumulation is much worse on these ill-scaled sums
    v = np.float32([1.0, 2.0 ** -25, 2.0 ** -25, 2.0 ** -25, 2.0 ** -25])
    assert float(S.sum2(v)) == 1.0 + 2.0 ** -23
    acc = np.float32(0)
    for a in v:
        acc = np.float32(acc + a)
    assert float(acc) == 1.0


@pytest.mark.parametrize("scheme", ["bf16x3", "bf16x4", "bf16x6"])
def test_split_gemm_within_bound_of_float64_gemm(scheme):
    rng = np.random.default_rng(19)
    a = rng.standard_normal((96, 160)).astype(np.float32)
    b = rng.standard_normal((160, 64)).astype(np.float32)
    ref = a.astype(np.float64) @ b.astype(np.float64)
    scale = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    got = S.split_gemm(a, b, scheme)
    ratio = np.max(np.abs(got - ref) / scale)
    assert ratio <= S.gemm_bound(scheme)


def test_split_gemm_keeps_exactly_the_scheme_products():
    """Operands whose float32 values have only 16 significant bits are exactly
    two bfloat16 parts, x = h + m. Then bf16x4 and bf16x6 (which keep every
    product of two nonzero parts) return A B exactly, and bf16x3 returns
    A B - A_m B_m: a closed form that any dropped, doubled or misplaced part
    product would break."""
    rng = np.random.default_rng(20)
    a = (rng.standard_normal((48, 160)).astype(np.float32).view(np.uint32) & 0xFFFFFF00).view(np.float32)
    b = (rng.standard_normal((160, 40)).astype(np.float32).view(np.uint32) & 0xFFFFFF00).view(np.float32)
    for x in (a, b):
        h, m, l = S.split_values(x, 3)
        assert np.all(l == 0.0) and np.all(h + m == x.astype(np.float64))
    ref = a.astype(np.float64) @ b.astype(np.float64)
    scale = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    for scheme in ("bf16x4", "bf16x6"):
        assert np.max(np.abs(S.split_gemm(a, b, scheme) - ref) / scale) < 1e-14
    am, bm = S.split_values(a, 2)[1], S.split_values(b, 2)[1]
    mm = am @ bm
    assert np.max(np.abs(mm) / scale) > 1e-7   # the term bf16x3 drops is not negligible
    assert np.max(np.abs(S.split_gemm(a, b, "bf16x3") - (ref - mm)) / scale) < 1e-14


def test_split_gemm_bounds_are_ordered_and_float32_accumulation_dominates_x6():
    assert S.gemm_bound("bf16x6") < S.gemm_bound("bf16x4") < S.gemm_bound("bf16x3")
    assert S.gemm_bound("bf16x6") < 2.0 ** -21
    assert 2.0 ** -16 < S.gemm_bound("bf16x3") < 2.0 ** -13
    # over an inner dimension of 160, the float32 sum of six products per term
    # is the larger part of the bf16x6 bound
    total = S.gemm_bound("bf16x6", inner=160, f32_accumulate=True)
    assert total - S.gemm_bound("bf16x6") > S.gemm_bound("bf16x6")
