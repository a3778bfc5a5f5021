"""The split-BF16 M2L operands on the GPU against oracle/split.py, bit for bit.

The library splits the far-field state at every apply and the translation
matrices when it builds operators (three bfloat16 parts each, the bf16x6
scheme of Henry, Tang and Heinecke). fmm_split_bf16 runs that same device
code on seeded synthetic float32 values, including exact bfloat16 ties and
values across a wide exponent range; every part must equal the oracle's."""

import numpy as np
import pytest

import workloads as W
from oracle import split as S

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which,r_pad,count", [(0, 160, 1000), (0, 32, 7), (1, 64, 5), (1, 160, 3)])
def test_gpu_split_parts_equal_the_oracle(which, r_pad, count):
    import paper_1605_01715_amd as F

    n = count * r_pad * (r_pad if which == 1 else 1)
    say(f"test_gpu_split_parts_equal_the_oracle: which={which} r_pad={r_pad} count={count} values={n}")
    x = W.float32_bits(n, seed=21 + which, lo=-60, hi=60, ties=n // 8)
    got = F.fmm_split_bf16(which, r_pad, dev(x)).cpu().numpy().view(np.uint16)
    want = np.stack(S.split(x, 3))
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} parts differ, first at (part, index) {tuple(bad[0])}"


def test_gpu_split_of_the_empty_set_and_bad_arguments():
    import torch

    import paper_1605_01715_amd as F

    lib = F._lib.load()
    assert lib.fmm_split_bf16(0, 160, 0, None, None, None) == F.FMM_OK
    buf = torch.zeros(160, device="cuda:0")
    out = torch.zeros(3 * 160, dtype=torch.int16, device="cuda:0")
    assert lib.fmm_split_bf16(0, 100, 1, buf.data_ptr(), out.data_ptr(), None) == F.FMM_ERR_ARG
    assert lib.fmm_split_bf16(2, 160, 1, buf.data_ptr(), out.data_ptr(), None) == F.FMM_ERR_ARG
    assert lib.fmm_split_bf16(0, 160, 1, None, out.data_ptr(), None) == F.FMM_ERR_ARG
