"""The issue-rate probes of the library (a measurement utility): every lane
runs the chains its kind names, so each output equals the same chains run on
the host (float32 arithmetic to a relative 1e-5, the reciprocal square root
being the hardware approximation; the integer chains and the exact bfloat16
matrix products bit for bit), the instruction count is the documented one,
and bad arguments are refused before any launch."""

import numpy as np
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu

A, B = np.float32(0.999), np.float32(1e-3)
IA, IB = np.uint32(0x9E3779B9), np.uint32(0x85EBCA6B)


def _host(kind, nthreads, iters):
    if kind == 4:  # 4 accumulators x 16 elements per lane, each gaining 16 x 1.0 x 0.5 per step
        return np.full(nthreads, 512.0 * iters, np.float32)
    t = (np.arange(nthreads) % 256).astype(np.float32)
    if kind == 3:
        acc = [(np.arange(nthreads) % 256).astype(np.uint64) * 2654435761 + i for i in range(8)]
        acc = [(a & 0xFFFFFFFF).astype(np.uint32) for a in acc]
        for _ in range(iters):
            acc = [(a + IA) ^ IB for a in acc]
        s = np.zeros(nthreads, np.uint32)
        for a in acc:
            s ^= a
        return s.astype(np.float32)
    nc = 8 if kind == 2 else 16
    acc = [(t * np.float32(1e-3) + np.float32(i) + np.float32(0 if kind == 0 else 1)).astype(np.float64)
           for i in range(nc)]
    for _ in range(iters):
        if kind in (0, 2):
            for _r in range(12 if kind == 2 else 1):
                acc = [a * float(A) + float(B) for a in acc]
        if kind in (1, 2):
            acc = [1.0 / np.sqrt(a) for a in acc]
    s = np.full(nthreads, float(A) + float(B) if kind == 1 else 0.0)
    for a in acc:
        s = s + a
    return s


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_issue_probe_runs_its_chains(kind):
    import torch

    import paper_1605_01715_amd as F

    nthreads, iters = 512, 4
    say(f"test_issue_probe_runs_its_chains: kind={kind} nthreads={nthreads} iters={iters}")
    out = torch.full((nthreads,), float("nan"), device="cuda:0")
    instr = F.fmm_issue_probe(kind, out, iters)
    torch.cuda.synchronize()
    assert instr == iters * {2: 104, 4: 4}.get(kind, 16)
    got = out.cpu().numpy()
    want = _host(kind, nthreads, iters)
    if kind in (3, 4):
        assert np.array_equal(got, want)
    else:
        np.testing.assert_allclose(got, want, rtol=1e-5)


def test_issue_probe_refuses_bad_arguments():
    import torch

    import paper_1605_01715_amd as F

    lib = F._lib.load()
    out = torch.zeros(256, device="cuda:0")
    p = out.data_ptr()
    assert lib.fmm_issue_probe(5, 256, 1, p, None, None) == F.FMM_ERR_ARG
    assert lib.fmm_issue_probe(-1, 256, 1, p, None, None) == F.FMM_ERR_ARG
    assert lib.fmm_issue_probe(0, 100, 1, p, None, None) == F.FMM_ERR_ARG
    assert lib.fmm_issue_probe(0, 0, 1, p, None, None) == F.FMM_ERR_ARG
    assert lib.fmm_issue_probe(0, 256, 0, p, None, None) == F.FMM_ERR_ARG
    assert lib.fmm_issue_probe(0, 256, 1, None, None, None) == F.FMM_ERR_ARG
    assert lib.fmm_issue_probe(0, 256, 1, p, None, None) == F.FMM_OK
    torch.cuda.synchronize()
