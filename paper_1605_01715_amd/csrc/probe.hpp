// Issue-rate probe kernels (a measurement utility).
#pragma once

#include "common.hpp"

namespace fmm {

// kind 0: float32 FMA chains, 1: reciprocal square root chains, 2: 12 FMAs
// and one reciprocal square root per chain step, 3: 32-bit integer add and
// exclusive-or chains. nthreads a positive multiple of 256; out [nthreads].
void issue_probe(int kind, int64_t nthreads, int iters, float *out, hipStream_t s);
// wave64 VALU instructions of the chains per lane and step
int64_t issue_probe_instr(int kind);

}  // namespace fmm
