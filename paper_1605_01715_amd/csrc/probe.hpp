// Issue-rate probe kernels (a measurement utility).
#pragma once

#include "common.hpp"

namespace fmm {

// kind 0: float32 FMA chains, 1: reciprocal square root chains, 2: 12 FMAs
// and one reciprocal square root per chain step, 3: 32-bit integer add and
// exclusive-or chains, 4: bfloat16 matrix products from registers.
// nthreads a positive multiple of 256; out [nthreads].
void issue_probe(int kind, int64_t nthreads, int iters, float *out, hipStream_t s);
// instructions of the chains per step: wave64 VALU per lane (kinds 0-3),
// MFMA per wave (kind 4)
int64_t issue_probe_instr(int kind);

}  // namespace fmm
