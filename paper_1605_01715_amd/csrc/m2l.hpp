// M2L translation kernel (V lists) on MFMA.
#pragma once

#include "common.hpp"

namespace fmm {

// ntile workgroups; tile t owns output vectors tile_cols[t][0..ncol) (-1 = unused)
// and the active directions term_dir[e] for e in [tile_term_off[t], tile_term_off[t+1]),
// with source vectors term_src[e][0..ncol) (-1 = none). Vectors are rows of
// r_pad floats (compressed far-field state); out += sum over the tile's terms.
// Block b runs tile (b % 8) * ntile / 8 + b / 8: ntile is a multiple of 8 and
// each eighth of the tiles runs on one XCD.
// FP32 form: mats holds the r_pad x r_pad float32 matrices (one per direction)
// rearranged by m2l_image_mats, and in the source vectors. Split-BF16 form:
// mats_bf and in_bf hold the same data split by m2l_split_mats and
// m2l_split_vecs. zero points to 192 bytes of zeros (16-byte aligned), read
// for columns without a source.
struct M2LLaunch {
    int r_pad = 0, ntile = 0, ncol = 0;
    const int64_t *tile_term_off = nullptr;
    const int32_t *term_dir = nullptr;
    const int32_t *term_src = nullptr;
    const int32_t *tile_cols = nullptr;
    const float *mats = nullptr;
    const float *in = nullptr;
    const uint16_t *mats_bf = nullptr;
    const uint16_t *in_bf = nullptr;
    const void *zero = nullptr;
    const int32_t *piece_slot = nullptr;  // per tile: -1, or the slot of partial it writes instead of adding to out
    float *partial = nullptr;             // [slot][ncol][r_pad]
    float *out = nullptr;
};

int m2l_ncol(int r_pad);
// M2L arithmetic ("form"): 0 float32; 6, 4 or 3 the split-BF16 part products
// (bf16x6 of three parts; bf16x4 and bf16x3 of two parts)
int m2l_form_parts(int form);                  // bfloat16 parts per value of a split form
int m2l_blocks_per_cu(int form, int r_pad);    // workgroups of the kernel that fit on one CU
// cut tiles: out[cols[t][c]] += sum over q < kpieces[t] of partial[slot0[t] + q][c] (q in order)
void m2l_reduce(int r_pad, int ntile, int ncol, const int32_t *cols, const int32_t *slot0, const int32_t *kpieces,
                const float *partial, float *out, hipStream_t s);
// pair tiles: out[targets[t]] += sum over e in [off[t], off[t+1]) of partial row rows[e] (in order)
void m2l_gather(int r_pad, int n, const int32_t *targets, const int32_t *off, const int32_t *rows,
                const float *partial, float *out, hipStream_t s);
bool m2l_supported(int r_pad);  // any multiple of 32 up to 512
void m2l_run(int form, const M2LLaunch &a, hipStream_t s);

// FP32 operands: row-major [ndir][r_pad][r_pad] -> the kernel's chunk order.
void m2l_image_mats(const float *rm, int r_pad, int ndir, float *out, hipStream_t s);
// Split-BF16 operands: each float32 value becomes np = 3 or 2 bfloat16 parts.
size_t m2l_split_mats_elems(int r_pad, int ndir, int np);    // uint16 elements of the split matrices
size_t m2l_split_vecs_elems(int r_pad, int64_t nvec, int np);
void m2l_split_mats(const float *rm, int r_pad, int ndir, int np, uint16_t *out, hipStream_t s);
void m2l_split_vecs(const float *in, int r_pad, int64_t nvec, int np, uint16_t *out, hipStream_t s);
// The three-part splits written out plainly: parts[p][i], p = 0..2, of the values in
// row-major order (which = 0: count vectors of r_pad; which = 1: count
// r_pad x r_pad matrices). Synchronises the stream.
void m2l_split_plain(int which, int r_pad, int64_t count, const float *in, uint16_t *parts, hipStream_t s);

}  // namespace fmm
