// Target-stationary batched box GEMMs on the matrix cores.
#pragma once

#include "common.hpp"

namespace fmm {

enum class GemmPrec { F32, BF16X6, F64 };

// One launch: `ntile` workgroups. Tile t owns up to ncol() output vectors
// (tile_cols[t][c], -1 = unused) and accumulates, over `nterm` terms,
//     out[col] (+)= col_scale[col] * sum_term  M[mat(t, term)] * in[src(t, term, col)]
// with src = -1 meaning "no contribution". Vectors are rows of n_pad floats;
// matrices are n_pad x n_pad in the fragment layout of the precision (see
// gemm.hip). A term whose sources are all -1 in a tile is skipped.
struct GemmLaunch {
    int n_pad = 0;
    int ntile = 0;
    int nterm = 0;
    const int32_t *tile_cols = nullptr;  // [ntile][ncol]
    const int32_t *term_src = nullptr;   // [ntile][nterm][ncol]
    const int32_t *term_mat = nullptr;   // [ntile][nterm], or NULL: matrix index = term
    const void *mats = nullptr;          // F32: float, BF16X6: 3 uint16 parts per matrix, F64: double
    size_t mat_elems = 0;                // elements of one matrix (one part for BF16X6)
    const float *in = nullptr;
    float *out = nullptr;
    const double *col_scale = nullptr;   // per output vector, or NULL
    int accumulate = 0;
};

int gemm_ncol(GemmPrec p);
void box_gemm(GemmPrec prec, const GemmLaunch &a, hipStream_t s);

// Fragment-layout conversion of a dense float64 matrix M [n][n] (row-major,
// leading dimension n) into the n_pad x n_pad layout of each precision.
size_t frag_elems(GemmPrec p, int n_pad);
void to_frag_f32(const double *M, int n, int n_pad, float *out, hipStream_t s);
void to_frag_bf16x3(const double *M, int n, int n_pad, uint16_t *out /* 3 parts */, hipStream_t s);
void to_frag_f64(const double *M, int n, int n_pad, double *out, hipStream_t s);

// Float64 helpers for the operator precompute.
// G[b][i][j] = scale_b / (4 pi |(ox_b + rx_b Y_i) - (oy_b + ry_b Y_j)|), b < nb.
void build_laplace_mats(const double *Y, int n, int nb, const double *params /* [nb][9] */, double *G,
                        hipStream_t s);
// C[b] = A[b] * B for nb matrices of n x n (row-major).
void dgemm_batched(const double *A, const double *B, double *C, int n, int nb, hipStream_t s);

}  // namespace fmm
