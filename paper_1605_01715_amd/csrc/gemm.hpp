// Target-stationary batched box GEMMs (float64 MFMA) and float64 helpers.
#pragma once

#include "common.hpp"

namespace fmm {

// One launch: `ntile` workgroups. Tile t owns up to 32 output vectors
// (tile_cols[t][c], -1 = unused) and accumulates, over `nterm` terms,
//     out[col] (+)= col_scale[col] * sum_term  M[mat(t, term)] * in[src(t, term, col)]
// with src = -1 meaning "no contribution". Input vectors are rows of k_pad
// floats, output vectors rows of m_pad floats; matrices are m_pad x k_pad
// float64 in the fragment layout of to_frag_f64. A term whose sources are
// all -1 in a tile is skipped. Arithmetic is float64 (inputs and outputs are
// float32).
struct GemmLaunch {
    int m_pad = 0, k_pad = 0;
    int ntile = 0;
    int nterm = 0;
    const int32_t *tile_cols = nullptr;  // [ntile][32]
    const int32_t *term_src = nullptr;   // [ntile][nterm][32]
    const int32_t *term_mat = nullptr;   // [ntile][nterm], or NULL: matrix index = term
    const double *mats = nullptr;
    size_t mat_elems = 0;                // m_pad * k_pad
    const float *in = nullptr;
    float *out = nullptr;
    const double *col_scale = nullptr;   // per output vector, or NULL
    int accumulate = 0;
};

constexpr int kGemmCols = 32;
void box_gemm_f64(const GemmLaunch &a, hipStream_t s);

// One float32 matrix M (m_pad x k_pad, zero-padded, in the fragment order of
// to_frag_f32) for every column, float32 MFMA arithmetic: for tile t and
// c < 32 with o = tile_cols[t][c] >= 0,
//     out[o] (+)= col_scale[o] * M * in[o]
// (in rows of k_pad floats, out rows of m_pad floats; col_scale may be NULL,
// accumulate adds to out, and so does a nonzero add_col[o] for column o).
// m_pad and k_pad are multiples of 32, m_pad <= 512.
void dense_gemm_f32(int m_pad, int k_pad, int ntile, const int32_t *tile_cols, const float *M, const float *in,
                    float *out, const double *col_scale, int accumulate, hipStream_t s,
                    const int8_t *add_col = nullptr);
// float64 row-major M [rows][cols] -> float32 fragment order for dense_gemm_f32, zero-padded to m_pad x k_pad.
void to_frag_f32(const double *M, int rows, int cols, int m_pad, int k_pad, float *out, hipStream_t s);

// Layout conversions of a dense float64 matrix M [rows][cols] (row-major):
// fragment order for box_gemm_f64, zero-padded to m_pad x k_pad; and a plain
// row-major float32 copy zero-padded to m_pad x k_pad.
void to_frag_f64(const double *M, int rows, int cols, int m_pad, int k_pad, double *out, hipStream_t s);
void to_padded_f32(const double *M, int rows, int cols, int m_pad, int k_pad, float *out, hipStream_t s);

// G[b][i][j] = scale_b / (4 pi |(ox_b + rx_b Y_i) - (oy_b + ry_b Y_j)|), b < nb.
void build_laplace_mats(const double *Y, int n, int nb, const double *params /* [nb][9] */, double *G,
                        hipStream_t s);
// C[b] = A[b] * B[b]: M x K times K x N, row-major; a batch stride of 0 shares the operand.
void dgemm_batched(const double *A, size_t sa, const double *B, size_t sb, double *C, size_t sc, int M, int N,
                   int K, int nb, hipStream_t s);

}  // namespace fmm
