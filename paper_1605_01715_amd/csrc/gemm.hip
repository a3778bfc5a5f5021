// Batched box GEMMs in float64 on the CDNA4 matrix cores, a float32 MFMA GEMM
// for the Chebyshev basis changes (below, k_gemm_f32), and float64 helpers
// for the operator precompute.
//
// The upward and downward passes apply small dense matrices to per-box
// vectors: M2M (8 octant matrices), L2L (8 octant matrices), the projections
// of point-generated check potentials onto the compressed basis and the
// check-to-equivalent expansions. They are cheap next to M2L and they feed
// every M2L, so they run in float64 (v_mfma_f64_16x16x4_f64) on float32 data.
// The kernel is target-stationary: a workgroup owns 64 rows of a tile of 32
// output vectors, keeps their accumulator in registers across all terms and
// writes each output once.
//
// Layout (4 waves of 64 lanes): the workgroup (tile, g) computes row blocks
// 4g .. 4g+3 of 16 rows, wave w row block 4g + w against both 16-column
// blocks. Splitting the rows over workgroups keeps the chain of float64
// MFMAs of one tile short: most tree levels have fewer tiles than the chip
// has CUs, so a level costs about one tile's latency (measured 3x faster
// than one workgroup per tile). Matrices are stored in the fragment order of
// the instruction; the source vectors of the tile are staged in LDS and
// shared by the four waves.
#include "gemm.hpp"

#include <algorithm>

namespace fmm {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// The tile's source vectors of one term are staged in LDS 128 k at a time
// (float32, [k][column], 18 KB, so up to eight workgroups share a CU and
// cover each other's staging and barriers), and the matrix fragments of the
// next 16-k chunk are loaded while the current chunk's MFMAs run.
constexpr int kMaxK = 512;
constexpr int kKChunk = 128;          // k rows staged at a time
constexpr int kBStr = kGemmCols + 4;  // floats per k row in LDS

template <int MAXRB>
__global__ __launch_bounds__(kThreads) void k_gemm_f64(GemmLaunch a) {
    constexpr int NCOL = kGemmCols;
    extern __shared__ float Bs[];  // [kKChunk][kBStr]
    __shared__ int32_t cols[NCOL], srcs[NCOL];
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6) + 4 * MAXRB * (int)blockIdx.y;  // first row block
    const int64_t tile = blockIdx.x;
    const int nrb = a.m_pad / 16, K = a.k_pad, nkc = K / 16;
    if (t < NCOL) cols[t] = a.tile_cols[tile * NCOL + t];
    f64x4 acc[MAXRB][2];
#pragma unroll
    for (int i = 0; i < MAXRB; ++i)
        for (int c = 0; c < 2; ++c) acc[i][c] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int term = 0; term < a.nterm; ++term) {
        __syncthreads();
        int mysrc = -1;
        if (t < NCOL) {
            mysrc = a.term_src[(tile * a.nterm + term) * NCOL + t];
            srcs[t] = mysrc;
        }
        if (!__syncthreads_or(mysrc >= 0)) continue;
        const int mat = a.term_mat ? a.term_mat[tile * a.nterm + term] : term;
        const double *M = a.mats + (size_t)mat * a.mat_elems;
        // matrix fragments: av[i][s] for row block w + 4 i, chunk kc
        double av0[MAXRB][4], av1[MAXRB][4];
        auto load_av = [&](double (&av)[MAXRB][4], int kc) {
#pragma unroll
            for (int i = 0; i < MAXRB; ++i) {
                const int rb = min(w + 4 * i, nrb - 1);  // clamped rows are loaded, never used
                const double *ap = M + (((size_t)rb * nkc + kc) * 64 + lane) * 4;
                for (int s = 0; s < 4; ++s) av[i][s] = ap[s];
            }
        };
        // chunk kc against the staged rows lk * 16 .. lk * 16 + 15 of the LDS slice
        auto mma = [&](const double (&av)[MAXRB][4], int lk) {
            double bf[4][2];
            for (int s = 0; s < 4; ++s)
                for (int cb = 0; cb < 2; ++cb)
                    bf[s][cb] = (double)Bs[(lk * 16 + 4 * s + (lane >> 4)) * kBStr + cb * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < MAXRB; ++i) {
                if (w + 4 * i >= nrb) continue;
                for (int s = 0; s < 4; ++s)
                    for (int cb = 0; cb < 2; ++cb)
                        acc[i][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s], bf[s][cb], acc[i][cb], 0, 0, 0);
            }
        };
        for (int k0 = 0; k0 < K; k0 += kKChunk) {
            const int kn = min(kKChunk, K - k0);  // a multiple of 16
            if (k0 > 0) __syncthreads();         // every wave is done with the previous slice
            // stage k0 .. k0 + kn of the 32 source vectors, transposed
            const int kq = kn / 4;
            for (int idx = t; idx < NCOL * kq; idx += kThreads) {
                const int col = idx / kq, k4 = (idx % kq) * 4;
                const int sidx = srcs[col];
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (sidx >= 0) x = *(const float4 *)(a.in + (size_t)sidx * K + k0 + k4);
                Bs[(k4 + 0) * kBStr + col] = x.x;
                Bs[(k4 + 1) * kBStr + col] = x.y;
                Bs[(k4 + 2) * kBStr + col] = x.z;
                Bs[(k4 + 3) * kBStr + col] = x.w;
            }
            __syncthreads();
            const int c0 = k0 / 16, c1 = (k0 + kn) / 16;
            load_av(av0, c0);
            for (int kc = c0; kc < c1; kc += 2) {
                if (kc + 1 < c1) load_av(av1, kc + 1);
                mma(av0, kc - c0);
                if (kc + 1 < c1) {
                    if (kc + 2 < c1) load_av(av0, kc + 2);
                    mma(av1, kc + 1 - c0);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXRB; ++i) {
        const int rb = w + 4 * i;
        if (rb >= nrb) continue;
        for (int cb = 0; cb < 2; ++cb) {
            const int o = cols[cb * 16 + (lane & 15)];
            if (o < 0) continue;
            const double sc = a.col_scale ? a.col_scale[o] : 1.0;
            // f64 16x16 accumulator: element v of lane l is row l/16 + 4 v
            float *op = a.out + (size_t)o * a.m_pad + rb * 16 + (lane >> 4);
            for (int v = 0; v < 4; ++v) {
                float r = (float)(acc[i][cb][v] * sc);
                op[4 * v] = a.accumulate ? op[4 * v] + r : r;
            }
        }
    }
}

__global__ void k_frag_f64(const double *M, int rows, int cols, int m_pad, int k_pad, double *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)m_pad * k_pad) return;
    const int nkc = k_pad / 16;
    int s = (int)(idx % 4);
    int64_t r = idx / 4;
    int lane = (int)(r % 64);
    r /= 64;
    int kc = (int)(r % nkc);
    int rb = (int)(r / nkc);
    int row = rb * 16 + (lane & 15), k = kc * 16 + 4 * s + (lane >> 4);
    out[idx] = (row < rows && k < cols) ? M[(int64_t)row * cols + k] : 0.0;
}

__global__ void k_padded_f32(const double *M, int rows, int cols, int m_pad, int k_pad, float *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)m_pad * k_pad) return;
    int row = (int)(idx / k_pad), k = (int)(idx % k_pad);
    out[idx] = (row < rows && k < cols) ? (float)M[(int64_t)row * cols + k] : 0.f;
}

__global__ void k_laplace_mats(const double *Y, int n, int nb, const double *prm, double *G) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t per = (int64_t)n * n;
    if (idx >= per * nb) return;
    int b = (int)(idx / per);
    int i = (int)((idx % per) / n), j = (int)(idx % n);
    const double *p = prm + 9 * b;
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double x = p[c] + p[3] * Y[3 * i + c];
        double y = p[4 + c] + p[7] * Y[3 * j + c];
        d2 += (x - y) * (x - y);
    }
    G[idx] = p[8] / (kFourPi * sqrt(d2));
}

__global__ __launch_bounds__(256) void k_dgemm(const double *A, size_t sa, const double *B, size_t sb, double *C,
                                              size_t sc, int M, int N, int K) {
    __shared__ double As[16][17], Bsh[16][17];
    const int b = blockIdx.z;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    const double *Ab = A + (size_t)b * sa;
    const double *Bb = B + (size_t)b * sb;
    double acc = 0.0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        As[ty][tx] = (row < M && k0 + tx < K) ? Ab[(size_t)row * K + k0 + tx] : 0.0;
        Bsh[ty][tx] = (k0 + ty < K && col < N) ? Bb[(size_t)(k0 + ty) * N + col] : 0.0;
        __syncthreads();
        for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bsh[k][tx];
        __syncthreads();
    }
    if (row < M && col < N) C[(size_t)b * sc + (size_t)row * N + col] = acc;
}

// One matrix for every column, float32 on the matrix cores
// (v_mfma_f32_32x32x2f32, float32 accumulation): the Chebyshev form's
// compression into the M2L basis and expansion out of it, the two largest
// box GEMMs (every box, 512 x r). One workgroup per tile of 32 columns, so
// the tile's source vectors are read from memory once: they are staged in
// LDS 128 k at a time with coalesced loads (rows of k_pad floats) and shared
// by the waves. Wave w owns the 32-row blocks w, w + NW (MAXRB of them) and
// reads its matrix fragments from global memory in fragment order (every
// load instruction reads 1 KB contiguous), the next chunk's while the
// current chunk's MFMAs run. Lane l supplies row (or column) l % 32 at
// k = 16 (l / 32) + q for MFMA q, so MFMA q contracts k = q and 16 + q of a
// 32-k chunk (a permutation of the k order, the same on both operands).
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kF32Slice = 128;            // k staged per slice
constexpr int kF32BStr = kF32Slice + 4;   // floats per column in LDS

template <int MAXRB>
__global__ __launch_bounds__(512) void k_gemm_f32(int m_pad, int k_pad, const int32_t *tile_cols, const float *Mf,
                                                  const float *in, float *out, const double *col_scale,
                                                  int accumulate, const int8_t *add_col) {
    __shared__ __align__(16) float Bs[kGemmCols * kF32BStr];
    __shared__ int32_t cols[kGemmCols];
    const int t = threadIdx.x, lane = t & 63, c = lane & 31, h = lane >> 5;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nt = blockDim.x, nw = nt >> 6, nrb = m_pad / 32, nkc = k_pad / 32;
    const int64_t tile = blockIdx.x;
    if (t < kGemmCols) cols[t] = tile_cols[tile * kGemmCols + t];
    const float4 *ap[MAXRB];
    bool live[MAXRB];
#pragma unroll
    for (int i = 0; i < MAXRB; ++i) {
        const int rb = w + nw * i;
        live[i] = rb < nrb;  // wave-uniform
        ap[i] = (const float4 *)Mf + (size_t)min(rb, nrb - 1) * nkc * 256 + lane;
    }
    float4 a[2][MAXRB][4];
    auto load_a = [&](int buf, int kc) {
#pragma unroll
        for (int i = 0; i < MAXRB; ++i)
            if (live[i])
#pragma unroll
                for (int f = 0; f < 4; ++f) a[buf][i][f] = ap[i][(size_t)kc * 256 + 64 * f];
    };
    f32x16 acc[MAXRB];
#pragma unroll
    for (int i = 0; i < MAXRB; ++i)
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
    auto mma = [&](int buf, int kl) {  // kl: chunk offset inside the staged slice
        float4 b[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) b[f] = *(const float4 *)&Bs[c * kF32BStr + kl + 16 * h + 4 * f];
#pragma unroll
        for (int i = 0; i < MAXRB; ++i) {
            if (!live[i]) continue;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i][f].x, b[f].x, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i][f].y, b[f].y, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i][f].z, b[f].z, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i][f].w, b[f].w, acc[i], 0, 0, 0);
            }
        }
    };
    load_a(0, 0);
    for (int k0 = 0; k0 < k_pad; k0 += kF32Slice) {
        const int kn = min(kF32Slice, k_pad - k0), kq = kn / 4;  // kn: a multiple of 32
        __syncthreads();  // cols; every wave is done with the previous slice
        for (int idx = t; idx < kGemmCols * kq; idx += nt) {
            const int col = idx / kq, k4 = (idx % kq) * 4;
            const int o = cols[col];
            *(float4 *)&Bs[col * kF32BStr + k4] =
                o >= 0 ? *(const float4 *)(in + (size_t)o * k_pad + k0 + k4) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
        const int c0 = k0 / 32, c1 = c0 + kn / 32;
        for (int kc = c0; kc < c1; kc += 2) {
            if (kc + 1 < nkc) load_a(1, kc + 1);
            mma(0, (kc - c0) * 32);
            if (kc + 1 < c1) {
                if (kc + 2 < nkc) load_a(0, kc + 2);
                mma(1, (kc + 1 - c0) * 32);
            }
        }
    }
    const int o = cols[c];
    if (o < 0) return;
    const float sc = col_scale ? (float)col_scale[o] : 1.f;
    const bool add = accumulate || (add_col && add_col[o]);
#pragma unroll
    for (int i = 0; i < MAXRB; ++i) {
        if (!live[i]) continue;
        // 32x32 accumulator: element v of lane l is row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
        float *op = out + (size_t)o * m_pad + (w + nw * i) * 32 + 4 * h;
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) {
            float4 r = make_float4(acc[i][4 * v4] * sc, acc[i][4 * v4 + 1] * sc, acc[i][4 * v4 + 2] * sc,
                                   acc[i][4 * v4 + 3] * sc);
            float4 *dst = (float4 *)(op + 8 * v4);
            if (add) {
                const float4 old = *dst;
                r.x += old.x;
                r.y += old.y;
                r.z += old.z;
                r.w += old.w;
            }
            *dst = r;
        }
    }
}

// float64 row-major [rows][cols] -> the float32 fragment order of k_gemm_f32:
// out[((rb * nkc + kc) * 4 + f) * 256 + 4 lane + e] = M[32 rb + lane % 32][32 kc + 16 (lane / 32) + 4 f + e]
__global__ void k_frag_f32(const double *M, int rows, int cols, int m_pad, int k_pad, float *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)m_pad * k_pad) return;
    const int nkc = k_pad / 32;
    const int e = (int)(idx % 4), lane = (int)((idx / 4) % 64), f = (int)((idx / 256) % 4);
    const int64_t q = idx / 1024;
    const int kc = (int)(q % nkc), rb = (int)(q / nkc);
    const int row = rb * 32 + (lane & 31), k = kc * 32 + 16 * (lane >> 5) + 4 * f + e;
    out[idx] = (row < rows && k < cols) ? (float)M[(int64_t)row * cols + k] : 0.f;
}

}  // namespace

void box_gemm_f64(const GemmLaunch &a, hipStream_t s) {
    if (a.ntile <= 0 || a.nterm <= 0) return;
    FMM_REQUIRE(a.m_pad % 16 == 0 && a.k_pad % 16 == 0 && a.m_pad <= 512 && a.k_pad <= kMaxK,
                "box_gemm: unsupported size");
    dim3 g((unsigned)a.ntile, (unsigned)((a.m_pad / 16 + 3) / 4)), b(kThreads);  // one row block per wave
    const size_t sh = (size_t)std::min(a.k_pad, kKChunk) * kBStr * sizeof(float);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, sh, s, a); };
    go(k_gemm_f64<1>);
    FMM_HIP(hipGetLastError());
}

void dense_gemm_f32(int m_pad, int k_pad, int ntile, const int32_t *tile_cols, const float *M, const float *in,
                    float *out, const double *col_scale, int accumulate, hipStream_t s, const int8_t *add_col) {
    if (ntile <= 0) return;
    FMM_REQUIRE(m_pad > 0 && k_pad > 0 && m_pad % 32 == 0 && k_pad % 32 == 0 && m_pad <= 512,
                "dense_gemm_f32: unsupported size");
    const int nrb = m_pad / 32, nw = std::min(nrb, 8);  // waves per workgroup; each owns ceil(nrb / nw) row blocks
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)ntile), dim3(64 * nw), 0, s, m_pad, k_pad, tile_cols, M, in, out,
                           col_scale, accumulate, add_col);
    };
    if (nrb <= 8)
        go(k_gemm_f32<1>);
    else
        go(k_gemm_f32<2>);
    FMM_HIP(hipGetLastError());
}

void to_frag_f32(const double *M, int rows, int cols, int m_pad, int k_pad, float *out, hipStream_t s) {
    FMM_REQUIRE(m_pad % 32 == 0 && k_pad % 32 == 0, "to_frag_f32: sizes must be multiples of 32");
    int64_t total = (int64_t)m_pad * k_pad;
    hipLaunchKernelGGL(k_frag_f32, dim3(grid_for(total, 256)), dim3(256), 0, s, M, rows, cols, m_pad, k_pad, out);
    FMM_HIP(hipGetLastError());
}

void to_frag_f64(const double *M, int rows, int cols, int m_pad, int k_pad, double *out, hipStream_t s) {
    int64_t total = (int64_t)m_pad * k_pad;
    hipLaunchKernelGGL(k_frag_f64, dim3(grid_for(total, 256)), dim3(256), 0, s, M, rows, cols, m_pad, k_pad, out);
    FMM_HIP(hipGetLastError());
}

void to_padded_f32(const double *M, int rows, int cols, int m_pad, int k_pad, float *out, hipStream_t s) {
    int64_t total = (int64_t)m_pad * k_pad;
    hipLaunchKernelGGL(k_padded_f32, dim3(grid_for(total, 256)), dim3(256), 0, s, M, rows, cols, m_pad, k_pad,
                       out);
    FMM_HIP(hipGetLastError());
}

void build_laplace_mats(const double *Y, int n, int nb, const double *params, double *G, hipStream_t s) {
    int64_t total = (int64_t)n * n * nb;
    hipLaunchKernelGGL(k_laplace_mats, dim3(grid_for(total, 256)), dim3(256), 0, s, Y, n, nb, params, G);
    FMM_HIP(hipGetLastError());
}

void dgemm_batched(const double *A, size_t sa, const double *B, size_t sb, double *C, size_t sc, int M, int N,
                   int K, int nb, hipStream_t s) {
    dim3 g((N + 15) / 16, (M + 15) / 16, nb);
    hipLaunchKernelGGL(k_dgemm, g, dim3(256), 0, s, A, sa, B, sb, C, sc, M, N, K);
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
