// Batched box-to-box GEMMs on the CDNA4 matrix cores (MFMA).
//
// Every translation of the upward and downward passes is a dense matrix
// applied to a per-box vector of n_s surface values: M2M (8 octant matrices),
// M2L (316 direction matrices), L2L (8 octant matrices) and the
// check-to-equivalent maps. The kernel is target-stationary: a workgroup owns
// a tile of output boxes, keeps their n_pad x ncol accumulator in registers and
// streams the matrices and the gathered source vectors of every term through
// it, so each output vector is written once per launch.
//
// Layout (4 waves of 64 lanes): wave w computes row blocks w, w+4, ... of 16
// rows against all column blocks of 16. Matrices are stored in the fragment
// order of the instruction so every lane loads its A fragment with one or two
// 16-byte loads; the B fragments (the source vectors of the tile) are staged
// in LDS once per k-chunk and shared by the four waves.
//
// Precisions:
//   F32     v_mfma_f32_16x16x4_f32
//   BF16X6  both operands split into three bfloat16 parts x = h + m + l; the
//           products hh + hm + mh + mm + hl + lh are accumulated in float32
//           with v_mfma_f32_16x16x32_bf16 (the bf16x6 scheme of Henry, Tang and
//           Heinecke, 2019)
//   F64     v_mfma_f64_16x16x4_f64, float32 in/out (check-to-equivalent maps)
#include "gemm.hpp"

namespace fmm {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

__device__ inline uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- float32
template <int MAXRB>
__global__ __launch_bounds__(kThreads) void k_gemm_f32(GemmLaunch a) {
    constexpr int NCOL = 64, KC = 32, BSTR = 80;
    __shared__ float Bs[KC * BSTR];
    __shared__ int32_t cols[NCOL], srcs[NCOL];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile = blockIdx.x;
    const int nrb = a.n_pad / 16, nkc = a.n_pad / KC;
    if (t < NCOL) cols[t] = a.tile_cols[tile * NCOL + t];
    f32x4 acc[MAXRB][4];
    for (int i = 0; i < MAXRB; ++i)
        for (int c = 0; c < 4; ++c) acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int term = 0; term < a.nterm; ++term) {
        __syncthreads();
        int mysrc = -1;
        if (t < NCOL) {
            mysrc = a.term_src[(tile * a.nterm + term) * NCOL + t];
            srcs[t] = mysrc;
        }
        if (!__syncthreads_or(mysrc >= 0)) continue;
        const int mat = a.term_mat ? a.term_mat[tile * a.nterm + term] : term;
        const float *M = (const float *)a.mats + (size_t)mat * a.mat_elems;
        for (int kc = 0; kc < nkc; ++kc) {
            {
                const int col = t >> 2, k8 = (t & 3) * 8;
                const int sidx = srcs[col];
                float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0;
                if (sidx >= 0) {
                    const float4 *p = (const float4 *)(a.in + (size_t)sidx * a.n_pad + kc * KC + k8);
                    x0 = p[0];
                    x1 = p[1];
                }
                const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                for (int i = 0; i < 8; ++i) Bs[(k8 + i) * BSTR + col] = v[i];
            }
            __syncthreads();
            float bf[8][4];
            for (int s = 0; s < 8; ++s)
                for (int cb = 0; cb < 4; ++cb) bf[s][cb] = Bs[(4 * s + (lane >> 4)) * BSTR + cb * 16 + (lane & 15)];
            for (int i = 0; i < MAXRB; ++i) {
                const int rb = w + 4 * i;
                if (rb >= nrb) break;
                const float4 *ap = (const float4 *)(M + (((size_t)rb * nkc + kc) * 64 + lane) * 8);
                const float4 a0 = ap[0], a1 = ap[1];
                const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                for (int s = 0; s < 8; ++s)
                    for (int cb = 0; cb < 4; ++cb)
                        acc[i][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bf[s][cb], acc[i][cb], 0, 0, 0);
            }
            __syncthreads();
        }
    }
    for (int i = 0; i < MAXRB; ++i) {
        const int rb = w + 4 * i;
        if (rb >= nrb) break;
        for (int cb = 0; cb < 4; ++cb) {
            const int o = cols[cb * 16 + (lane & 15)];
            if (o < 0) continue;
            const float sc = a.col_scale ? (float)a.col_scale[o] : 1.f;
            float *op = a.out + (size_t)o * a.n_pad + rb * 16 + 4 * (lane >> 4);
            for (int v = 0; v < 4; ++v) {
                float r = acc[i][cb][v] * sc;
                op[v] = a.accumulate ? op[v] + r : r;
            }
        }
    }
}

// ---------------------------------------------------------------- bf16 x6
template <int MAXRB>
__global__ __launch_bounds__(kThreads) void k_gemm_bf16x6(GemmLaunch a) {
    constexpr int NCOL = 64, KC = 32, BSTR = 40;  // bf16 elements per LDS column (80 bytes)
    __shared__ uint16_t Bs[3][NCOL * BSTR];
    __shared__ int32_t cols[NCOL], srcs[NCOL];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile = blockIdx.x;
    const int nrb = a.n_pad / 16, nkc = a.n_pad / KC;
    if (t < NCOL) cols[t] = a.tile_cols[tile * NCOL + t];
    f32x4 acc[MAXRB][4];
    for (int i = 0; i < MAXRB; ++i)
        for (int c = 0; c < 4; ++c) acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int term = 0; term < a.nterm; ++term) {
        __syncthreads();
        int mysrc = -1;
        if (t < NCOL) {
            mysrc = a.term_src[(tile * a.nterm + term) * NCOL + t];
            srcs[t] = mysrc;
        }
        if (!__syncthreads_or(mysrc >= 0)) continue;
        const int mat = a.term_mat ? a.term_mat[tile * a.nterm + term] : term;
        const uint16_t *M = (const uint16_t *)a.mats + (size_t)mat * 3 * a.mat_elems;
        for (int kc = 0; kc < nkc; ++kc) {
            {
                const int col = t >> 2, k8 = (t & 3) * 8;
                const int sidx = srcs[col];
                float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0;
                if (sidx >= 0) {
                    const float4 *p = (const float4 *)(a.in + (size_t)sidx * a.n_pad + kc * KC + k8);
                    x0 = p[0];
                    x1 = p[1];
                }
                const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                u16x8 h, m, l;
                for (int i = 0; i < 8; ++i) {
                    uint16_t hh = f2bf(v[i]);
                    float r1 = v[i] - bf2f(hh);
                    uint16_t mm = f2bf(r1);
                    float r2 = r1 - bf2f(mm);
                    h[i] = hh;
                    m[i] = mm;
                    l[i] = f2bf(r2);
                }
                *(u16x8 *)&Bs[0][col * BSTR + k8] = h;
                *(u16x8 *)&Bs[1][col * BSTR + k8] = m;
                *(u16x8 *)&Bs[2][col * BSTR + k8] = l;
            }
            __syncthreads();
            bf16x8 bfr[3][4];
            for (int p = 0; p < 3; ++p)
                for (int cb = 0; cb < 4; ++cb) {
                    u16x8 raw = *(const u16x8 *)&Bs[p][(cb * 16 + (lane & 15)) * BSTR + 8 * (lane >> 4)];
                    bfr[p][cb] = __builtin_bit_cast(bf16x8, raw);
                }
            for (int i = 0; i < MAXRB; ++i) {
                const int rb = w + 4 * i;
                if (rb >= nrb) break;
                const size_t fo = (((size_t)rb * nkc + kc) * 64 + lane) * 8;
                const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const u16x8 *)(M + fo));
                const bf16x8 am = __builtin_bit_cast(bf16x8, *(const u16x8 *)(M + a.mat_elems + fo));
                const bf16x8 al = __builtin_bit_cast(bf16x8, *(const u16x8 *)(M + 2 * a.mat_elems + fo));
                for (int cb = 0; cb < 4; ++cb) {
                    f32x4 c = acc[i][cb];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bfr[0][cb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bfr[2][cb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bfr[1][cb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bfr[0][cb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bfr[1][cb], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bfr[0][cb], c, 0, 0, 0);
                    acc[i][cb] = c;
                }
            }
            __syncthreads();
        }
    }
    for (int i = 0; i < MAXRB; ++i) {
        const int rb = w + 4 * i;
        if (rb >= nrb) break;
        for (int cb = 0; cb < 4; ++cb) {
            const int o = cols[cb * 16 + (lane & 15)];
            if (o < 0) continue;
            const float sc = a.col_scale ? (float)a.col_scale[o] : 1.f;
            float *op = a.out + (size_t)o * a.n_pad + rb * 16 + 4 * (lane >> 4);
            for (int v = 0; v < 4; ++v) {
                float r = acc[i][cb][v] * sc;
                op[v] = a.accumulate ? op[v] + r : r;
            }
        }
    }
}

// ---------------------------------------------------------------- float64
template <int MAXRB>
__global__ __launch_bounds__(kThreads) void k_gemm_f64(GemmLaunch a) {
    constexpr int NCOL = 32, KC = 16, BSTR = 48;
    __shared__ double Bs[KC * BSTR];
    __shared__ int32_t cols[NCOL], srcs[NCOL];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile = blockIdx.x;
    const int nrb = a.n_pad / 16, nkc = a.n_pad / KC;
    if (t < NCOL) cols[t] = a.tile_cols[tile * NCOL + t];
    f64x4 acc[MAXRB][2];
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
        const double *M = (const double *)a.mats + (size_t)mat * a.mat_elems;
        for (int kc = 0; kc < nkc; ++kc) {
            {
                const int col = t >> 3, k2 = (t & 7) * 2;
                const int sidx = srcs[col];
                float2 x = make_float2(0.f, 0.f);
                if (sidx >= 0) x = *(const float2 *)(a.in + (size_t)sidx * a.n_pad + kc * KC + k2);
                Bs[k2 * BSTR + col] = (double)x.x;
                Bs[(k2 + 1) * BSTR + col] = (double)x.y;
            }
            __syncthreads();
            double bf[4][2];
            for (int s = 0; s < 4; ++s)
                for (int cb = 0; cb < 2; ++cb) bf[s][cb] = Bs[(4 * s + (lane >> 4)) * BSTR + cb * 16 + (lane & 15)];
            for (int i = 0; i < MAXRB; ++i) {
                const int rb = w + 4 * i;
                if (rb >= nrb) break;
                const double *ap = M + (((size_t)rb * nkc + kc) * 64 + lane) * 4;
                const double av[4] = {ap[0], ap[1], ap[2], ap[3]};
                for (int s = 0; s < 4; ++s)
                    for (int cb = 0; cb < 2; ++cb)
                        acc[i][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bf[s][cb], acc[i][cb], 0, 0, 0);
            }
            __syncthreads();
        }
    }
    for (int i = 0; i < MAXRB; ++i) {
        const int rb = w + 4 * i;
        if (rb >= nrb) break;
        for (int cb = 0; cb < 2; ++cb) {
            const int o = cols[cb * 16 + (lane & 15)];
            if (o < 0) continue;
            const double sc = a.col_scale ? a.col_scale[o] : 1.0;
            // f64 16x16 accumulator: element v of lane l is row l/16 + 4 v
            float *op = a.out + (size_t)o * a.n_pad + rb * 16 + (lane >> 4);
            for (int v = 0; v < 4; ++v) {
                float r = (float)(acc[i][cb][v] * sc);
                op[4 * v] = a.accumulate ? op[4 * v] + r : r;
            }
        }
    }
}

template <template <int> class K>
struct Dummy {};

#define FMM_DISPATCH(KERNEL, a, s)                                                               \
    do {                                                                                         \
        int nrb_ = (a).n_pad / 16;                                                               \
        int per_ = (nrb_ + 3) / 4;                                                               \
        dim3 g_((unsigned)(a).ntile), b_(kThreads);                                              \
        if (per_ <= 2) hipLaunchKernelGGL(KERNEL<2>, g_, b_, 0, s, a);                           \
        else if (per_ <= 4) hipLaunchKernelGGL(KERNEL<4>, g_, b_, 0, s, a);                      \
        else if (per_ <= 6) hipLaunchKernelGGL(KERNEL<6>, g_, b_, 0, s, a);                      \
        else hipLaunchKernelGGL(KERNEL<8>, g_, b_, 0, s, a);                                     \
    } while (0)

// ---------------------------------------------------------------- layouts
__global__ void k_frag_f32(const double *M, int n, int n_pad, float *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t total = (int64_t)n_pad * n_pad;
    if (idx >= total) return;
    const int nkc = n_pad / 32;
    int s = (int)(idx % 8);
    int64_t r = idx / 8;
    int lane = (int)(r % 64);
    r /= 64;
    int kc = (int)(r % nkc);
    int rb = (int)(r / nkc);
    int row = rb * 16 + (lane & 15), k = kc * 32 + 4 * s + (lane >> 4);
    out[idx] = (row < n && k < n) ? (float)M[(int64_t)row * n + k] : 0.f;
}

__global__ void k_frag_bf16x3(const double *M, int n, int n_pad, uint16_t *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t total = (int64_t)n_pad * n_pad;
    if (idx >= total) return;
    const int nkc = n_pad / 32;
    int v = (int)(idx % 8);
    int64_t r = idx / 8;
    int lane = (int)(r % 64);
    r /= 64;
    int kc = (int)(r % nkc);
    int rb = (int)(r / nkc);
    int row = rb * 16 + (lane & 15), k = kc * 32 + 8 * (lane >> 4) + v;
    double x = (row < n && k < n) ? M[(int64_t)row * n + k] : 0.0;
    // three-way bfloat16 split of the float64 value, round to nearest even
    uint16_t part[3];
    double rem = x;
    for (int p = 0; p < 3; ++p) {
        float f = (float)rem;
        uint16_t h = f2bf(f);
        part[p] = h;
        rem = rem - (double)bf2f(h);
    }
    out[idx] = part[0];
    out[total + idx] = part[1];
    out[2 * total + idx] = part[2];
}

__global__ void k_frag_f64(const double *M, int n, int n_pad, double *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t total = (int64_t)n_pad * n_pad;
    if (idx >= total) return;
    const int nkc = n_pad / 16;
    int s = (int)(idx % 4);
    int64_t r = idx / 4;
    int lane = (int)(r % 64);
    r /= 64;
    int kc = (int)(r % nkc);
    int rb = (int)(r / nkc);
    int row = rb * 16 + (lane & 15), k = kc * 16 + 4 * s + (lane >> 4);
    out[idx] = (row < n && k < n) ? M[(int64_t)row * n + k] : 0.0;
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

__global__ __launch_bounds__(256) void k_dgemm(const double *A, const double *B, double *C, int n) {
    __shared__ double As[16][17], Bsh[16][17];
    const int b = blockIdx.z;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    const double *Ab = A + (size_t)b * n * n;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += 16) {
        As[ty][tx] = (row < n && k0 + tx < n) ? Ab[(size_t)row * n + k0 + tx] : 0.0;
        Bsh[ty][tx] = (k0 + ty < n && col < n) ? B[(size_t)(k0 + ty) * n + col] : 0.0;
        __syncthreads();
        for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bsh[k][tx];
        __syncthreads();
    }
    if (row < n && col < n) C[(size_t)b * n * n + (size_t)row * n + col] = acc;
}

}  // namespace

int gemm_ncol(GemmPrec p) { return p == GemmPrec::F64 ? 32 : 64; }

size_t frag_elems(GemmPrec p, int n_pad) {
    (void)p;
    return (size_t)n_pad * n_pad;
}

void box_gemm(GemmPrec prec, const GemmLaunch &a, hipStream_t s) {
    if (a.ntile <= 0 || a.nterm <= 0) return;
    FMM_REQUIRE(a.n_pad % 32 == 0 && a.n_pad <= 512, "box_gemm: unsupported surface size");
    switch (prec) {
    case GemmPrec::F32: FMM_DISPATCH(k_gemm_f32, a, s); break;
    case GemmPrec::BF16X6: FMM_DISPATCH(k_gemm_bf16x6, a, s); break;
    case GemmPrec::F64: FMM_DISPATCH(k_gemm_f64, a, s); break;
    }
    FMM_HIP(hipGetLastError());
}

void to_frag_f32(const double *M, int n, int n_pad, float *out, hipStream_t s) {
    int64_t total = (int64_t)n_pad * n_pad;
    hipLaunchKernelGGL(k_frag_f32, dim3(grid_for(total, 256)), dim3(256), 0, s, M, n, n_pad, out);
    FMM_HIP(hipGetLastError());
}
void to_frag_bf16x3(const double *M, int n, int n_pad, uint16_t *out, hipStream_t s) {
    int64_t total = (int64_t)n_pad * n_pad;
    hipLaunchKernelGGL(k_frag_bf16x3, dim3(grid_for(total, 256)), dim3(256), 0, s, M, n, n_pad, out);
    FMM_HIP(hipGetLastError());
}
void to_frag_f64(const double *M, int n, int n_pad, double *out, hipStream_t s) {
    int64_t total = (int64_t)n_pad * n_pad;
    hipLaunchKernelGGL(k_frag_f64, dim3(grid_for(total, 256)), dim3(256), 0, s, M, n, n_pad, out);
    FMM_HIP(hipGetLastError());
}

void build_laplace_mats(const double *Y, int n, int nb, const double *params, double *G, hipStream_t s) {
    int64_t total = (int64_t)n * n * nb;
    hipLaunchKernelGGL(k_laplace_mats, dim3(grid_for(total, 256)), dim3(256), 0, s, Y, n, nb, params, G);
    FMM_HIP(hipGetLastError());
}

void dgemm_batched(const double *A, const double *B, double *C, int n, int nb, hipStream_t s) {
    dim3 g((n + 15) / 16, (n + 15) / 16, nb);
    hipLaunchKernelGGL(k_dgemm, g, dim3(256), 0, s, A, B, C, n);
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
