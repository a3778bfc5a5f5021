// M2L: the far-field box-to-box translation over the V lists, on MFMA.
//
// For every target box B and every V-list partner A (the children of
// parent(B)'s neighbours that are not B's neighbours), the compressed downward
// state of B gains M_d * u_A, where u_A is A's compressed upward state (r
// values) and M_d the float64-built r x r translation of the offset d = A - B
// (316 possible offsets). This is the kernel-independent counterpart of the
// paper's interpolation-based far field (Sec. III.A.1 Eq. p2m, K_r between
// interpolation nodes), grouped by translation direction into dense GEMMs.
//
// Blocking. A workgroup (8 waves) owns a tile of 128 target boxes of one
// octant; each wave takes one 32-column block and one half of the rows, and
// the workgroup keeps the r_pad x 128
// accumulator in registers across all directions, so every output is written
// once. Each step of the tile is one (direction, 32-wide k-chunk): the 32
// columns of M_d for that chunk are loaded once per workgroup as float32,
// split into the operand format and staged in LDS (double-buffered when it
// fits), and the waves multiply them against their own 32 source columns,
// which each lane loads straight from HBM into registers. With
// 32x32 MFMA tiles each staged matrix element is read from LDS once per 32
// columns. The next step's loads are issued before the current step's MFMAs.
// Tiles are ordered so that consecutive tiles run on the same XCD and share
// its L2 for the gathered source vectors.
//
// The k index inside a chunk is permuted so that every lane's operand is a
// run of consecutive values (16-byte loads); the dot product is the same.
//
// Forms: FP32 (v_mfma_f32_32x32x2_f32) and split-BF16 (both operands split
// into three bfloat16 parts, six products hh hm mh mm hl lh accumulated in
// float32 with v_mfma_f32_32x32x16_bf16).
#include "m2l.hpp"

namespace fmm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));  // plain vector: promotable to registers
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;  // 8 waves: 4 column blocks of 32 x 2 row halves
constexpr int kCols = 128;
constexpr int KC = 32;         // k per step

__device__ inline uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
    h = f2bf(x);
    float r1 = x - bf2f(h);
    m = f2bf(r1);
    l = f2bf(r1 - bf2f(m));
}

// LDS bytes of one staged A chunk (r_pad rows x 32 k)
template <int NRB, bool BF16>
constexpr int a_chunk_bytes() {
    return BF16 ? NRB * 32 * KC * 2 * 3 : NRB * 32 * KC * 4;
}

// A chunk in LDS, fragment order:
//   BF16 (32x32x16): part p, row block rb, k-half h (16 k each), lane, 8 slots;
//                    element (row, k) -> lane = row % 32 + 32 * ((k % 16) / 8), slot = k % 8
//   FP32 (32x32x2):  row block rb, lane, 16 slots;
//                    element (row, k) -> lane = row % 32 + 32 * (k / 16), slot = k % 16
template <int NRB, bool BF16, int NBUF>
__global__ __launch_bounds__(kThreads) void k_m2l(M2LLaunch a) {
    constexpr int NF4 = NRB * 32 * KC / 4;                   // float4 per chunk
    constexpr int NLOAD = (NF4 + kThreads - 1) / kThreads;   // float4 per thread per chunk
    constexpr int PART = NRB * 2 * 64 * 8;                   // bf16 elements of one part
    constexpr int RBH = (NRB + 1) / 2;                       // row blocks per row half
    extern __shared__ __align__(16) unsigned char lds[];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int hf = lane >> 5, r32 = lane & 31;
    const int cblk = w & 3, rhalf = w >> 2;                  // wave -> (column block, row half)
    const int rb0 = rhalf * RBH;
    const int nrb = (rb0 + RBH <= NRB) ? RBH : NRB - rb0;    // row blocks of this wave

    // XCD-aware tile order: blocks are dealt to the 8 XCDs round-robin, so
    // block b runs on XCD b % 8. Each XCD gets a contiguous range of tiles
    // (neighbouring target boxes share source vectors in that XCD's L2).
    // XCD x receives cnt(x) blocks and owns tiles [start(x), start(x) + cnt(x)),
    // a bijection of [0, ntile).
    int tile;
    {
        const int nb = gridDim.x, b = blockIdx.x;
        const int per = (nb + 7) / 8;
        const int rem = nb - (per - 1) * 8;
        const int x = b % 8, k = b / 8;
        const int cnt = (x < rem) ? per : per - 1;
        const int start = (x < rem) ? x * per : rem * per + (x - rem) * (per - 1);
        if (k >= cnt) return;
        tile = start + k;
    }
    const int64_t toff = a.tile_term_off[tile];
    const int nact = (int)(a.tile_term_off[tile + 1] - toff);
    constexpr int nkc = (NRB * 32) / KC;
    const int nsteps = nact * nkc;
    const int my_col = 32 * cblk + r32;
    const int outv = a.tile_cols[(int64_t)tile * kCols + my_col];

    f32x16 acc[RBH];
#pragma unroll
    for (int i = 0; i < RBH; ++i)
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;

    f32x4 areg[NLOAD];
    f32x4 breg[4];
    bool bnext_live = false;

    auto load_step = [&](int s) {
        const int e = s / nkc, kc = s % nkc;
        const int dir = a.term_dir[toff + e];
        const float *M = a.mats + (size_t)dir * (NRB * 32) * (NRB * 32);
        // every areg[j] is written unconditionally (a clamped index on the
        // ragged last pass; store_a drops it) so the array stays in registers
#pragma unroll
        for (int j = 0; j < NLOAD; ++j) {
            const int f = min(t + kThreads * j, NF4 - 1);  // float4 index within the chunk
            const int row = f >> 3, k4 = (f & 7) * 4;
            areg[j] = *(const f32x4 *)(M + (size_t)row * (NRB * 32) + kc * KC + k4);
        }
        const int sv = a.term_src[(toff + e) * kCols + my_col];
        if (sv >= 0) {
            const float *p = a.in + (size_t)sv * (NRB * 32) + kc * KC;
            if (BF16) {  // k = 16 h2 + 8 hf + v for the two 16-k halves
                breg[0] = *(const f32x4 *)(p + 8 * hf);
                breg[1] = *(const f32x4 *)(p + 8 * hf + 4);
                breg[2] = *(const f32x4 *)(p + 16 + 8 * hf);
                breg[3] = *(const f32x4 *)(p + 16 + 8 * hf + 4);
            } else {     // k = 16 hf + q
                for (int q = 0; q < 4; ++q) breg[q] = *(const f32x4 *)(p + 16 * hf + 4 * q);
            }
        } else {
            for (int q = 0; q < 4; ++q) breg[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        bnext_live = __ballot(sv >= 0) != 0;  // wave-uniform: some column of this wave has a source
    };
    auto store_a = [&](int buf) {
        unsigned char *base = lds + buf * a_chunk_bytes<NRB, BF16>();
#pragma unroll
        for (int j = 0; j < NLOAD; ++j) {
            const int f = t + kThreads * j;
            if (NF4 % kThreads != 0 && f >= NF4) continue;
            const int row = f >> 3, k4 = (f & 7) * 4;
            const int rb = row >> 5;
            if (BF16) {
                const int h2 = k4 >> 4, fl = (row & 31) + 32 * ((k4 & 15) >> 3), slot = k4 & 7;
                const float v[4] = {areg[j].x, areg[j].y, areg[j].z, areg[j].w};
                u16x4 hh, mm, ll;
                for (int q = 0; q < 4; ++q) {
                    uint16_t x0, x1, x2;
                    split3(v[q], x0, x1, x2);
                    hh[q] = x0;
                    mm[q] = x1;
                    ll[q] = x2;
                }
                uint16_t *p = (uint16_t *)base;
                const int off = ((rb * 2 + h2) * 64 + fl) * 8 + slot;
                *(u16x4 *)(p + off) = hh;
                *(u16x4 *)(p + PART + off) = mm;
                *(u16x4 *)(p + 2 * PART + off) = ll;
            } else {
                const int fl = (row & 31) + 32 * (k4 >> 4), slot = k4 & 15;
                *(f32x4 *)((float *)base + (rb * 64 + fl) * 16 + slot) = areg[j];
            }
        }
    };

    if (nsteps > 0) {
        load_step(0);
        store_a(0);
    }
    for (int s = 0; s < nsteps; ++s) {
        const int buf = NBUF == 2 ? (s & 1) : 0;
        const bool live = bnext_live;
        // consume this step's B registers before the prefetch overwrites them
        bf16x8 bh[2], bm[2], bl[2];
        float bv[16];
        {
            const float v[16] = {breg[0].x, breg[0].y, breg[0].z, breg[0].w, breg[1].x, breg[1].y,
                                 breg[1].z, breg[1].w, breg[2].x, breg[2].y, breg[2].z, breg[2].w,
                                 breg[3].x, breg[3].y, breg[3].z, breg[3].w};
            if (BF16) {
                for (int h2 = 0; h2 < 2; ++h2) {
                    u16x8 x0, x1, x2;
                    for (int q = 0; q < 8; ++q) {
                        uint16_t a0, a1, a2;
                        split3(v[8 * h2 + q], a0, a1, a2);
                        x0[q] = a0;
                        x1[q] = a1;
                        x2[q] = a2;
                    }
                    bh[h2] = __builtin_bit_cast(bf16x8, x0);
                    bm[h2] = __builtin_bit_cast(bf16x8, x1);
                    bl[h2] = __builtin_bit_cast(bf16x8, x2);
                }
            } else {
                for (int q = 0; q < 16; ++q) bv[q] = v[q];
            }
        }
        __syncthreads();  // A(s) visible in LDS
        if (s + 1 < nsteps) load_step(s + 1);
        const unsigned char *base = lds + buf * a_chunk_bytes<NRB, BF16>();
        if (live) {
            if (BF16) {
                const uint16_t *p = (const uint16_t *)base;
#pragma unroll
                for (int i = 0; i < RBH; ++i) {
                    if (i >= nrb) continue;  // static index i keeps acc in registers
                    const int rb = rb0 + i;
                    f32x16 c = acc[i];
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int off = ((rb * 2 + h2) * 64 + lane) * 8;
                        const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const u16x8 *)(p + off));
                        const bf16x8 am = __builtin_bit_cast(bf16x8, *(const u16x8 *)(p + PART + off));
                        const bf16x8 al = __builtin_bit_cast(bf16x8, *(const u16x8 *)(p + 2 * PART + off));
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[h2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[h2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm[h2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh[h2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm[h2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[h2], c, 0, 0, 0);
                    }
                    acc[i] = c;
                }
            } else {
                const float *p = (const float *)base;
#pragma unroll
                for (int i = 0; i < RBH; ++i) {
                    if (i >= nrb) continue;
                    const int rb = rb0 + i;
                    const f32x4 *ap = (const f32x4 *)(p + (rb * 64 + lane) * 16);
                    const f32x4 a0 = ap[0], a1 = ap[1], a2 = ap[2], a3 = ap[3];
                    const float av[16] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w,
                                          a2.x, a2.y, a2.z, a2.w, a3.x, a3.y, a3.z, a3.w};
                    f32x16 c = acc[i];
                    for (int q = 0; q < 16; ++q) c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q], bv[q], c, 0, 0, 0);
                    acc[i] = c;
                }
            }
        }
        if (s + 1 < nsteps) {
            if (NBUF == 1) __syncthreads();  // every wave is done with the single buffer
            store_a(NBUF == 2 ? ((s + 1) & 1) : 0);
        }
    }
    // write back: element v of lane l in a 32x32 block is row 8 (v / 4) + 4 (l / 32) + v % 4
    if (outv >= 0) {
#pragma unroll
        for (int i = 0; i < RBH; ++i) {
            if (i >= nrb) continue;
            const int rb = rb0 + i;
            for (int v4 = 0; v4 < 4; ++v4) {
                float4 *op = (float4 *)(a.out + (size_t)outv * (NRB * 32) + rb * 32 + 8 * v4 + 4 * hf);
                float4 cur = *op;
                cur.x += acc[i][4 * v4];
                cur.y += acc[i][4 * v4 + 1];
                cur.z += acc[i][4 * v4 + 2];
                cur.w += acc[i][4 * v4 + 3];
                *op = cur;
            }
        }
    }
}

template <int NRB, bool BF16>
void launch(const M2LLaunch &a, hipStream_t s) {
    constexpr int bytes1 = a_chunk_bytes<NRB, BF16>();
    constexpr int NBUF = 2 * bytes1 <= 160 * 1024 ? 2 : 1;
    constexpr int bytes = NBUF * bytes1;
    static_assert(bytes <= 160 * 1024, "A chunk does not fit in LDS");
    auto k = k_m2l<NRB, BF16, NBUF>;
    FMM_HIP(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    hipLaunchKernelGGL(k, dim3(a.ntile), dim3(kThreads), bytes, s, a);
    FMM_HIP(hipGetLastError());
}

template <bool BF16, int NRB = 1>
void dispatch(int nrb, const M2LLaunch &a, hipStream_t s) {
    if constexpr (NRB <= 16) {
        if (nrb == NRB)
            launch<NRB, BF16>(a, s);
        else
            dispatch<BF16, NRB + 1>(nrb, a, s);
    } else {
        throw Error(FMM_ERR_ARG, "m2l: unsupported state size");
    }
}

}  // namespace

int m2l_ncol(int r_pad) {
    (void)r_pad;
    return kCols;
}

bool m2l_supported(int r_pad) { return r_pad > 0 && r_pad % 32 == 0 && r_pad <= 512; }

void m2l_run(bool bf16, const M2LLaunch &a, hipStream_t s) {
    if (a.ntile <= 0) return;
    FMM_REQUIRE(m2l_supported(a.r_pad), "m2l: unsupported state size");
    FMM_REQUIRE(a.ncol == m2l_ncol(a.r_pad), "m2l: tile width mismatch");
    if (bf16)
        dispatch<true>(a.r_pad / 32, a, s);
    else
        dispatch<false>(a.r_pad / 32, a, s);
}

}  // namespace fmm
