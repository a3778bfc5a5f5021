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
// the workgroup keeps the r_pad x 128 accumulator in registers across all
// directions, so every output is written once. Each step of the tile is one
// (direction, 32-wide k-chunk) or two: the chunk of M_d and the tile's 128
// source chunks are copied to LDS (double-buffered) and every wave multiplies
// them. With 32x32 MFMA tiles each staged matrix element is read from LDS once
// per 32 columns. The next step's loads are issued before the current step's
// MFMAs. Tiles are dealt to the XCDs so that each XCD runs a contiguous range.
//
// The k index inside a chunk is permuted so that every lane's operand is a
// run of consecutive values (16-byte loads); the dot product is the same.
//
// Forms:
//   FP32        v_mfma_f32_32x32x2_f32; the float32 matrix chunk is
//               rearranged into fragment order on its way to LDS.
//   split-BF16  both operands split into three bfloat16 parts x = h + m + l;
//               the six products hh hm mh mm hl lh are accumulated in float32
//               with v_mfma_f32_32x32x16_bf16 (the bf16x6 scheme of Henry,
//               Tang and Heinecke, 2019). The split is done once, outside the
//               inner loop: the matrices when the operators are built (stored
//               chunk by chunk in the exact LDS image), the source vectors by
//               one pass over the upward state per apply. The inner loop is
//               then only copies and MFMAs.
#include "m2l.hpp"

namespace fmm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));  // plain vectors: promotable to registers
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 512;  // 8 waves: 4 column blocks of 32 x 2 row halves
constexpr int kCols = 128;
constexpr int KC = 32;         // k per step

// float32 -> bfloat16, round to nearest even (finite inputs)
__device__ inline uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// x = h + m + l up to 2^-24 |x| (each residual is exact in float32)
__device__ inline void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
    h = f2bf(x);
    float r1 = x - bf2f(h);
    m = f2bf(r1);
    l = f2bf(r1 - bf2f(m));
}

// One staged A chunk (r_pad rows x 32 k) in LDS, fragment order:
//   BF16 (32x32x16): part p, row block rb, k-half h (16 k each), lane, 8 slots;
//                    element (row, k) -> lane = row % 32 + 32 * ((k % 16) / 8), slot = k % 8
//   FP32 (32x32x2):  row block rb, lane, 16 slots;
//                    element (row, k) -> lane = row % 32 + 32 * (k / 16), slot = k % 16
template <int NRB, bool BF16>
constexpr int a_chunk_bytes() {
    return BF16 ? NRB * 32 * KC * 2 * 3 : NRB * 32 * KC * 4;
}

// Split-BF16 source vector layout: per vector, per 32-k chunk, 3 parts of 32
// bfloat16 (192 bytes, so one lane's three parts of a run share cache lines).
__host__ __device__ constexpr int64_t vec_bf_stride(int r_pad) { return 3 * (int64_t)r_pad; }

// XCD-aware tile order: blocks are dealt to the 8 XCDs round-robin, so
// block b runs on XCD b % 8. Each XCD gets a contiguous range of tiles
// (neighbouring target boxes share source vectors in that XCD's L2).
// XCD x receives cnt(x) blocks and owns tiles [start(x), start(x) + cnt(x)),
// a bijection of [0, ntile). Returns -1 for blocks beyond it.
__device__ inline int xcd_tile(int nb, int b) {
    const int per = (nb + 7) / 8;
    const int rem = nb - (per - 1) * 8;
    const int x = b % 8, k = b / 8;
    const int cnt = (x < rem) ? per : per - 1;
    const int start = (x < rem) ? x * per : rem * per + (x - rem) * (per - 1);
    return k < cnt ? start + k : -1;
}

// A step covers GPS consecutive 32-k chunks ("granules") of one direction
// (two when both fit in LDS double-buffered: more MFMA work between two
// workgroup barriers; the last step of a direction holds fewer granules when
// GPS does not divide r_pad / 32). Both operands are staged through LDS: each
// step the workgroup copies the matrix granule and the 128 columns' source
// granules with contiguous 16-byte pieces (12 or 8 lanes per column, measured
// 18% faster than every lane gathering its own column), then every wave reads
// its fragments from LDS. The column stride of the source granule in LDS is
// padded by 16 bytes so the operand reads of 16 consecutive lanes hit
// distinct banks.
template <bool BF16>
constexpr int b_col_stride() { return BF16 ? 192 + 16 : 128 + 16; }

template <int NRB, bool BF16, int NBUF, int GPS>
__global__ __launch_bounds__(kThreads) void k_m2l(M2LLaunch a) {
    constexpr int RP = NRB * 32;
    constexpr int CHUNK = a_chunk_bytes<NRB, BF16>();        // bytes of one A granule in LDS
    constexpr int NF4 = CHUNK / 16;
    constexpr int NLOAD = (NF4 + kThreads - 1) / kThreads;
    constexpr int PART = NRB * 2 * 64 * 8;
    constexpr int RBH = (NRB + 1) / 2;
    constexpr int NGR = RP / KC;
    constexpr int NST = (NGR + GPS - 1) / GPS;
    constexpr int PPC = BF16 ? 12 : 8;                       // 16-byte pieces per column granule
    constexpr int NBL = kCols * PPC / kThreads;              // pieces per thread per granule
    constexpr int BSTR = b_col_stride<BF16>();
    constexpr int BCH = kCols * BSTR;                        // bytes of one B granule in LDS
    static_assert(kCols * PPC % kThreads == 0, "B pieces must divide evenly");
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *ldsA = lds;
    unsigned char *ldsB = lds + NBUF * GPS * CHUNK;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int hf = lane >> 5, r32 = lane & 31;
    const int cblk = w & 3, rhalf = w >> 2;
    const int rb0 = rhalf * RBH;
    const int nrb = (rb0 + RBH <= NRB) ? RBH : NRB - rb0;

    const int tile = xcd_tile(gridDim.x, blockIdx.x);
    if (tile < 0) return;
    const int64_t toff = a.tile_term_off[tile];
    const int nact = (int)(a.tile_term_off[tile + 1] - toff);
    const int nsteps = nact * NST;
    const int my_col = 32 * cblk + r32;
    const int outv = a.tile_cols[(int64_t)tile * kCols + my_col];
    __shared__ int32_t s_dir[kNumDirs];
    for (int i = t; i < nact; i += kThreads) s_dir[i] = a.term_dir[toff + i];
    // B stream: this thread's loader columns and their source indices for the
    // direction being loaded and the next one; each lane's own column index
    // only decides whether its wave has any source (skips dead MFMAs)
    int a_e = 0, a_st = 0, b_e = 0, b_st = 0;
    int cur_sv[NBL], nxt_sv[NBL], cur_own = -1, nxt_own = -1;
#pragma unroll
    for (int j = 0; j < NBL; ++j) cur_sv[j] = nxt_sv[j] = -1;
    auto fetch_src = [&](int e, int (&sv)[NBL], int &own) {
        const int64_t row = (toff + e) * kCols;
#pragma unroll
        for (int j = 0; j < NBL; ++j) sv[j] = a.term_src[row + (t + kThreads * j) / PPC];
        own = a.term_src[row + my_col];
    };
    if (nact > 0) {
        fetch_src(0, cur_sv, cur_own);
        fetch_src(min(1, nact - 1), nxt_sv, nxt_own);
    }
    __syncthreads();  // s_dir

    f32x16 acc[RBH];
#pragma unroll
    for (int i = 0; i < RBH; ++i)
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;

    u32x4 ar[GPS][NLOAD];
    u32x4 br[GPS][NBL];
    uint32_t bkeep[NBL];
    bool live_next = false;
    auto granules = [&](int st) { return min(GPS, NGR - st * GPS); };

    auto load_a = [&]() {
        const int dir = __builtin_amdgcn_readfirstlane(s_dir[min(a_e, nact - 1)]);
#pragma unroll
        for (int g = 0; g < GPS; ++g) {
            const int kc = a_st * GPS + (a_st * GPS + g < NGR ? g : 0);
#pragma unroll
            for (int j = 0; j < NLOAD; ++j) {
                const int f = min(t + kThreads * j, NF4 - 1);
                if (BF16) {
                    ar[g][j] = ((const u32x4 *)(a.mats_bf + ((int64_t)dir * NGR + kc) * 3 * PART))[f];
                } else {
                    const int row = f >> 3, k4 = (f & 7) * 4;
                    ar[g][j] = *(const u32x4 *)(a.mats + ((size_t)dir * RP + row) * RP + kc * KC + k4);
                }
            }
        }
        if (++a_st == NST) {
            a_st = 0;
            ++a_e;
        }
    };
    auto load_b = [&]() {
#pragma unroll
        for (int g = 0; g < GPS; ++g) {
            const int kc = b_st * GPS + (b_st * GPS + g < NGR ? g : 0);
#pragma unroll
            for (int j = 0; j < NBL; ++j) {
                const int piece = (t + kThreads * j) % PPC;
                const int svl = max(cur_sv[j], 0);
                if (BF16)
                    br[g][j] = *(const u32x4 *)(a.in_bf + svl * vec_bf_stride(RP) + kc * 3 * KC + 8 * piece);
                else
                    br[g][j] = *(const u32x4 *)(a.in + (size_t)svl * RP + kc * KC + 4 * piece);
            }
        }
#pragma unroll
        for (int j = 0; j < NBL; ++j) bkeep[j] = cur_sv[j] >= 0 ? 0xffffffffu : 0u;
        live_next = __ballot(cur_own >= 0) != 0;
        if (++b_st == NST) {
            b_st = 0;
            ++b_e;
#pragma unroll
            for (int j = 0; j < NBL; ++j) cur_sv[j] = nxt_sv[j];
            cur_own = nxt_own;
            if (NST == 1) fetch_src(min(b_e + 1, nact - 1), nxt_sv, nxt_own);
        } else if (b_st == 1) {
            fetch_src(min(b_e + 1, nact - 1), nxt_sv, nxt_own);
        }
    };
    auto store_ab = [&](int buf, int ng) {
#pragma unroll
        for (int g = 0; g < GPS; ++g) {
            if (g >= ng) continue;
            unsigned char *base = ldsA + (buf * GPS + g) * CHUNK;
#pragma unroll
            for (int j = 0; j < NLOAD; ++j) {
                const int f = t + kThreads * j;
                if (NF4 % kThreads != 0 && f >= NF4) continue;
                if (BF16) {
                    ((u32x4 *)base)[f] = ar[g][j];
                } else {
                    const int row = f >> 3, k4 = (f & 7) * 4;
                    const int rb = row >> 5;
                    const int fl = (row & 31) + 32 * (k4 >> 4), slot = k4 & 15;
                    *(u32x4 *)((float *)base + (rb * 64 + fl) * 16 + slot) = ar[g][j];
                }
            }
            unsigned char *bb = ldsB + (buf * GPS + g) * BCH;
#pragma unroll
            for (int j = 0; j < NBL; ++j) {
                const int f = t + kThreads * j;
                *(u32x4 *)(bb + (f / PPC) * BSTR + (f % PPC) * 16) = br[g][j] & bkeep[j];
            }
        }
    };

    bool live = false;
    if (nsteps > 0) {
        load_a();
        load_b();
        live = live_next;
        store_ab(0, granules(0));
    }
    for (int s = 0; s < nsteps; ++s) {
        const int buf = NBUF == 2 ? (s & 1) : 0;
        const int ng = granules(s % NST);
        const bool live_s = live;
        __syncthreads();  // A(s), B(s) visible in LDS; every wave is done with the other buffer
        if (s + 1 < nsteps) {
            load_a();
            load_b();
            live = live_next;
        }
        if (live_s) {
#pragma unroll
            for (int g = 0; g < GPS; ++g) {
                if (g >= ng) continue;
                const unsigned char *base = ldsA + (buf * GPS + g) * CHUNK;
                const unsigned char *bb = ldsB + (buf * GPS + g) * BCH + my_col * BSTR;
                if (BF16) {
                    const uint16_t *p = (const uint16_t *)base;
                    bf16x8 bh[2], bm[2], bl[2];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        bh[h2] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(bb + 0 * 64 + 32 * h2 + 16 * hf));
                        bm[h2] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(bb + 1 * 64 + 32 * h2 + 16 * hf));
                        bl[h2] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(bb + 2 * 64 + 32 * h2 + 16 * hf));
                    }
#pragma unroll
                    for (int i = 0; i < RBH; ++i) {
                        if (i >= nrb) continue;
                        const int rb = rb0 + i;
                        f32x16 c = acc[i];
#pragma unroll
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
                    f32x4 bv4[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) bv4[q] = *(const f32x4 *)(bb + 64 * hf + 16 * q);
#pragma unroll
                    for (int i = 0; i < RBH; ++i) {
                        if (i >= nrb) continue;
                        const int rb = rb0 + i;
                        const f32x4 *ap4 = (const f32x4 *)(p + (rb * 64 + lane) * 16);
                        const f32x4 av4[4] = {ap4[0], ap4[1], ap4[2], ap4[3]};
                        f32x16 c = acc[i];
#pragma unroll
                        for (int q = 0; q < 16; ++q)
                            c = __builtin_amdgcn_mfma_f32_32x32x2f32(av4[q >> 2][q & 3], bv4[q >> 2][q & 3], c, 0, 0,
                                                                     0);
                        acc[i] = c;
                    }
                }
            }
        }
        if (s + 1 < nsteps) {
            if (NBUF == 1) __syncthreads();
            store_ab(NBUF == 2 ? buf ^ 1 : 0, granules((s + 1) % NST));
        }
    }
    if (outv >= 0) {
#pragma unroll
        for (int i = 0; i < RBH; ++i) {
            if (i >= nrb) continue;
            const int rb = rb0 + i;
#pragma unroll
            for (int v4 = 0; v4 < 4; ++v4) {
                f32x4 *op = (f32x4 *)(a.out + (size_t)outv * RP + rb * 32 + 8 * v4 + 4 * hf);
                f32x4 cur = *op;
                cur[0] += acc[i][4 * v4];
                cur[1] += acc[i][4 * v4 + 1];
                cur[2] += acc[i][4 * v4 + 2];
                cur[3] += acc[i][4 * v4 + 3];
                *op = cur;
            }
        }
    }
}

// Matrices [ndir][r_pad][r_pad] float32 -> split-BF16 chunks in LDS image order.
__global__ void k_split_mats(const float *rm, int r_pad, int64_t total, uint16_t *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;  // total = ndir * r_pad * r_pad
    const int nrb = r_pad / 32, nkc = r_pad / KC;
    const int64_t part_sz = (int64_t)nrb * 2 * 64 * 8;
    // idx enumerates (dir, kc, rb, h2, lane, slot); each thread writes all three parts
    const int slot = (int)(idx % 8);
    int64_t r = idx / 8;
    const int ln = (int)(r % 64);
    r /= 64;
    const int h2 = (int)(r % 2);
    r /= 2;
    const int rb = (int)(r % nrb);
    r /= nrb;
    const int kc = (int)(r % nkc);
    const int64_t dir = r / nkc;
    const int row = rb * 32 + (ln & 31);
    const int k = kc * KC + 16 * h2 + 8 * (ln >> 5) + slot;
    uint16_t h, m, l;
    split3(rm[(dir * r_pad + row) * r_pad + k], h, m, l);
    uint16_t *o = out + (dir * nkc + kc) * 3 * part_sz + ((int64_t)(rb * 2 + h2) * 64 + ln) * 8 + slot;
    o[0] = h;
    o[part_sz] = m;
    o[2 * part_sz] = l;
}

__global__ void k_split_vecs(const float *in, int r_pad, int64_t total, uint16_t *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;  // total = nvec * r_pad
    const int64_t v = idx / r_pad;
    const int k = (int)(idx % r_pad), kc = k / KC, kk = k % KC;
    uint16_t h, m, l;
    split3(in[idx], h, m, l);
    uint16_t *o = out + v * vec_bf_stride(r_pad) + kc * 3 * KC + kk;
    o[0] = h;
    o[KC] = m;
    o[2 * KC] = l;
}

template <int NRB, bool BF16>
void launch(const M2LLaunch &a, hipStream_t s) {
    constexpr int chunk = a_chunk_bytes<NRB, BF16>() + kCols * b_col_stride<BF16>();  // A + B granule
    constexpr int GPS = 4 * chunk <= 160 * 1024 ? 2 : 1;
    constexpr int NBUF = 2 * GPS * chunk <= 160 * 1024 ? 2 : 1;
    constexpr int bytes = NBUF * GPS * chunk;
    static_assert(bytes <= 160 * 1024, "A and B granules do not fit in LDS");
    auto k = k_m2l<NRB, BF16, NBUF, GPS>;
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

size_t m2l_split_mats_elems(int r_pad, int ndir) { return (size_t)ndir * 3 * r_pad * r_pad; }
size_t m2l_split_vecs_elems(int r_pad, int64_t nvec) { return (size_t)nvec * vec_bf_stride(r_pad); }

void m2l_split_mats(const float *rm, int r_pad, int ndir, uint16_t *out, hipStream_t s) {
    FMM_REQUIRE(m2l_supported(r_pad), "m2l: unsupported state size");
    const int64_t total = (int64_t)ndir * r_pad * r_pad;
    if (total == 0) return;
    hipLaunchKernelGGL(k_split_mats, dim3(grid_for(total, 256)), dim3(256), 0, s, rm, r_pad, total, out);
    FMM_HIP(hipGetLastError());
}

void m2l_split_vecs(const float *in, int r_pad, int64_t nvec, uint16_t *out, hipStream_t s) {
    const int64_t total = nvec * r_pad;
    if (total == 0) return;
    hipLaunchKernelGGL(k_split_vecs, dim3(grid_for(total, 256)), dim3(256), 0, s, in, r_pad, total, out);
    FMM_HIP(hipGetLastError());
}

void m2l_run(bool bf16, const M2LLaunch &a, hipStream_t s) {
    if (a.ntile <= 0) return;
    FMM_REQUIRE(m2l_supported(a.r_pad), "m2l: unsupported state size");
    FMM_REQUIRE(a.ncol == m2l_ncol(a.r_pad), "m2l: tile width mismatch");
    FMM_REQUIRE(bf16 ? (a.mats_bf && a.in_bf) : (a.mats && a.in), "m2l: operands missing for this form");
    if (bf16)
        dispatch<true>(a.r_pad / 32, a, s);
    else
        dispatch<false>(a.r_pad / 32, a, s);
}

}  // namespace fmm
