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
// Blocking. A workgroup owns a tile of 128 target boxes of one octant. With
// 8 waves each takes one 32-column block and one half of the rows; with 4
// (split-BF16 up to r_pad 192, two or three workgroups per CU) each takes one column
// block and all rows. The workgroup keeps the r_pad x 128 accumulator in
// registers across all directions, so every output is written once. Each step of the tile is one
// (direction, 32-wide k-chunk): the chunk of M_d and the tile's 128 source
// chunks are copied from global memory straight into LDS (global_load_lds,
// 16 bytes per lane, no registers on the way) and every wave multiplies
// them. With 32x32 MFMA tiles each staged matrix element is read from LDS once
// per 32 columns. With two LDS buffers (8-wave split-BF16) the copies of step s + 1
// are issued at the start of step s and run under its MFMAs; with one
// (float32, and the 4-wave split-BF16 form), two or three workgroups share
// each CU.
// The tiles of one octant run on one XCD (they share most directions, so
// concurrently running tiles reuse the matrices in that XCD's L2).
//
// The k index inside a chunk is permuted so that every lane's operand is a
// run of consecutive values (16-byte reads); the dot product is the same.
//
// Forms:
//   FP32        v_mfma_f32_32x32x2_f32; the float32 matrices are stored chunk
//               by chunk in fragment order (the exact LDS image).
//   split-BF16  both operands split into bfloat16 parts and the part products
//               accumulated in float32 with v_mfma_f32_32x32x16_bf16 (the
//               schemes of Henry, Tang and Heinecke, 2019): three parts
//               x = h + m + l and the six products hh hm mh mm hl lh (bf16x6,
//               about float32 accuracy), or two parts x = h + m and the
//               products hh hm mh (bf16x3), optionally with mm (bf16x4), with
//               two thirds of the bytes and half (or two thirds) of the MFMAs.
//               The split is done once, outside the inner loop: the matrices
//               when the operators are built (stored chunk by chunk in the
//               exact LDS image), the source vectors by one pass over the
//               upward state per apply. The inner loop is then only copies
//               and MFMAs.
#include <type_traits>

#include "m2l.hpp"

namespace fmm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));  // plain vectors: promotable to registers
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kCols = 128;     // 4 column blocks of 32
constexpr int KC = 32;         // k per step

// float32 -> bfloat16, round to nearest even (finite inputs)
__device__ inline uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// x = h + m + l up to 2^-24 |x| (each residual is exact in float32); the
// two-part split is h and m (x = h + m up to 2^-16 |x|)
__device__ inline void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
    h = f2bf(x);
    float r1 = x - bf2f(h);
    m = f2bf(r1);
    l = f2bf(r1 - bf2f(m));
}

// One A chunk (r_pad rows x 32 k) in LDS and in the global image, fragment order:
//   BF16 (32x32x16): part p (of NP = 3 or 2), row block rb, k-half h (16 k each), lane, 8 slots;
//                    element (row, k) -> lane = row % 32 + 32 * ((k % 16) / 8), slot = k % 8
//   FP32 (32x32x2):  row block rb, lane, 16 slots;
//                    element (row, k) -> lane = row % 32 + 32 * (k / 16), slot = k % 16
// Split-BF16 source vector layout: per vector, per 32-k chunk, NP parts of 32
// bfloat16 (64 NP bytes); float32 vectors are plain rows of r_pad values.
__host__ __device__ constexpr int64_t vec_bf_stride(int r_pad, int np) { return np * (int64_t)r_pad; }

// M2L arithmetic: 0 float32; 6, 4, 3 the split-BF16 products (parts: 3, 2, 2)
__host__ __device__ constexpr int form_parts(int form) { return form == 6 ? 3 : 2; }

// XCD-aware tile order: blocks are dealt to the 8 XCDs round-robin, so
// block b runs on XCD b % 8. XCD x receives cnt(x) blocks and owns tiles
// [start(x), start(x) + cnt(x)), a bijection of [0, ntile) (the plan pads
// ntile to a multiple of 8, one range per octant). Returns -1 for blocks
// beyond it.
__device__ inline int xcd_tile(int nb, int b) {
    const int per = (nb + 7) / 8;
    const int rem = nb - (per - 1) * 8;
    const int x = b % 8, k = b / 8;
    const int cnt = (x < rem) ? per : per - 1;
    const int start = (x < rem) ? x * per : rem * per + (x - rem) * (per - 1);
    return k < cnt ? start + k : -1;
}

typedef __attribute__((address_space(3))) void lds_void;

// 16 bytes per lane from global memory to LDS: lane i writes dst + 16 i
// (dst wave-uniform)
__device__ inline void copy_to_lds(const void *src, void *dst) {
    __builtin_amdgcn_global_load_lds(src, (lds_void *)dst, 16, 0, 0);
}

// NW = 8 waves: 4 column blocks x 2 row halves, two LDS buffers when they
// fit. NW = 4 waves: one column block each with every row block, one buffer,
// so that two or three workgroups share a CU and cover each other's copies and
// barriers. Either way every wave reads the matrix chunk rows it multiplies
// (4 reads of the chunk per step); with 4 waves the source chunk is read
// once per column block instead of twice (one row half each).
template <int NRB, int FORM, int NW>
struct Shape {
    static_assert(NW == 8 || NW == 4, "8 or 4 waves");
    static constexpr bool BF16 = FORM != 0;
    static constexpr int NP = form_parts(FORM);                // bfloat16 parts per value
    static constexpr int RP = NRB * 32;
    static constexpr int RBH = NW == 8 ? (NRB + 1) / 2 : NRB;  // row blocks per wave
    static constexpr int CHUNK = BF16 ? NRB * 32 * KC * 2 * NP : NRB * 32 * KC * 4;  // A chunk bytes
    static constexpr int NIA = CHUNK / 1024;                   // 1 KB copies per A chunk
    static constexpr int PPC = BF16 ? 4 * NP : 8;              // 16-byte pieces per column chunk
    static constexpr int SPC = PPC + 1;                        // LDS slots per column (one pad slot)
    static constexpr int BSTR = SPC * 16;                      // column stride in LDS: 16 lanes hit distinct banks
    static constexpr int BCH = kCols * BSTR;                   // B chunk bytes in LDS
    static constexpr int NIB = kCols * SPC / 64;               // 1 KB copies per B chunk
    static constexpr int JA = (NIA + NW - 1) / NW, JB = (NIB + NW - 1) / NW;  // copies per wave (at most)
    static constexpr int LDS2 = 2 * (CHUNK + BCH) + 4 * kNumDirs;
    // Split-BF16: two buffers when they fit in LDS. Float32: one buffer (43 KB at r_pad 192), so two workgroups
    // share a CU and each covers the other's barriers (measured 6% faster
    // than two buffers; for split-BF16 two buffers are 6% faster at the
    // tuned leaf size).
    static constexpr int NBUF = (NW == 8 && BF16 && LDS2 <= 160 * 1024) ? 2 : 1;
    static_assert(kCols * SPC % 64 == 0, "B slots must fill whole copies");
};

template <int NRB, int FORM, int NW>
__global__ __launch_bounds__(NW * 64, 2) void k_m2l(M2LLaunch a) {
    using S = Shape<NRB, FORM, NW>;
    constexpr bool BF16 = S::BF16;
    constexpr int NP = S::NP;
    constexpr int kThreads = NW * 64;
    constexpr int RP = S::RP, RBH = S::RBH, CHUNK = S::CHUNK, NIA = S::NIA, PPC = S::PPC, SPC = S::SPC,
                  BSTR = S::BSTR, BCH = S::BCH, NIB = S::NIB, JA = S::JA, JB = S::JB, NBUF = S::NBUF;
    constexpr int PART = NRB * 2 * 64 * 8;  // bfloat16 elements of one part of an A chunk
    constexpr int NGR = RP / KC;            // steps per direction
    __shared__ __align__(16) unsigned char sA0[CHUNK], sA1[NBUF == 2 ? CHUNK : 16];
    __shared__ __align__(16) unsigned char sB0[BCH], sB1[NBUF == 2 ? BCH : 16];
    unsigned char *sA[2] = {sA0, sA1};
    unsigned char *sB[2] = {sB0, sB1};
    __shared__ int32_t s_dir[kNumDirs];
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6) & (NW - 1);
    const int hf = lane >> 5, r32 = lane & 31;
    const int cblk = w & 3, rhalf = NW == 8 ? w >> 2 : 0;
    const int rb0 = rhalf * RBH;
    const int nrb = (rb0 + RBH <= NRB) ? RBH : NRB - rb0;

    const int tile = xcd_tile(gridDim.x, blockIdx.x);
    if (tile < 0) return;
    const int64_t toff = a.tile_term_off[tile];
    const int nact = (int)(a.tile_term_off[tile + 1] - toff);
    const int nsteps = nact * NGR;
    const int my_col = 32 * cblk + r32;
    const int outv = a.tile_cols[(int64_t)tile * kCols + my_col];
    for (int i = t; i < nact; i += kThreads) s_dir[i] = a.term_dir[toff + i];

    // B copies: copy i = w + NW j fills LDS slots 64 i .. 64 i + 63; slot q is
    // piece q % SPC of column q / SPC (piece PPC is the pad slot). Columns
    // without a source for the direction, and pad slots, copy zeros.
    int bcol[JB], bpiece[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        const int q = (w + NW * j) * 64 + lane;
        bcol[j] = min(q / SPC, kCols - 1);
        bpiece[j] = q % SPC;
    }
    int cur_sv[JB], nxt_sv[JB], cur_own = -1, nxt_own = -1;
    auto fetch_src = [&](int e, int (&sv)[JB], int &own) {
        const int64_t row = (toff + e) * kCols;
#pragma unroll
        for (int j = 0; j < JB; ++j) sv[j] = a.term_src[row + bcol[j]];
        own = a.term_src[row + my_col];
    };
    if (nact > 0) {
        fetch_src(0, cur_sv, cur_own);
        fetch_src(nact > 1 ? 1 : 0, nxt_sv, nxt_own);
    }
    __syncthreads();  // s_dir

    f32x16 acc[RBH];
#pragma unroll
    for (int i = 0; i < RBH; ++i)
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;

    // issue the copies of the next step (direction e_ld, chunk st_ld) into buffer BUF
    int e_ld = 0, st_ld = 0;
    bool live_q[NBUF];
    auto issue = [&](auto buf_tag) {
        constexpr int BUF = decltype(buf_tag)::value;
        const int dir = __builtin_amdgcn_readfirstlane(s_dir[min(e_ld, nact - 1)]);
        const int kc = st_ld;
        const unsigned char *ag = BF16 ? (const unsigned char *)(a.mats_bf + ((int64_t)dir * NGR + kc) * NP * PART)
                                       : (const unsigned char *)(a.mats + ((int64_t)dir * NGR + kc) * (CHUNK / 4));
#pragma unroll
        for (int j = 0; j < JA; ++j) {
            const int i = w + NW * j;
            if (NIA % NW != 0 && i >= NIA) continue;  // wave-uniform
            copy_to_lds(ag + (size_t)i * 1024 + lane * 16, &sA[BUF][i * 1024]);
        }
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            const int i = w + NW * j;
            if (NIB % NW != 0 && i >= NIB) continue;
            const int pc = bpiece[j];
            const unsigned char *src;
            if (cur_sv[j] < 0 || pc == PPC)
                src = (const unsigned char *)a.zero + 16 * (pc % PPC);
            else if (BF16)
                src = (const unsigned char *)(a.in_bf + cur_sv[j] * vec_bf_stride(RP, NP) + kc * NP * KC + 8 * pc);
            else
                src = (const unsigned char *)(a.in + (size_t)cur_sv[j] * RP + kc * KC + 4 * pc);
            copy_to_lds(src, &sB[BUF][i * 1024]);
        }
        live_q[BUF] = __ballot(cur_own >= 0) != 0;  // does this wave's column block have any source?
        // k-chunk major: every direction of the tile at chunk kc, then chunk kc + 1
        if (++e_ld == nact) {
            e_ld = 0;
            ++st_ld;
        }
#pragma unroll
        for (int j = 0; j < JB; ++j) cur_sv[j] = nxt_sv[j];
        cur_own = nxt_own;
        fetch_src(e_ld + 1 < nact ? e_ld + 1 : 0, nxt_sv, nxt_own);
    };

    // Operand fragments of one step. The two buffers are distinct LDS
    // objects, so the compiler can tell that reads of one do not wait for
    // copies into the other: the next step's copies are issued first and
    // the fragments are read one row block at a time under the MFMAs.
    constexpr int NFA = BF16 ? 2 * NP : 4;  // 16-byte A fragments per row block
    constexpr int NFB = BF16 ? 2 * NP : 4;
    u32x4 fa[NFA], fb[NFB];
    auto read_b = [&](int buf) {
        const unsigned char *bb = sB[buf] + my_col * BSTR;
#pragma unroll
        for (int f = 0; f < NFB; ++f)
            fb[f] = BF16 ? *(const u32x4 *)(bb + (f % NP) * 64 + 32 * (f / NP) + 16 * hf)  // part f % NP, k-half f / NP
                         : *(const u32x4 *)(bb + 64 * hf + 16 * f);
    };
    auto read_a = [&](int buf, int rb, u32x4 (&fr)[NFA]) {
        if (BF16) {
            const uint16_t *p = (const uint16_t *)sA[buf];
#pragma unroll
            for (int f = 0; f < NFA; ++f)
                fr[f] = *(const u32x4 *)(p + (f % NP) * PART + ((rb * 2 + f / NP) * 64 + lane) * 8);
        } else {
            const float *p = (const float *)sA[buf];
#pragma unroll
            for (int f = 0; f < NFA; ++f) fr[f] = *(const u32x4 *)(p + (rb * 64 + lane) * 16 + 4 * f);
        }
    };
    // the products of one row block (index i) on fragments fr, chained on acc[i]
    auto mfma_row = [&](int i, const u32x4 (&fr)[NFA]) {
        f32x16 c = acc[i];
        if (BF16) {
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const bf16x8 ah = __builtin_bit_cast(bf16x8, fr[NP * h2]), am = __builtin_bit_cast(bf16x8, fr[NP * h2 + 1]);
                const bf16x8 bh = __builtin_bit_cast(bf16x8, fb[NP * h2]), bm = __builtin_bit_cast(bf16x8, fb[NP * h2 + 1]);
                // smallest products first
                if constexpr (NP == 3) {
                    const bf16x8 al = __builtin_bit_cast(bf16x8, fr[NP * h2 + 2]);
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, fb[NP * h2 + 2]);
                    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
                }
                if constexpr (FORM != 3) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q)
                c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(f32x4, fr[q >> 2])[q & 3],
                                                         __builtin_bit_cast(f32x4, fb[q >> 2])[q & 3], c, 0, 0, 0);
        }
        acc[i] = c;
    };

    if constexpr (NBUF == 2) {
        if (nsteps > 0) issue(std::integral_constant<int, 0>{});
        auto step = [&](auto buf_tag, int s) {
            constexpr int BUF = decltype(buf_tag)::value;
            const bool live_s = live_q[BUF];
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's copies of step s are in LDS
            __syncthreads();                      // every wave's are; the other buffer is no longer read
            if (s + 1 < nsteps) issue(std::integral_constant<int, 1 - BUF>{});
            if (live_s) {
                read_b(BUF);
#pragma unroll
                for (int i = 0; i < RBH; ++i) {
                    if (i >= nrb) continue;
                    read_a(BUF, rb0 + i, fa);
                    mfma_row(i, fa);
                }
            }
        };
        for (int s = 0; s < nsteps; s += 2) {
            step(std::integral_constant<int, 0>{}, s);
            if (s + 1 < nsteps) step(std::integral_constant<int, 1>{}, s + 1);
        }
    } else {
        if (nsteps > 0) issue(std::integral_constant<int, 0>{});
        for (int s = 0; s < nsteps; ++s) {
            const bool live_s = live_q[0];
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            __syncthreads();                      // step s is in LDS
            if (live_s) {
                read_b(0);
#pragma unroll
                for (int i = 0; i < RBH; ++i) {
                    if (i >= nrb) continue;
                    read_a(0, rb0 + i, fa);
                    mfma_row(i, fa);
                }
            }
            __syncthreads();  // every wave is done with the buffer
            if (s + 1 < nsteps) issue(std::integral_constant<int, 0>{});
        }
    }
    const int slot = a.piece_slot ? a.piece_slot[tile] : -1;
    if (slot >= 0 && outv >= 0) {  // a piece of a cut tile: its partial sum, added to out by k_m2l_reduce
#pragma unroll
        for (int i = 0; i < RBH; ++i) {
            if (i >= nrb) continue;
            const int rb = rb0 + i;
#pragma unroll
            for (int v4 = 0; v4 < 4; ++v4) {
                f32x4 v;
                for (int c = 0; c < 4; ++c) v[c] = acc[i][4 * v4 + c];
                *(f32x4 *)(a.partial + ((size_t)slot * kCols + my_col) * RP + rb * 32 + 8 * v4 + 4 * hf) = v;
            }
        }
    } else if (outv >= 0) {
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

// Cut tiles: out[cols[c]] += partial[slot0] + partial[slot0 + 1] + ... (in
// piece order, so the result does not depend on which piece ran first).
// Block (tile, g) adds columns 16 g .. 16 g + 15, four values per thread.
constexpr int kRedCols = 16;
__global__ __launch_bounds__(256) void k_m2l_reduce(int r_pad, int ncol, const int32_t *cols, const int32_t *slot0,
                                                    const int32_t *kpieces, const float *partial, float *out) {
    const int tl = blockIdx.x;
    const int k = kpieces[tl];
    const size_t per = (size_t)ncol * r_pad;  // floats per slot
    const int q4 = r_pad / 4;
    for (int idx = threadIdx.x; idx < kRedCols * q4; idx += 256) {
        const int c = blockIdx.y * kRedCols + idx / q4, r4 = (idx % q4) * 4;
        const int v = cols[(size_t)tl * ncol + c];
        if (v < 0) continue;
        const float *p = partial + (size_t)slot0[tl] * per + (size_t)c * r_pad + r4;
        f32x4 sum = *(const f32x4 *)p;
        for (int q = 1; q < k; ++q) sum += *(const f32x4 *)(p + q * per);
        f32x4 *o = (f32x4 *)(out + (size_t)v * r_pad + r4);
        *o = *o + sum;
    }
}

// Pair tiles: out[targets[t]] += the partial rows rows[off[t]] .. rows[off[t+1] - 1]
// (row i at partial + i * r_pad), added in the given (direction) order. One
// wave per target, four values per lane. The row indices are loaded 64 at a
// time (one per lane) and broadcast with readlane, so four row loads are in
// flight at once instead of one dependent index-then-row chain per row.
__global__ __launch_bounds__(256) void k_m2l_gather(int r_pad, int n, const int32_t *targets, const int32_t *off,
                                                    const int32_t *rows, const float *partial, float *out) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= n) return;
    const int v = targets[t], e0 = off[t], m = off[t + 1] - e0;
    auto row = [&](int i, int c) { return *(const f32x4 *)(partial + (size_t)i * r_pad + c); };
    for (int c0 = 0; c0 < r_pad; c0 += 256) {
        const int c = c0 + 4 * lane;
        const bool act = c < r_pad;
        f32x4 sum = {0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < m; b += 64) {
            const int idx = b + lane < m ? rows[e0 + b + lane] : 0;
            const int cnt = min(64, m - b);
            int k = 0;
            for (; k + 4 <= cnt; k += 4) {
                const int i0 = __builtin_amdgcn_readlane(idx, k), i1 = __builtin_amdgcn_readlane(idx, k + 1);
                const int i2 = __builtin_amdgcn_readlane(idx, k + 2), i3 = __builtin_amdgcn_readlane(idx, k + 3);
                if (act) {
                    const f32x4 a0 = row(i0, c), a1 = row(i1, c), a2 = row(i2, c), a3 = row(i3, c);
                    sum += a0;
                    sum += a1;
                    sum += a2;
                    sum += a3;
                }
            }
            for (; k < cnt; ++k) {
                const int i = __builtin_amdgcn_readlane(idx, k);
                if (act) sum += row(i, c);
            }
        }
        if (act) {
            f32x4 *o = (f32x4 *)(out + (size_t)v * r_pad + c);
            *o = *o + sum;
        }
    }
}

// Matrices [ndir][r_pad][r_pad] float32 -> split-BF16 chunks (np = 3 or 2
// parts) in LDS image order.
__global__ void k_split_mats(const float *rm, int r_pad, int np, int64_t total, uint16_t *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;  // total = ndir * r_pad * r_pad
    const int nrb = r_pad / 32, nkc = r_pad / KC;
    const int64_t part_sz = (int64_t)nrb * 2 * 64 * 8;
    // idx enumerates (dir, kc, rb, h2, lane, slot); each thread writes all parts
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
    uint16_t *o = out + (dir * nkc + kc) * np * part_sz + ((int64_t)(rb * 2 + h2) * 64 + ln) * 8 + slot;
    o[0] = h;
    o[part_sz] = m;
    if (np == 3) o[2 * part_sz] = l;
}

__global__ void k_split_vecs(const float *in, int r_pad, int np, int64_t total, uint16_t *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;  // total = nvec * r_pad
    const int64_t v = idx / r_pad;
    const int k = (int)(idx % r_pad), kc = k / KC, kk = k % KC;
    uint16_t h, m, l;
    split3(in[idx], h, m, l);
    uint16_t *o = out + v * vec_bf_stride(r_pad, np) + kc * np * KC + kk;
    o[0] = h;
    o[KC] = m;
    if (np == 3) o[2 * KC] = l;
}

// Inverse maps of the two split layouts (three parts), for inspection:
// parts[p][i] is part p of the i-th value in row-major order (vectors of
// r_pad values, or r_pad x r_pad matrices).
__global__ void k_unsplit_vecs(const uint16_t *img, int r_pad, int64_t total, uint16_t *parts) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int64_t v = idx / r_pad;
    const int k = (int)(idx % r_pad), kc = k / KC, kk = k % KC;
    const uint16_t *src = img + v * vec_bf_stride(r_pad, 3) + kc * 3 * KC + kk;
    for (int p = 0; p < 3; ++p) parts[p * total + idx] = src[p * KC];
}

__global__ void k_unsplit_mats(const uint16_t *img, int r_pad, int64_t total, uint16_t *parts) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;  // total = ndir * r_pad * r_pad, idx = (dir, row, k)
    const int nrb = r_pad / 32, nkc = r_pad / KC;
    const int64_t part_sz = (int64_t)nrb * 2 * 64 * 8;
    const int k = (int)(idx % r_pad), row = (int)((idx / r_pad) % r_pad);
    const int64_t dir = idx / ((int64_t)r_pad * r_pad);
    const int kc = k / KC, kk = k % KC;
    const int h2 = kk / 16, ln = (row & 31) + 32 * ((kk % 16) / 8), slot = kk % 8, rb = row / 32;
    const uint16_t *src = img + (dir * nkc + kc) * 3 * part_sz + ((int64_t)(rb * 2 + h2) * 64 + ln) * 8 + slot;
    for (int p = 0; p < 3; ++p) parts[p * total + idx] = src[p * part_sz];
}

// Matrices [ndir][r_pad][r_pad] float32 -> float32 chunks in LDS image order.
__global__ void k_image_f32(const float *rm, int r_pad, int64_t total, float *out) {
    int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;  // total = ndir * r_pad * r_pad
    const int nrb = r_pad / 32, nkc = r_pad / KC;
    // idx enumerates (dir, kc, rb, lane, slot)
    const int slot = (int)(idx % 16);
    int64_t r = idx / 16;
    const int ln = (int)(r % 64);
    r /= 64;
    const int rb = (int)(r % nrb);
    r /= nrb;
    const int kc = (int)(r % nkc);
    const int64_t dir = r / nkc;
    const int row = rb * 32 + (ln & 31);
    const int k = kc * KC + 16 * (ln >> 5) + slot;
    out[idx] = rm[(dir * r_pad + row) * r_pad + k];
}

// waves per workgroup: 4 for split-BF16 states up to 192 values (the
// accumulators of every row block fit beside a second workgroup), else 8
template <int NRB, int FORM>
constexpr int waves_for() {
    return (FORM != 0 && NRB <= 6) ? 4 : 8;
}

template <int NRB, int FORM>
void launch(const M2LLaunch &a, hipStream_t s) {
    constexpr int NW = waves_for<NRB, FORM>();
    using S = Shape<NRB, FORM, NW>;
    static_assert(S::NBUF == 2 || S::LDS2 / 2 <= 160 * 1024, "chunks do not fit in LDS");
    hipLaunchKernelGGL((k_m2l<NRB, FORM, NW>), dim3(a.ntile), dim3(NW * 64), 0, s, a);
    FMM_HIP(hipGetLastError());
}

template <int FORM, int NRB = 1>
int blocks_per_cu(int nrb) {
    if constexpr (NRB <= 16) {
        if (nrb != NRB) return blocks_per_cu<FORM, NRB + 1>(nrb);
        int n = 0;
        constexpr int NW = waves_for<NRB, FORM>();
        FMM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_m2l<NRB, FORM, NW>, NW * 64, 0));
        return n > 0 ? n : 1;
    } else {
        return 1;
    }
}

template <int FORM, int NRB = 1>
void dispatch(int nrb, const M2LLaunch &a, hipStream_t s) {
    if constexpr (NRB <= 16) {
        if (nrb == NRB)
            launch<NRB, FORM>(a, s);
        else
            dispatch<FORM, NRB + 1>(nrb, a, s);
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

int m2l_form_parts(int form) { return form_parts(form); }
size_t m2l_split_mats_elems(int r_pad, int ndir, int np) { return (size_t)ndir * np * r_pad * r_pad; }
size_t m2l_split_vecs_elems(int r_pad, int64_t nvec, int np) { return (size_t)nvec * vec_bf_stride(r_pad, np); }

void m2l_split_mats(const float *rm, int r_pad, int ndir, int np, uint16_t *out, hipStream_t s) {
    FMM_REQUIRE(m2l_supported(r_pad), "m2l: unsupported state size");
    FMM_REQUIRE(np == 2 || np == 3, "m2l: 2 or 3 bfloat16 parts");
    const int64_t total = (int64_t)ndir * r_pad * r_pad;
    if (total == 0) return;
    hipLaunchKernelGGL(k_split_mats, dim3(grid_for(total, 256)), dim3(256), 0, s, rm, r_pad, np, total, out);
    FMM_HIP(hipGetLastError());
}

void m2l_image_mats(const float *rm, int r_pad, int ndir, float *out, hipStream_t s) {
    FMM_REQUIRE(m2l_supported(r_pad), "m2l: unsupported state size");
    const int64_t total = (int64_t)ndir * r_pad * r_pad;
    if (total == 0) return;
    hipLaunchKernelGGL(k_image_f32, dim3(grid_for(total, 256)), dim3(256), 0, s, rm, r_pad, total, out);
    FMM_HIP(hipGetLastError());
}

void m2l_split_vecs(const float *in, int r_pad, int64_t nvec, int np, uint16_t *out, hipStream_t s) {
    FMM_REQUIRE(np == 2 || np == 3, "m2l: 2 or 3 bfloat16 parts");
    const int64_t total = nvec * r_pad;
    if (total == 0) return;
    hipLaunchKernelGGL(k_split_vecs, dim3(grid_for(total, 256)), dim3(256), 0, s, in, r_pad, np, total, out);
    FMM_HIP(hipGetLastError());
}

void m2l_split_plain(int which, int r_pad, int64_t count, const float *in, uint16_t *parts, hipStream_t s) {
    FMM_REQUIRE(m2l_supported(r_pad), "m2l: unsupported state size");
    if (count <= 0) return;
    const int64_t total = count * r_pad * (which == 1 ? r_pad : 1);
    DBuf<uint16_t> img(3 * (size_t)total);
    if (which == 1) {
        m2l_split_mats(in, r_pad, (int)count, 3, img.p, s);
        hipLaunchKernelGGL(k_unsplit_mats, dim3(grid_for(total, 256)), dim3(256), 0, s, img.p, r_pad, total, parts);
    } else {
        m2l_split_vecs(in, r_pad, count, 3, img.p, s);
        hipLaunchKernelGGL(k_unsplit_vecs, dim3(grid_for(total, 256)), dim3(256), 0, s, img.p, r_pad, total, parts);
    }
    FMM_HIP(hipGetLastError());
    FMM_HIP(hipStreamSynchronize(s));
}

int m2l_blocks_per_cu(int form, int r_pad) {
    FMM_REQUIRE(m2l_supported(r_pad), "m2l: unsupported state size");
    switch (form) {
    case 0: return blocks_per_cu<0>(r_pad / 32);
    case 3: return blocks_per_cu<3>(r_pad / 32);
    case 4: return blocks_per_cu<4>(r_pad / 32);
    case 6: return blocks_per_cu<6>(r_pad / 32);
    default: throw Error(FMM_ERR_ARG, "m2l: unknown arithmetic");
    }
}

void m2l_reduce(int r_pad, int ntile, int ncol, const int32_t *cols, const int32_t *slot0, const int32_t *kpieces,
                const float *partial, float *out, hipStream_t s) {
    if (ntile <= 0) return;
    FMM_REQUIRE(ncol % kRedCols == 0 && r_pad % 4 == 0, "m2l_reduce: unsupported tile shape");
    hipLaunchKernelGGL(k_m2l_reduce, dim3(ntile, ncol / kRedCols), dim3(256), 0, s, r_pad, ncol, cols, slot0, kpieces,
                       partial, out);
    FMM_HIP(hipGetLastError());
}

void m2l_gather(int r_pad, int n, const int32_t *targets, const int32_t *off, const int32_t *rows,
                const float *partial, float *out, hipStream_t s) {
    if (n <= 0) return;
    FMM_REQUIRE(r_pad % 4 == 0, "m2l_gather: unsupported state size");
    hipLaunchKernelGGL(k_m2l_gather, dim3((n + 3) / 4), dim3(256), 0, s, r_pad, n, targets, off, rows, partial, out);
    FMM_HIP(hipGetLastError());
}

void m2l_run(int form, const M2LLaunch &a, hipStream_t s) {
    if (a.ntile <= 0) return;
    FMM_REQUIRE(m2l_supported(a.r_pad), "m2l: unsupported state size");
    FMM_REQUIRE(a.ncol == m2l_ncol(a.r_pad), "m2l: tile width mismatch");
    FMM_REQUIRE(form ? (a.mats_bf && a.in_bf) : (a.mats && a.in), "m2l: operands missing for this form");
    FMM_REQUIRE(a.zero, "m2l: zero source chunk missing");
    switch (form) {
    case 0: dispatch<0>(a.r_pad / 32, a, s); break;
    case 3: dispatch<3>(a.r_pad / 32, a, s); break;
    case 4: dispatch<4>(a.r_pad / 32, a, s); break;
    case 6: dispatch<6>(a.r_pad / 32, a, s); break;
    default: throw Error(FMM_ERR_ARG, "m2l: unknown arithmetic");
    }
}

}  // namespace fmm
