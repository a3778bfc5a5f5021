// Device-wide primitives: exclusive prefix sums and a stable LSD radix sort.
//
// The Morton sort of the octree build (points mapped to a 1-D array by their
// z-value, Sec. III.B) runs on these. The radix sort is stable, so equal keys
// keep their input order, which makes the sorted order (and the tree) a pure
// function of the input.
#include "common.hpp"

namespace fmm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Inclusive scan of one value per thread across the block (Hillis-Steele in LDS).
template <class T>
__device__ T block_inclusive_scan(T v, T *sh) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T add = (t >= off) ? sh[t - off] : T(0);
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    T r = sh[t];
    __syncthreads();
    return r;
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const T *in, int64_t n, T *sums) {
    __shared__ T sh[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T acc = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) acc += in[base + i];
    T inc = block_inclusive_scan(acc, sh);
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = inc;
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T *in, T *out, int64_t n, const T *offsets) {
    __shared__ T sh[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T acc = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : T(0);
        acc += v[i];
    }
    T inc = block_inclusive_scan(acc, sh);
    T run = inc - acc + (offsets ? offsets[blockIdx.x] : T(0));
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

template <class T>
void scan_impl(const T *in, T *out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 1) {
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kScanThreads), 0, s, in, out, n, (const T *)nullptr);
        FMM_HIP(hipGetLastError());
        return;
    }
    DBuf<T> sums(nt);
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, n, sums.p);
    FMM_HIP(hipGetLastError());
    scan_impl<T>(sums.p, sums.p, nt, s);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, out, n,
                       (const T *)sums.p);
    FMM_HIP(hipGetLastError());
    FMM_HIP(hipStreamSynchronize(s));  // `sums` is freed on return
}

template <class T>
T scan_total(const T *in, T *out, int64_t n, hipStream_t s, bool want_total) {
    if (n <= 0) return 0;
    T last_in = 0;
    if (want_total) d2h(&last_in, in + (n - 1), 1, s);
    scan_impl<T>(in, out, n, s);
    if (!want_total) return 0;
    T last_out = 0;
    d2h(&last_out, out + (n - 1), 1, s);
    return last_out + last_in;
}

// ---------------------------------------------------------------- radix sort
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                       uint32_t *hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int i = 0; i < kRsItems; ++i) {
        int64_t idx = base + (int64_t)i * kRsThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: rounds of 256 keys in input order; within a round the rank
// of a key among equal digits comes from wave ballots (lanes below it) and
// the counts of the waves before it.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t *kin, const int64_t *vin,
                                                          uint64_t *kout, int64_t *vout, int64_t n,
                                                          int shift, const uint32_t *offs, int nblk) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    run[t] = offs[(int64_t)t * nblk + blockIdx.x];
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        wcnt[0][t] = 0;
        wcnt[1][t] = 0;
        wcnt[2][t] = 0;
        wcnt[3][t] = 0;
        __syncthreads();
        int64_t idx = base + (int64_t)r * kRsThreads + t;
        bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0ull;
        int64_t val = valid ? vin[idx] : 0;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0) wcnt[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w2 = 0; w2 < wv; ++w2) pos += wcnt[w2][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        __syncthreads();
    }
}

}  // namespace

int64_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, bool want_total) {
    return scan_total<int64_t>(in, out, n, s, want_total);
}
int64_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, bool want_total) {
    return scan_total<int32_t>(in, out, n, s, want_total);
}
uint32_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s, bool want_total) {
    return scan_total<uint32_t>(in, out, n, s, want_total);
}

void radix_sort_pairs(uint64_t *keys, int64_t *vals, int64_t n, int bits, hipStream_t s) {
    if (n <= 1) return;
    FMM_REQUIRE(n < (int64_t(1) << 31), "radix sort: more than 2^31 - 1 points");
    int nblk = (int)((n + kRsTile - 1) / kRsTile);
    DBuf<uint64_t> k2(n);
    DBuf<int64_t> v2(n);
    DBuf<uint32_t> hist((size_t)256 * nblk);
    uint64_t *ka = keys, *kb = k2.p;
    int64_t *va = vals, *vb = v2.p;
    int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kRsThreads), 0, s, ka, n, shift, hist.p, nblk);
        FMM_HIP(hipGetLastError());
        scan_impl<uint32_t>(hist.p, hist.p, (int64_t)256 * nblk, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kRsThreads), 0, s, ka, va, kb, vb, n, shift,
                           hist.p, nblk);
        FMM_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        FMM_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        FMM_HIP(hipMemcpyAsync(vals, va, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    }
    FMM_HIP(hipStreamSynchronize(s));
}

}  // namespace fmm
