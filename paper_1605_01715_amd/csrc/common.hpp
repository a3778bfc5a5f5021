// Shared definitions of the MI355X KIFMM library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "fmm.h"

namespace fmm {

constexpr int kMaxLevel = 21;   // finest level of the 63-bit Morton key
constexpr int kNumDirs = 316;   // M2L offsets d in {-3..3}^3 with max|d| >= 2
constexpr int kMaxOrder = 12;
constexpr double kRadIn = 1.05;   // upward-equivalent / downward-check surface radius (box half-widths)
constexpr double kRadOut = 2.95;  // upward-check / downward-equivalent surface radius
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kFourPi = 12.566370614359172953850573533118;

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define FMM_HIP(x)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess)                                                                 \
            throw ::fmm::Error(e_ == hipErrorOutOfMemory ? FMM_ERR_NOMEM : FMM_ERR_DEVICE,    \
                               std::string(#x) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define FMM_REQUIRE(c, msg)                                  \
    do {                                                     \
        if (!(c)) throw ::fmm::Error(FMM_ERR_ARG, (msg));    \
    } while (0)

// Failure injection for tests of the error paths: with the environment
// variable FMM_FAULT_INJECT=alloc:<k> the k-th device allocation counted from
// when the variable took its current value fails as if the device were out
// of memory (FMM_ERR_NOMEM). Returns true for the allocation that must fail.
bool inject_alloc_failure();

// Owning device buffer (hipMalloc'd; freed on destruction).
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (!count) return;
        // on failure, the work already queued finishes before the buffers the
        // failing call had allocated are released on the way out
        if (inject_alloc_failure()) {
            (void)hipDeviceSynchronize();
            throw Error(FMM_ERR_NOMEM, "device allocation failed (injected by FMM_FAULT_INJECT)");
        }
        const hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipDeviceSynchronize();
            FMM_HIP(e);
        }
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
    size_t bytes() const { return n * sizeof(T); }
};

// Host-to-device copy that has finished reading `src` on return (the host
// buffer may be freed or reused right after).
template <class T>
void h2d(T *dst, const T *src, size_t n, hipStream_t s) {
    if (!n) return;
    FMM_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
    FMM_HIP(hipStreamSynchronize(s));
}
template <class T>
void d2h(T *dst, const T *src, size_t n, hipStream_t s) {
    if (n) FMM_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
}
template <class T>
DBuf<T> upload(const std::vector<T> &v, hipStream_t s) {
    DBuf<T> b(v.size());
    h2d(b.p, v.data(), v.size(), s);
    return b;
}

// Diagnostics on stderr, on when the environment variable FMM_LOG is set to
// a value other than 0 (read once per process).
bool log_enabled();
void log_printf(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
#define FMM_LOG(...)                                            \
    do {                                                        \
        if (::fmm::log_enabled()) ::fmm::log_printf(__VA_ARGS__); \
    } while (0)

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

// Device-wide exclusive prefix sum (in may equal out). Returns the total when
// want_total is set (synchronises the stream), else 0.
int64_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, bool want_total);
int64_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, bool want_total);
uint32_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s, bool want_total);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of key.
void radix_sort_pairs(uint64_t *keys, int64_t *vals, int64_t n, int bits, hipStream_t s);

}  // namespace fmm
