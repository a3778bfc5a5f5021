// Autotuning of the octree's leaf size (and the M2L piece count) by trial
// runs, and the on-disk cache that plans built with leaf_size = 0 consult.
//
// The paper tunes the height of its octree for each problem by trial runs
// (Sec. III.A.1 and Sec. IV.A): the height sets the balance between the near
// field and the far field. Here the leaf cap plays that role; a candidate plan
// is built for each cap in the search space, timed over a few applies on
// random densities, and the fastest is kept. Accuracy is not tuned: the
// candidates share the caller's far-field form, order and threshold.
//
// Cache: one JSON object per line,
//   {"key": "...", "leaf_size": L, "m2l_pieces": P, "ms": T}
// keyed by the device (architecture and compute units), the form (basis,
// order, threshold, M2L arithmetic), the kernels and outputs, nrhs, whether
// targets differ from sources, whether the plan is a batch, and the size
// bucket floor(log2(points per instance)). A later entry with the same key
// replaces an earlier one.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

#include "plan.hpp"

namespace fmm {

namespace {

// uniform values in [-1, 1) from a 32-bit integer hash of (seed, index)
__global__ void k_fill_random(float *out, int64_t n, uint32_t seed) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    out[i] = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
}

std::mutex g_cache_mu;

std::string json_string_field(const std::string &line, const std::string &name) {
    const std::string tag = "\"" + name + "\": \"";
    size_t a = line.find(tag);
    if (a == std::string::npos) return "";
    a += tag.size();
    size_t b = line.find('"', a);
    return b == std::string::npos ? "" : line.substr(a, b - a);
}

bool json_number_field(const std::string &line, const std::string &name, double &v) {
    const std::string tag = "\"" + name + "\": ";
    size_t a = line.find(tag);
    if (a == std::string::npos) return false;
    char *end = nullptr;
    v = std::strtod(line.c_str() + a + tag.size(), &end);
    return end != line.c_str() + a + tag.size();
}

}  // namespace

bool log_enabled() {
    static const bool on = [] {
        const char *v = std::getenv("FMM_LOG");
        return v != nullptr && *v != 0 && std::strcmp(v, "0") != 0;
    }();
    return on;
}

bool inject_alloc_failure() {
    static std::mutex mu;
    static std::string value;  // the variable's value the count belongs to
    static long count = 0;
    const char *v = std::getenv("FMM_FAULT_INJECT");
    if (v == nullptr || std::strncmp(v, "alloc:", 6) != 0) return false;
    std::lock_guard<std::mutex> lock(mu);
    if (value != v) {
        value = v;
        count = 0;
    }
    const long k = std::strtol(v + 6, nullptr, 10);
    return ++count == k;
}

void log_printf(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[fmm] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    va_end(ap);
    std::fflush(stderr);
}

std::string tune_cache_path() {
    if (const char *p = std::getenv("FMM_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/fmm_mi355x_tune.jsonl";
}

std::string tune_key(const fmm_options &o, int64_t points_per_instance, bool tsm, bool batch) {
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FMM_HIP(hipGetDeviceProperties(&prop, dev));
    const double eps = o.pinv_eps > 0 ? o.pinv_eps : default_pinv_eps(o.basis, o.order);
    const int lg = points_per_instance > 0 ? (int)std::floor(std::log2((double)points_per_instance)) : 0;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s/%dcu|basis=%d|order=%d|eps=%.3g|prec=%d|src=%d|out=%d|nrhs=%d|tsm=%d|batch=%d|log2n=%d",
                  prop.gcnArchName, prop.multiProcessorCount, o.basis, o.order, eps, o.precision, o.src_kernels,
                  o.outputs, o.nrhs, tsm ? 1 : 0, batch ? 1 : 0, lg);
    return buf;
}

bool tune_cache_lookup(const std::string &path, const std::string &key, int &leaf, int &pieces) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ifstream f(path);
    if (!f) return false;
    bool found = false;
    std::string line;
    while (std::getline(f, line)) {
        if (json_string_field(line, "key") != key) continue;
        double l = 0, p = 0;
        if (json_number_field(line, "leaf_size", l) && json_number_field(line, "m2l_pieces", p) && l >= 1 &&
            p >= 0 && p <= 8) {
            leaf = (int)l;
            pieces = (int)p;
            found = true;  // keep reading: the last entry wins
        }
    }
    return found;
}

void tune_cache_store(const std::string &path, const std::string &key, int leaf, int pieces, double ms) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line))
            if (!line.empty() && json_string_field(line, "key") != key) keep.push_back(line);
    }
    char buf[768];
    std::snprintf(buf, sizeof buf, "{\"key\": \"%s\", \"leaf_size\": %d, \"m2l_pieces\": %d, \"ms\": %.4f}",
                  key.c_str(), leaf, pieces, ms);
    keep.push_back(buf);
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        FMM_REQUIRE((bool)f, "fmm_autotune: cannot write the cache file " + tmp);
        for (const auto &l : keep) f << l << "\n";
        FMM_REQUIRE((bool)f, "fmm_autotune: writing the cache file failed");
    }
    FMM_REQUIRE(std::rename(tmp.c_str(), path.c_str()) == 0, "fmm_autotune: cannot replace the cache file " + path);
}

void fill_random(float *out, int64_t n, uint32_t seed, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_random, dim3(grid_for(n, 256)), dim3(256), 0, s, out, n, seed);
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
