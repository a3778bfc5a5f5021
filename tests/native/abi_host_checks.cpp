// Host-side checks of the C ABI, built and run under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU: every path here
// returns before any device work (argument checks, unknown handles, the host
// SVD pseudo-inverse and the unit surface). Exits non-zero on the first
// failed expectation; the sanitizers abort on any memory or UB error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fmm.h"

static int failures = 0;
#define EXPECT(c)                                                       \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

int main() {
    fmm_options o;
    fmm_default_options(&o);
    EXPECT(o.order == 6 && o.leaf_size == 64 && o.nrhs == 1);
    fmm_default_options(nullptr);

    // unit surface: query, then fill
    int ns = 0;
    EXPECT(fmm_unit_surface(8, nullptr, &ns) == FMM_OK && ns == 296);
    std::vector<double> y(3 * ns);
    EXPECT(fmm_unit_surface(8, y.data(), &ns) == FMM_OK);
    EXPECT(fmm_unit_surface(1, y.data(), &ns) == FMM_ERR_ARG);
    EXPECT(std::strlen(fmm_last_error()) > 0);

    // pseudo-inverse of the check-from-equivalent map of order 6 (host SVD)
    int n6 = 0;
    fmm_unit_surface(6, nullptr, &n6);
    std::vector<double> y6(3 * n6), K((size_t)n6 * n6), P((size_t)n6 * n6);
    fmm_unit_surface(6, y6.data(), &n6);
    for (int i = 0; i < n6; ++i)
        for (int j = 0; j < n6; ++j) {
            double d = 0;
            for (int c = 0; c < 3; ++c) d += std::pow(2.95 * y6[3 * i + c] - 1.05 * y6[3 * j + c], 2);
            K[(size_t)i * n6 + j] = 1.0 / (4 * M_PI * std::sqrt(d));
        }
    EXPECT(fmm_pinv(K.data(), n6, 1e-12, P.data()) == FMM_OK);
    // K P K = K
    std::vector<double> KP((size_t)n6 * n6, 0.0);
    for (int i = 0; i < n6; ++i)
        for (int k = 0; k < n6; ++k)
            for (int j = 0; j < n6; ++j) KP[(size_t)i * n6 + j] += K[(size_t)i * n6 + k] * P[(size_t)k * n6 + j];
    double err = 0, nrm = 0;
    for (int i = 0; i < n6; ++i)
        for (int j = 0; j < n6; ++j) {
            double v = 0;
            for (int k = 0; k < n6; ++k) v += KP[(size_t)i * n6 + k] * K[(size_t)k * n6 + j];
            err = std::fmax(err, std::fabs(v - K[(size_t)i * n6 + j]));
            nrm = std::fmax(nrm, std::fabs(K[(size_t)i * n6 + j]));
        }
    EXPECT(err < 1e-8 * nrm);
    EXPECT(fmm_pinv(nullptr, 4, 0.0, P.data()) == FMM_ERR_ARG);
    EXPECT(fmm_pinv(K.data(), 0, 0.0, P.data()) == FMM_ERR_ARG);

    // setup argument errors (host checks before device work)
    fmm_plan plan = nullptr;
    float dummy[3] = {0, 0, 0};
    EXPECT(fmm_setup(dummy, nullptr, 1, nullptr, nullptr, 0, nullptr, nullptr, &plan) == FMM_ERR_ARG);
    EXPECT(fmm_setup(dummy, nullptr, 1, nullptr, nullptr, 0, &o, nullptr, nullptr) == FMM_ERR_ARG);
    fmm_options bad = o;
    bad.order = 11;
    EXPECT(fmm_setup(dummy, nullptr, 1, nullptr, nullptr, 0, &bad, nullptr, &plan) == FMM_ERR_ARG && !plan);
    bad = o;
    bad.nrhs = 5;
    EXPECT(fmm_setup(dummy, nullptr, 1, nullptr, nullptr, 0, &bad, nullptr, &plan) == FMM_ERR_ARG);
    bad = o;
    bad.src_kernels = FMM_SRC_DOUBLE;
    EXPECT(fmm_setup(dummy, nullptr, 1, nullptr, nullptr, 0, &bad, nullptr, &plan) == FMM_ERR_ARG);
    EXPECT(fmm_setup(nullptr, nullptr, 5, nullptr, nullptr, 0, &o, nullptr, &plan) == FMM_ERR_ARG);
    EXPECT(fmm_setup(dummy, nullptr, -1, nullptr, nullptr, 0, &o, nullptr, &plan) == FMM_ERR_ARG);
    int64_t off_bad[4] = {0, 60, 50, 100};
    EXPECT(fmm_setup_batch(3, off_bad, nullptr, dummy, nullptr, nullptr, nullptr, &o, nullptr, &plan) == FMM_ERR_ARG);
    int64_t off0[2] = {5, 100};
    EXPECT(fmm_setup_batch(1, off0, nullptr, dummy, nullptr, nullptr, nullptr, &o, nullptr, &plan) == FMM_ERR_ARG);
    EXPECT(fmm_setup_batch(0, off0, nullptr, dummy, nullptr, nullptr, nullptr, &o, nullptr, &plan) == FMM_ERR_ARG);

    // handles the library never issued
    fmm_plan bogus = reinterpret_cast<fmm_plan>(static_cast<uintptr_t>(0x1000));
    EXPECT(fmm_apply(bogus, nullptr, nullptr, nullptr, nullptr, nullptr) == FMM_ERR_ARG);
    fmm_info info;
    EXPECT(fmm_plan_info(bogus, &info) == FMM_ERR_ARG);
    EXPECT(fmm_set_graph(bogus, 1) == FMM_ERR_ARG);
    EXPECT(fmm_destroy(bogus) == FMM_ERR_ARG);
    EXPECT(fmm_destroy(nullptr) == FMM_OK);
    int it = 0;
    double rr = 0;
    fmm_operator op{FMM_OP_FK, nullptr, nullptr, nullptr};
    EXPECT(gmres_solve(bogus, &op, nullptr, nullptr, 1e-6, 30, 100, &it, &rr, nullptr) == FMM_ERR_ARG);

    // other host argument checks
    EXPECT(fmm_direct(nullptr, nullptr, -1, nullptr, 0, nullptr, nullptr, 1e-5f, nullptr, nullptr, nullptr) ==
           FMM_ERR_ARG);
    EXPECT(fmm_split_bf16(0, 100, 1, nullptr, nullptr, nullptr) == FMM_ERR_ARG);
    EXPECT(fmm_split_bf16(0, 160, 0, nullptr, nullptr, nullptr) == FMM_OK);

    if (failures) {
        std::fprintf(stderr, "%d host ABI checks failed\n", failures);
        return 1;
    }
    std::printf("host ABI checks passed\n");
    return 0;
}
