// Precomputed surfaces and translation operators for one order p.
#pragma once

#include <memory>

#include "common.hpp"

namespace fmm {

// All matrices act on check potentials (the well-conditioned quantities) and
// are built in float64 from the unit-box geometry, then stored in the
// fragment layouts of gemm.hip:
//   m2m[o]  = 1/2 G(2.95 Y, s_o/2 + 0.525 Y) UC2E          child check -> parent check
//   m2l[d]  = G(1.05 Y, 2 d + 1.05 Y) UC2E                  source up-check -> target down-check
//   l2l[o]  = G(s_o/2 + 0.525 Y, 2.95 Y) DC2E               parent down-check -> child down-check
//   uc2e, dc2e                                               check -> equivalent density (float64)
// with UC2E = pinv(G(2.95 Y, 1.05 Y)) and DC2E = pinv(G(1.05 Y, 2.95 Y)) = UC2E^T.
struct Operators {
    int p = 0, ns = 0, n_pad = 0;
    double eps = 0;
    std::vector<double> Y;  // [ns][3]
    DBuf<double> dY;
    DBuf<float> m2l_f32;
    DBuf<double> m2m_f64, l2l_f64;  // M2M and L2L run in float64 (cheap, and they feed every M2L)
    DBuf<uint16_t> m2l_bf;  // 316 matrices x 3 parts
    DBuf<double> uc2e_f64, dc2e_f64;
    size_t mat_elems = 0;   // n_pad * n_pad
    std::vector<double> uc2e_host;  // [ns][ns] row-major (float64)
};

// Unit surface Y(p): boundary nodes of the p^3 grid on [-1,1]^3, lexicographic.
std::vector<double> unit_surface(int p);

// Truncated-SVD pseudo-inverse (one-sided Jacobi SVD, float64) of an n x n
// row-major matrix; singular values below eps * sigma_max are dropped.
std::vector<double> pinv_jacobi(const std::vector<double> &K, int n, double eps);

// Cached per (device, p, eps); built on first use.
std::shared_ptr<const Operators> get_operators(int p, double eps, hipStream_t s);

double default_pinv_eps(int p);

}  // namespace fmm
