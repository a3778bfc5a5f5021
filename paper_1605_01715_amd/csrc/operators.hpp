// Precomputed surfaces and translation operators for one order p.
#pragma once

#include <memory>

#include "common.hpp"

namespace fmm {

// Far-field state in compressed coordinates.
//
// With K = G(2.95 Y, 1.05 Y) = U S V^T (truncated to the r singular values
// above eps * sigma_max) the check-to-equivalent maps are
// UC2E = V S^-1 U^T and DC2E = pinv(K^T) = U S^-1 V^T. Everything the
// upward pass produces reaches the rest of the method only through U^T, and
// everything the downward check potential feeds passes through V^T, so the
// state is kept as r-vectors: ut = U^T u (upward) and dt = V^T d (downward).
// The translations then are r x r matrices, built in float64 on unit boxes:
//   m2m[o] = U^T (1/2 G(2.95 Y, s_o/2 + 0.525 Y)) V S^-1       child ut -> parent ut
//   m2l[d] = V^T G(1.05 Y, 2 d + 1.05 Y) V S^-1                 source ut -> target dt
//   l2l[o] = V^T G(s_o/2 + 0.525 Y, 2.95 Y) U S^-1              parent dt -> child dt
// with the projections pu = U^T, pv = V^T (r x n_s) for check potentials
// computed from points (P2M, P2L) and the expansions cu = V S^-1 and
// cd = U S^-1 (n_s x r) giving equivalent densities (times the box half-width).
//
// Chebyshev basis (the paper's form, Sec. III.A.1 Eq. p2m), order n: Y holds
// the n^3 tensor-product Chebyshev nodes on [-1,1]^3 (ns = n^3) and the state
// of a box is its node weights W (upward) and node values L (downward), ns
// per box. Child o's weights map to the parent's by S[o_x] (x) S[o_y] (x)
// S[o_z] with the 1D tables cheb_s1[side][i][i'] = S(x_i, -+1/2 + x_i' / 2),
// L2L by the transposes, both exact. M2L: K_d = G(x, 2 d + x) between unit boxes,
// Q (ns x r) the leading eigenvectors of sum_d K_d K_d^T, m2l[d] = Q^T K_d Q
// (r x r), pv = Q^T compresses W, cd = Q expands (times 1 / half-width).
// cheb_coef[i][k] (n x n, float64) are the Chebyshev coefficients of node
// i's Lagrange polynomial: 1/n for k = 0, (2/n) T_k(x_i) after.
enum Basis { kBasisSurface = 0, kBasisChebyshev = 1 };

struct Operators {
    int basis = kBasisSurface;
    int p = 0, ns = 0, n_pad = 0;  // surface points (or Chebyshev nodes), padded to 32
    int r = 0, r_pad = 0;          // kept singular values, padded to 32
    double eps = 0;
    std::vector<double> Y;         // [ns][3]
    DBuf<double> dY;
    DBuf<float> m2l_f32;           // [316] r_pad x r_pad float32, M2L kernel chunk order (FP32 form)
    DBuf<uint16_t> m2l_bf;         // the same, split into three bfloat16 parts (M2L kernel, bf16x6)
    DBuf<uint16_t> m2l_bf2;        // the same, split into two bfloat16 parts (bf16x3, bf16x4)
    DBuf<double> m2m_f64, l2l_f64; // [8] r_pad x r_pad, float64 fragment layout
    DBuf<double> pu_f64, pv_f64;   // r_pad x n_pad fragment layout
    DBuf<double> cu_f64, cd_f64;   // n_pad x r_pad fragment layout
    DBuf<float> pv_f32, cd_f32;    // Chebyshev basis: Q^T (r_pad x n_pad) and Q (n_pad x r_pad), to_frag_f32 order
    std::vector<double> U, V;      // host [ns][r] row-major (reconstruction for inspection)
    DBuf<double> cheb_coef;        // Chebyshev basis: [n][n]
    DBuf<double> cheb_s1;          // Chebyshev basis: [2][n][n]
};

// Chebyshev nodes of the first kind, cos((2i + 1) pi / (2n)), i = 0..n-1.
std::vector<double> chebyshev_nodes(int n);

// Unit surface Y(p): boundary nodes of the p^3 grid on [-1,1]^3, lexicographic.
std::vector<double> unit_surface(int p);

// One-sided Jacobi SVD of an n x n row-major matrix: K = U diag(s) V^T with
// s in descending order. U and V are n x n row-major.
void svd_jacobi(const std::vector<double> &K, int n, std::vector<double> &U, std::vector<double> &s,
                std::vector<double> &V);

// Truncated-SVD pseudo-inverse of an n x n row-major matrix; singular values
// below eps * sigma_max are dropped.
std::vector<double> pinv_jacobi(const std::vector<double> &K, int n, double eps);

// Cached per (device, basis, order, eps); built on first use.
std::shared_ptr<const Operators> get_operators(int basis, int p, double eps, hipStream_t s);

double default_pinv_eps(int basis, int p);

}  // namespace fmm
