// Interpolation kernels of the Chebyshev far field (Sec. III.A.1 Eq. p2m):
// sources onto the nodes of their leaf (P2M) and node values back to the
// targets of a leaf (L2P). Everything between the two is shared with the
// surface form (GEMMs on node vectors, M2L in a compressed basis, P2L and M2P
// as kernel sums at the nodes).
#pragma once

#include "nbody.hpp"

namespace fmm {

constexpr int kChebMaxOrder = 8;

// P2M: for work item i (box b = items[i], centre c, half-width h) write
//   out[(b * nrhs + r) * n_pad + m] = sum_j q_j S(xbar_m, t_j) + (m_j / h) . grad_t S(xbar_m, t_j)
// over the sources j in ranges rng[roff[i] .. roff[i+1]) (pairs s0, s1), with
// t_j = (y_j - c) / h, S the tensor product of the order-n Lagrange
// polynomials (float64 coefficients coef [n][n] in the Chebyshev basis) and nodes
// m = (i n + j) n + k. The double layer enters through the gradient of S
// (the paper's second method). g supplies centres, half-widths and n_pad.
void points_to_nodes(int nrhs, bool sl, bool dl, int n, const double *coef, const int32_t *items, int nitems,
                     const int32_t *roff, const int32_t *rng, const SurfaceGeom &g, const PointSrc &src, float *out,
                     hipStream_t s);

// L2P: for every work item of the leaf evaluation (a.wleaf / a.wt0: up to 64
// targets of one leaf) write sum_m S(xbar_m, t) L_m to a.pot and
// -(1/h) grad_t of it to a.field (user order through a.trg_perm; either may be
// NULL), where L = node values [(leaf * nrhs + r) * g.n_pad + m]. With
// a.accumulate = 1 the values are added to what is there (the plan runs the
// leaf evaluation first, on a side stream, and L2P after the join).
void nodes_to_points(int nrhs, int n, const double *coef, const EvalArgs &a, const SurfaceGeom &g, const float *L,
                     hipStream_t s);

// M2M / L2L by the tensor-product structure of the octant maps: with
// S[side][i][i'] = S(xbar_i, side / 2 + xbar_i' / 2) (side 0: -, 1: +) the map
// from child o's node weights to the parent's is S[o_x] (x) S[o_y] (x) S[o_z]
// (o_x = bit 2 of o, o_y bit 1, o_z bit 0), applied axis by axis (3 n^4
// FMAs instead of n^6). One wave per item:
//   M2M (l2l = false): out[dst[i]] = sum_{o < 8, src[8 i + o] >= 0} M_o in[src[8 i + o]]
//   L2L (l2l = true):  out[dst[i]] += M_{oct[i]}^T in[src[i]]
// Vectors are rows [(box * nrhs + r) * n_pad + m], s1 is [2][n][n] float64;
// arithmetic is float64.
void cheb_tensor(int nrhs, int n, bool l2l, const double *s1, int nitems, const int32_t *dst, const int32_t *src,
                 const int8_t *oct, const float *in, float *out, int n_pad, hipStream_t s);

}  // namespace fmm
