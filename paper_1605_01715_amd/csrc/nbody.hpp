// n-body shaped kernels: kernel sums between point sets and box surfaces.
#pragma once

#include "common.hpp"

namespace fmm {

// Sorted sources: coordinates and, per right-hand side r, the single-layer
// density q[r * n + j] and the double-layer dipole m = mu n (mx, my, mz).
struct PointSrc {
    const float *x = nullptr, *y = nullptr, *z = nullptr;
    const float *q = nullptr;
    const float *mx = nullptr, *my = nullptr, *mz = nullptr;
    int64_t n = 0;
};

struct SurfaceGeom {
    const double *Y = nullptr;  // [ns][3] unit surface
    int ns = 0, n_pad = 0;
    const double *centre = nullptr, *half = nullptr;
};

// P2M / P2L: for work item i (box items[i]) accumulate into
// out[(items[i] * nrhs + r) * n_pad + m] the potential of the sources in ranges
// rng[roff[i] .. roff[i+1]) (pairs s0, s1) at the surface points
// centre + rfac * half * Y_m.
void points_to_surface(int nrhs, bool sl, bool dl, const int32_t *items, int nitems, const int32_t *roff,
                       const int32_t *rng, double rfac, const SurfaceGeom &g, const PointSrc &src, float *out,
                       bool accumulate, hipStream_t s);

// Leaf evaluation (L2P + M2P + P2P). Work item i is leaf wleaf[i] with targets
// [tbeg + wt0[i], min(tbeg + wt0[i] + 64, tend)). Surface sources of a leaf are
// the entries sbox/skind[soff[leaf] .. soff[leaf+1]) (kind 0: the downward
// equivalent density phi_d of that box at radius rad_down, kind 1: the upward
// density phi_u at radius rad_up, both times the box half-width and around
// its centre; for the surface form 2.95 and 1.05, for the Chebyshev form
// the node weights at the nodes, radius 1); point sources are the ranges
// prng[poff[leaf] .. poff[leaf+1]). Results go to pot[r * n_trg + perm[k]] and
// field[(r * n_trg + perm[k]) * 3 + c] (user order), overwriting (accumulate =
// 0) or added to what is there (accumulate = 1).
struct EvalArgs {
    const int32_t *wleaf = nullptr, *wt0 = nullptr;
    int nwork = 0;
    const int32_t *soff = nullptr, *sbox = nullptr;
    const int8_t *skind = nullptr;
    const int32_t *poff = nullptr, *prng = nullptr;
    const int32_t *pmid = nullptr;  // per box: ranges [poff, pmid) need the r < delta test (NULL: all)
    const int64_t *tbeg = nullptr, *tend = nullptr;
    const float *tx = nullptr, *ty = nullptr, *tz = nullptr;
    const int64_t *trg_perm = nullptr;  // NULL: identity
    int64_t n_trg = 0;
    const float *phi_d = nullptr, *phi_u = nullptr;
    double rad_down = 0.0, rad_up = 0.0;
    float delta2 = 0.f;
    float *pot = nullptr, *field = nullptr;
    int accumulate = 0;
    int surf_mask = 3;  // surface kinds evaluated: bit 0 kind 0 (phi_d), bit 1 kind 1 (phi_u)
    int points = 1;     // 0: skip the point ranges (surfaces only)
};
void eval_leaves(int nrhs, bool sl, bool dl, const EvalArgs &a, const SurfaceGeom &g, const PointSrc &src,
                 hipStream_t s);

// All pairs, no tree: pot[i] = sum_j K(x_i, y_j), field likewise (nrhs = 1).
void direct_all_pairs(const float *trg, int64_t n_trg, const float *src, const float *nrm, int64_t n_src,
                      const float *q, const float *mu, float delta, float *pot, float *field, hipStream_t s);

}  // namespace fmm
