// Work lists and the apply pipeline of one FMM evaluation.
//
// Upward pass: P2M at the leaves (check potentials from points, projected
// onto the compressed basis), M2M level by level towards the root.
// Far-field translation: M2L over the V lists, P2L over the X lists (again
// projected). Downward pass: L2L level by level towards the leaves, then the
// expansions to equivalent densities in float64. Evaluation: one fused kernel
// per leaf adds L2P, M2P (W lists) and the near field (U lists and the direct
// W/X pairs) and writes the results in the caller's order.
//
// Paper-silent reading: a W or X partner holding at most n_s points is
// evaluated directly rather than through a surface (this never changes what
// is computed, only how).
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <limits>
#include <queue>

#include "plan.hpp"

#include "chebyshev.hpp"

namespace fmm {

namespace {

constexpr int kBlock = 256;

// plain fill (a memset node does not replay reliably inside captured graphs)
// Tight bounding boxes of the points of listed boxes: one wave per box,
// out[6 b .. 6 b + 5] = min x, y, z, max x, y, z over [beg[box], end[box]).
__global__ __launch_bounds__(64) void k_point_boxes(const int32_t *boxes, const int64_t *beg, const int64_t *end,
                                                    const float *x, const float *y, const float *z, float *out) {
    const int b = blockIdx.x, lane = threadIdx.x;
    const int32_t box = boxes[b];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = beg[box] + lane; i < end[box]; i += 64) {
        const float v[3] = {x[i], y[i], z[i]};
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], v[c]);
            hi[c] = fmaxf(hi[c], v[c]);
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], __shfl_xor(lo[c], o));
            hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], o));
        }
    if (lane == 0)
        for (int c = 0; c < 3; ++c) {
            out[6 * b + c] = lo[c];
            out[6 * b + 3 + c] = hi[c];
        }
}

constexpr int kMaskWords = (kNumDirs + 63) / 64;

// The order in which a tile runs its directions. The targets of a tile share
// one octant, hence one parity per axis, so the sources of two directions
// overlap only when the offsets differ by even amounts in every axis. The
// offsets are therefore grouped by parity class and, within a class, visited
// in a boustrophedon over (i, j, k) with steps of two, so that consecutive
// directions mostly differ by 2 along one axis and the kernel's consecutive
// steps (one k-chunk of every direction, then the next chunk) re-read most
// of the previous step's source chunks from L2.
const std::vector<int> &m2l_direction_order() {
    static const std::vector<int> order = [] {
        int idx[7][7][7];
        int k = 0;
        for (int i = -3; i <= 3; ++i)
            for (int j = -3; j <= 3; ++j)
                for (int l = -3; l <= 3; ++l)
                    idx[i + 3][j + 3][l + 3] =
                        std::max(std::abs(i), std::max(std::abs(j), std::abs(l))) >= 2 ? k++ : -1;
        std::vector<int> out;
        for (int cls = 0; cls < 8; ++cls) {
            const int pi = cls >> 2, pj = (cls >> 1) & 1, pl = cls & 1;
            bool flip_j = false, flip_l = false;
            for (int i = -3; i <= 3; ++i) {
                if ((i & 1) != pi) continue;
                for (int jj = 0; jj < 7; ++jj) {
                    const int j = flip_j ? 3 - jj : jj - 3;
                    if ((j & 1) != pj) continue;
                    for (int ll = 0; ll < 7; ++ll) {
                        const int l = flip_l ? 3 - ll : ll - 3;
                        if ((l & 1) != pl) continue;
                        if (idx[i + 3][j + 3][l + 3] >= 0) out.push_back(idx[i + 3][j + 3][l + 3]);
                    }
                    flip_l = !flip_l;
                }
                flip_j = !flip_j;
            }
        }
        return out;
    }();
    return order;
}

// Host wall time since the previous call (or construction), logged with FMM_LOG.
struct Lap {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    void operator()(const char *what) {
        const auto now = std::chrono::steady_clock::now();
        FMM_LOG("setup: %s %.2f ms\n", what, std::chrono::duration<double, std::milli>(now - t0).count());
        t0 = now;
    }
};

// Per box b, bit 63 - d % 64 of out[b * kMaskWords + d / 64] is set when the
// V partner in direction d exists and holds sources.
__global__ void k_dir_masks(const int32_t *vdense, int64_t nb, const int64_t *sbeg, const int64_t *send,
                            uint64_t *out) {
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    for (int w = 0; w < kMaskWords; ++w) {
        uint64_t m = 0;
        for (int i = 0; i < 64 && w * 64 + i < kNumDirs; ++i) {
            const int32_t a = vdense[b * kNumDirs + w * 64 + i];
            if (a >= 0 && send[a] > sbeg[a]) m |= 1ull << (63 - i);
        }
        out[b * kMaskWords + w] = m;
    }
}

// M2L sources: for step e (work item item[e], direction dir[e]) and column c
// with target vector v = cols[item[e] * nc + c] (box v / nrhs, rhs v % nrhs),
// out[e * nc + c] = a * nrhs + v % nrhs for the V partner a of that box in
// that direction when it holds sources, else -1.
__global__ void k_m2l_sources(const int32_t *item, const int32_t *dir, int64_t nsteps, const int32_t *cols, int nc,
                              const int32_t *vdense, const int64_t *sbeg, const int64_t *send, int nrhs,
                              int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nsteps * nc) return;
    const int64_t e = i / nc;
    const int c = (int)(i - e * nc);
    const int32_t v = cols[(int64_t)item[e] * nc + c];
    int32_t sv = -1;
    if (v >= 0) {
        const int32_t a = vdense[(int64_t)(v / nrhs) * kNumDirs + dir[e]];
        if (a >= 0 && send[a] > sbeg[a]) sv = a * nrhs + v % nrhs;
    }
    out[i] = sv;
}

__global__ void k_zero(float *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Both layers: the two densities side by side first (coalesced), so that the
// gather into tree order below fetches one 8-byte pair per point from a
// random place instead of two 4-byte values from two (the caller's order is
// arbitrary, so every such fetch moves a whole cache line).
__global__ void k_pair_densities(int64_t total, const float *q, const float *mu, float2 *qm) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < total) qm[i] = make_float2(q[i], mu[i]);
}

__global__ void k_sort_density_pairs(const int64_t *perm, int64_t n, int nrhs, const float2 *qm, const float *nx,
                                     const float *ny, const float *nz, float *qs, float *mx, float *my, float *mz) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t o = perm[i];
    for (int r = 0; r < nrhs; ++r) {
        const float2 v = qm[r * n + o];
        qs[r * n + i] = v.x;
        mx[r * n + i] = v.y * nx[i];
        my[r * n + i] = v.y * ny[i];
        mz[r * n + i] = v.y * nz[i];
    }
}

__global__ void k_sort_densities(const int64_t *perm, int64_t n, int nrhs, const float *q, const float *mu,
                                 const float *nx, const float *ny, const float *nz, float *qs, float *mx, float *my,
                                 float *mz) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t o = perm[i];
    for (int r = 0; r < nrhs; ++r) {
        if (q) qs[r * n + i] = q[r * n + o];
        if (mu) {
            float m = mu[r * n + o];
            mx[r * n + i] = m * nx[i];
            my[r * n + i] = m * ny[i];
            mz[r * n + i] = m * nz[i];
        }
    }
}

// Pack output-vector lists into tiles of `ncol` columns; vector index = box * nrhs + r.
std::vector<int32_t> tile_columns(const std::vector<int32_t> &boxes, int nrhs, int ncol, int &ntile) {
    std::vector<int32_t> cols;
    for (int32_t b : boxes)
        for (int r = 0; r < nrhs; ++r) cols.push_back(b * nrhs + r);
    ntile = (int)((cols.size() + ncol - 1) / ncol);
    cols.resize((size_t)ntile * ncol, -1);
    return cols;
}

void add_range(std::vector<int32_t> &rng, int64_t s0, int64_t s1) {
    if (s1 <= s0) return;
    rng.push_back((int32_t)s0);
    rng.push_back((int32_t)s1);
}

// sort ranges by start and merge touching ones
void merge_ranges(std::vector<int32_t> &r, size_t from) {
    size_t n = (r.size() - from) / 2;
    if (n < 2) return;
    std::vector<std::pair<int32_t, int32_t>> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = {r[from + 2 * i], r[from + 2 * i + 1]};
    std::sort(v.begin(), v.end());
    r.resize(from);
    int32_t a = v[0].first, b = v[0].second;
    for (size_t i = 1; i < n; ++i) {
        if (v[i].first == b) {
            b = v[i].second;
        } else {
            r.push_back(a);
            r.push_back(b);
            a = v[i].first;
            b = v[i].second;
        }
    }
    r.push_back(a);
    r.push_back(b);
}

}  // namespace

void plan_build_worklists(Plan &P, hipStream_t s) {
    auto clock0 = std::chrono::steady_clock::now();
    auto phase_end = [&](int k) {
        FMM_HIP(hipStreamSynchronize(s));
        const auto now = std::chrono::steady_clock::now();
        P.setup_phase_ms[k] += std::chrono::duration<double, std::milli>(now - clock0).count();
        clock0 = now;
    };
    Tree &t = P.t;
    Lap wl;
    const int64_t nb = t.nb;
    const int nrhs = P.nrhs, ns = P.ns;
    auto nsrc = [&](int64_t b) { return t.h_send[b] - t.h_sbeg[b]; };
    auto ntrg = [&](int64_t b) { return t.h_tend[b] - t.h_tbeg[b]; };
    auto leaf = [&](int64_t b) { return t.h_leaf[b] != 0; };
    auto lvl = [&](int64_t b) { return t.h_level[b]; };
    const auto &U = t.U, &W = t.W, &X = t.X;

    // per-vector scale = box half-width (check-to-equivalent maps)
    {
        std::vector<double> sc((size_t)nb * nrhs);
        for (int64_t b = 0; b < nb; ++b)
            for (int r = 0; r < nrhs; ++r) sc[b * nrhs + r] = t.h_half[b];
        P.col_scale = upload(sc, s);
    }

    // P2M
    {
        std::vector<int32_t> items, roff{0}, rng;
        for (int64_t b = 0; b < nb; ++b)
            if (leaf(b) && lvl(b) >= 2 && nsrc(b) > 0) {
                items.push_back((int32_t)b);
                add_range(rng, t.h_sbeg[b], t.h_send[b]);
                roff.push_back((int32_t)(rng.size() / 2));
                P.p2m_evals += nsrc(b) * ns;
            }
        P.n_p2m = (int)items.size();
        P.p2m_items = upload(items, s);
        P.p2m_roff = upload(roff, s);
        P.p2m_rng = upload(rng, s);
        GemmJob &j = P.p2m_proj;
        std::vector<int32_t> cols = tile_columns(items, nrhs, kGemmCols, j.ntile);
        j.nterm = 1;
        j.cols = upload(cols, s);
        j.src = upload(cols, s);
    }

    wl("scales and P2M lists");
    const int ncol64 = kGemmCols;
    // M2M, bottom-up (float64 tiles)
    for (int l = t.nlev - 2; l >= 2; --l) {
        std::vector<int32_t> boxes;
        for (int64_t b = t.lvl_off[l]; b < t.lvl_off[l + 1]; ++b)
            if (!leaf(b) && nsrc(b) > 0) boxes.push_back((int32_t)b);
        if (boxes.empty()) continue;
        GemmJob j;
        std::vector<int32_t> cols = tile_columns(boxes, nrhs, ncol64, j.ntile);
        j.nterm = 8;
        std::vector<int32_t> src((size_t)j.ntile * 8 * ncol64, -1);
        for (int tl = 0; tl < j.ntile; ++tl)
            for (int c = 0; c < ncol64; ++c) {
                int32_t v = cols[(size_t)tl * ncol64 + c];
                if (v < 0) continue;
                int32_t box = v / nrhs, r = v % nrhs;
                for (int o = 0; o < 8; ++o) {
                    int32_t ch = t.h_child[8 * (size_t)box + o];
                    if (ch >= 0 && nsrc(ch) > 0) src[((size_t)tl * 8 + o) * ncol64 + c] = ch * nrhs + r;
                }
            }
        j.cols = upload(cols, s);
        j.src = upload(src, s);
        P.m2m_jobs.push_back(std::move(j));
    }

    wl("M2M lists");
    phase_end(6);
    // M2L: every target box at level >= 2 with at least one V partner holding sources
    {
        Lap lap;
        // per box, the directions whose V partner holds sources, as a bit mask
        // (direction d is bit 63 - d % 64 of word d / 64, so that comparing the
        // words in order compares the sets lexicographically)
        std::vector<uint64_t> mask((size_t)nb * kMaskWords);
        {
            DBuf<uint64_t> dm(mask.size());
            hipLaunchKernelGGL(k_dir_masks, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.vdense.p, nb,
                               t.sbeg.p, t.send.p, dm.p);
            FMM_HIP(hipGetLastError());
            d2h(mask.data(), dm.p, mask.size(), s);
        }
        lap("m2l direction masks");
        auto mask_of = [&](int64_t b) { return &mask[(size_t)b * kMaskWords]; };
        std::vector<int32_t> boxes;
        for (int64_t b = 0; b < nb; ++b) {
            if (lvl(b) < 2 || ntrg(b) == 0) continue;
            int64_t live = 0;
            for (int w = 0; w < kMaskWords; ++w) live += __builtin_popcountll(mask_of(b)[w]);
            if (live) {
                boxes.push_back((int32_t)b);
                P.m2l_pairs += live;
            }
        }
        FMM_REQUIRE(m2l_supported(P.r_pad), "M2L: unsupported compressed state size");
        lap("m2l target boxes");
        // Tiles of m2l_ncol output vectors, each with its list of active
        // directions. A box's V-list offsets are fixed by its octant inside
        // its parent (189 of the 316), so tiles hold one octant only: the
        // directions a tile runs are then (nearly) the ones every column needs.
        const int nc = m2l_ncol(P.r_pad);
        int ntile = 0;
        std::vector<int32_t> cols;
        std::vector<int> tile_oct;  // octant of each tile
        // Within an octant, boxes are ordered by their set of active
        // directions (lexicographically, then by index), so a tile gathers
        // boxes with similar V lists and runs few directions that most of its
        // columns do not need (measured: fill 0.69 -> 0.78 on the clustered
        // cloud, worth more than the spatial locality it gives up).
        for (int o = 0; o < 8; ++o) {
            std::vector<std::pair<std::array<uint64_t, kMaskWords>, int32_t>> keyed;
            for (int32_t b : boxes) {
                const int32_t *an = &t.h_anchor[3 * (size_t)b];
                if ((((an[0] & 1) << 2) | ((an[1] & 1) << 1) | (an[2] & 1)) != o) continue;
                std::array<uint64_t, kMaskWords> m;
                std::copy(mask_of(b), mask_of(b) + kMaskWords, m.begin());
                keyed.push_back({m, b});
            }
            std::sort(keyed.begin(), keyed.end());
            std::vector<int32_t> grp;
            for (auto &kb : keyed) grp.push_back(kb.second);
            int nt = 0;
            std::vector<int32_t> c = tile_columns(grp, nrhs, nc, nt);
            cols.insert(cols.end(), c.begin(), c.end());
            ntile += nt;
            tile_oct.insert(tile_oct.end(), nt, o);
        }
        lap("m2l tiles");
        // per tile and direction, the columns with a source there
        std::vector<int32_t> tcnt((size_t)ntile * kNumDirs, 0);
#pragma omp parallel for schedule(dynamic, 8)
        for (int tl = 0; tl < ntile; ++tl) {
            int32_t *cnt = &tcnt[(size_t)tl * kNumDirs];
            for (int c = 0; c < nc; ++c) {
                const int32_t v = cols[(size_t)tl * nc + c];
                if (v < 0) continue;
                const uint64_t *m = mask_of(v / nrhs);
                for (int w = 0; w < kMaskWords; ++w)
                    for (uint64_t bits = m[w]; bits; bits &= bits - 1) ++cnt[w * 64 + 63 - __builtin_ctzll(bits)];
            }
        }
        lap("m2l direction counts");
        // A tile's directions are run in the order of m2l_direction_order():
        // by parity class, so that the sources of consecutive directions
        // (the tile's targets shifted by the two offsets) overlap
        const std::vector<int> &dorder = m2l_direction_order();
        std::vector<int64_t> toff{0};
        std::vector<int32_t> tdir;
        for (int tl = 0; tl < ntile; ++tl) {
            for (int d : dorder)
                if (tcnt[(size_t)tl * kNumDirs + d]) tdir.push_back(d);
            toff.push_back((int64_t)tdir.size());
        }
        // Sparse tiles become pair tiles. Where boxes have few and varied V
        // partners (points on surfaces), a tile runs every direction for
        // only a fraction of its columns (fill 0.2-0.3 on the sphere
        // workloads). The (direction, target) pairs of tiles with fill below
        // kPairFill are regrouped by octant and direction into tiles of one
        // direction whose columns are pairs, all live; each writes its
        // products to a partial-sum slot, and a gather adds each target's
        // partials in direction order. Costs: a tile does 6 steps per
        // direction; a pair tile 6 steps plus writing and reading back its
        // partials. Measured: with the threshold at 0.45 instead of 0.6 the
        // 4M-point cloud's apply is 4% faster (its tiles between the two
        // fills are cheaper as tiles), and the sphere workloads, whose sparse
        // tiles sit near fill 0.2-0.3, are unchanged.
        lap("m2l direction lists");
        constexpr double kPairFill = 0.45;
        std::vector<uint8_t> pair_tile(ntile, 0);
        {
            // the columns of the sparse tiles, per octant
            std::vector<std::vector<int32_t>> sparse(8);
            std::vector<uint8_t> keep(ntile, 1);
            bool moved = false;
            for (int tl = 0; tl < ntile; ++tl) {
                const int64_t n = toff[tl + 1] - toff[tl];
                int64_t live = 0;
                for (int d = 0; d < kNumDirs; ++d) live += tcnt[(size_t)tl * kNumDirs + d];
                if (n == 0 || (double)live >= kPairFill * (double)n * nc) continue;
                keep[tl] = 0;
                moved = true;
                for (int c = 0; c < nc; ++c) {
                    const int32_t v = cols[(size_t)tl * nc + c];
                    if (v >= 0) sparse[tile_oct[tl]].push_back(v);
                }
            }
            if (moved) {
                std::vector<int64_t> toff2{0};
                std::vector<int32_t> tdir2, cols2;
                std::vector<int> oct2;
                std::vector<uint8_t> pair2;
                for (int tl = 0; tl < ntile; ++tl) {
                    if (!keep[tl]) continue;
                    tdir2.insert(tdir2.end(), tdir.begin() + toff[tl], tdir.begin() + toff[tl + 1]);
                    toff2.push_back((int64_t)tdir2.size());
                    cols2.insert(cols2.end(), cols.begin() + (size_t)tl * nc, cols.begin() + (size_t)(tl + 1) * nc);
                    oct2.push_back(tile_oct[tl]);
                    pair2.push_back(0);
                }
                // per octant (in parallel), the (direction, target) pairs ordered
                // by direction, then target: a counting sort over the directions
                // of the targets taken in increasing order
                std::vector<std::vector<int32_t>> pdir(8), pcols(8);
#pragma omp parallel for schedule(dynamic, 1)
                for (int o = 0; o < 8; ++o) {
                    std::vector<int32_t> &sv = sparse[o];
                    std::sort(sv.begin(), sv.end());
                    std::vector<int64_t> start(kNumDirs + 1, 0);
                    for (int32_t v : sv) {
                        const uint64_t *m = mask_of(v / nrhs);
                        for (int w = 0; w < kMaskWords; ++w)
                            for (uint64_t bits = m[w]; bits; bits &= bits - 1)
                                ++start[w * 64 + 63 - __builtin_ctzll(bits) + 1];
                    }
                    for (int d = 0; d < kNumDirs; ++d) start[d + 1] += start[d];
                    std::vector<int32_t> by_dir(start[kNumDirs]);
                    std::vector<int64_t> pos(start.begin(), start.end() - 1);
                    for (int32_t v : sv) {
                        const uint64_t *m = mask_of(v / nrhs);
                        for (int w = 0; w < kMaskWords; ++w)
                            for (uint64_t bits = m[w]; bits; bits &= bits - 1)
                                by_dir[pos[w * 64 + 63 - __builtin_ctzll(bits)]++] = v;
                    }
                    for (int d = 0; d < kNumDirs; ++d)
                        for (int64_t i = start[d]; i < start[d + 1]; i += nc) {
                            const int64_t j = std::min(start[d + 1], i + nc);
                            pdir[o].push_back(d);
                            for (int64_t q = i; q < i + nc; ++q) pcols[o].push_back(q < j ? by_dir[q] : -1);
                        }
                }
                for (int o = 0; o < 8; ++o) {
                    for (int32_t d : pdir[o]) {
                        tdir2.push_back(d);
                        toff2.push_back((int64_t)tdir2.size());
                        oct2.push_back(o);
                        pair2.push_back(1);
                    }
                    cols2.insert(cols2.end(), pcols[o].begin(), pcols[o].end());
                }
                toff.swap(toff2);
                tdir.swap(tdir2);
                cols.swap(cols2);
                tile_oct.swap(oct2);
                pair_tile.swap(pair2);
                ntile = (int)pair_tile.size();
            }
        }
        // Launch order: the kernel gives XCD x the x-th eighth of the work
        // items. XCD x runs the tiles of octant x: they draw on the same 189
        // directions in the same order, so tiles running at the same time
        // share the matrices in that XCD's L2 (measured: 23% less traffic
        // beyond L2 than an even mix of octants).
        //
        // Balance: an XCD holds about 87 tiles (at 4M points) for 32 CUs, so
        // whole tiles leave a tail (a simulated 89% of the ideal time). A
        // tile's active directions are therefore cut into k contiguous
        // pieces, k the same for all tiles and chosen by simulating the
        // dispatch (pieces heaviest first, each started on the first free
        // workgroup slot) for k = 1..6 unless the options force k. Pieces of a cut tile write partial
        // sums, added to the output in piece order by a second kernel.
        {
            const int slots = 32 * m2l_blocks_per_cu(P.m2l_form, P.r_pad);  // concurrent workgroups per XCD
            auto ndir = [&](int tl) { return (int)(toff[tl + 1] - toff[tl]); };
            // makespan of one XCD in steps, with a cost of 2 directions per piece of a cut tile
            std::vector<std::vector<int>> tiles_of(8);
            for (int tl = 0; tl < ntile; ++tl) tiles_of[tile_oct[tl]].push_back(tl);
            auto makespan = [&](int k) {
                double worst = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst)
                for (int x = 0; x < 8; ++x) {
                    std::vector<double> w;
                    for (int tl : tiles_of[x]) {
                        const int kk = std::min(k, ndir(tl));
                        for (int q = 0; q < kk; ++q) w.push_back((double)ndir(tl) / kk + (kk > 1 ? 2.0 : 0.0));
                    }
                    std::sort(w.begin(), w.end(), std::greater<double>());
                    std::priority_queue<double, std::vector<double>, std::greater<double>> busy;
                    for (int q = 0; q < slots; ++q) busy.push(0.0);
                    double end = 0.0;
                    for (double v : w) {
                        const double t0 = busy.top();
                        busy.pop();
                        busy.push(t0 + v);
                        end = std::max(end, t0 + v);
                    }
                    worst = std::max(worst, end);
                }
                return worst;
            };
            int kbest = P.opt.m2l_pieces;  // forced, or 0: simulated
            if (kbest == 0) {
                kbest = 1;
                double best = makespan(1);
                for (int k = 2; k <= 6; ++k) {
                    const double m = makespan(k);
                    if (m < best * 0.995) {
                        best = m;
                        kbest = k;
                    }
                }
            }
            lap("m2l pair tiles and piece model");
            P.m2l_pieces_per_tile = kbest;
            // pieces: (tile, first direction, last direction + 1, partial slot or -1)
            struct Piece {
                int tile, e0, e1, slot;
            };
            std::vector<std::vector<Piece>> per_oct(8);
            std::vector<int32_t> red_cols, red_slot0, red_k;
            struct GatherE {
                int32_t v, dir, idx;  // target vector, direction, partial row slot * nc + column
            };
            std::vector<GatherE> gather;
            int nslot = 0;
            for (int tl = 0; tl < ntile; ++tl) {
                const int n = ndir(tl), kk = std::max(1, std::min(kbest, n));
                if (n == 0) continue;
                if (pair_tile[tl]) {  // one direction, its own slot, summed by the gather
                    const int slot = nslot++;
                    for (int c = 0; c < nc; ++c) {
                        const int32_t v = cols[(size_t)tl * nc + c];
                        if (v >= 0) gather.push_back({v, tdir[toff[tl]], slot * nc + c});
                    }
                    per_oct[tile_oct[tl]].push_back({tl, (int)toff[tl], (int)toff[tl + 1], slot});
                    continue;
                }
                const int slot0 = kk > 1 ? nslot : -1;
                if (kk > 1) {
                    red_cols.insert(red_cols.end(), cols.begin() + (size_t)tl * nc, cols.begin() + (size_t)(tl + 1) * nc);
                    red_slot0.push_back(slot0);
                    red_k.push_back(kk);
                    nslot += kk;
                }
                for (int q = 0; q < kk; ++q)
                    per_oct[tile_oct[tl]].push_back(
                        {tl, (int)toff[tl] + n * q / kk, (int)toff[tl] + n * (q + 1) / kk, kk > 1 ? slot0 + q : -1});
            }
            size_t len = 0;
            for (auto &v : per_oct) {
                std::stable_sort(v.begin(), v.end(), [](const Piece &x, const Piece &y) { return x.e1 - x.e0 > y.e1 - y.e0; });
                len = std::max(len, v.size());
            }
            // work item x * len + k is piece k of octant x (empty past the
            // octant's last piece); each octant's block is filled in parallel
            std::vector<int64_t> sbase(9, 0);
            for (int x = 0; x < 8; ++x) {
                int64_t n = 0;
                for (const Piece &pc : per_oct[x]) n += pc.e1 - pc.e0;
                sbase[x + 1] = sbase[x] + n;
            }
            std::vector<int64_t> toff2(8 * len + 1, 0);
            std::vector<int32_t> tdir2(sbase[8]), cols2(8 * len * (size_t)nc, -1), slot2(8 * len, -1);
#pragma omp parallel for schedule(dynamic, 1)
            for (int x = 0; x < 8; ++x) {
                int64_t e = sbase[x];
                for (size_t k = 0; k < len; ++k) {
                    const size_t item = (size_t)x * len + k;
                    if (k < per_oct[x].size()) {
                        const Piece &pc = per_oct[x][k];
                        std::copy(tdir.begin() + pc.e0, tdir.begin() + pc.e1, tdir2.begin() + e);
                        e += pc.e1 - pc.e0;
                        std::copy(cols.begin() + (size_t)pc.tile * nc, cols.begin() + (size_t)(pc.tile + 1) * nc,
                                  cols2.begin() + item * nc);
                        slot2[item] = pc.slot;
                    }
                    toff2[item + 1] = e;
                }
            }
            toff.swap(toff2);
            tdir.swap(tdir2);
            cols.swap(cols2);
            ntile = (int)(8 * len);
            lap("m2l pieces");
            P.m2l_slot = upload(slot2, s);
            P.m2l_nsplit = (int)red_k.size();
            if (nslot > 0) P.m2l_partial.alloc((size_t)nslot * nc * P.r_pad);
            if (P.m2l_nsplit > 0) {
                P.m2l_red_cols = upload(red_cols, s);
                P.m2l_red_slot0 = upload(red_slot0, s);
                P.m2l_red_k = upload(red_k, s);
            }
            // pair tiles: per target vector, its partial rows in direction
            // order. A target's pair tiles were made from its octant's pairs
            // in increasing direction, so they were met in that order above,
            // and a stable counting sort by target keeps it.
            std::vector<int32_t> gt, goff{0}, gidx(gather.size());
            {
                const int64_t nvec = nb * nrhs;
                std::vector<int32_t> gstart(nvec + 1, 0);
                for (const GatherE &g : gather) ++gstart[g.v + 1];
                for (int64_t v = 0; v < nvec; ++v) {
                    if (gstart[v + 1]) {
                        gt.push_back((int32_t)v);
                        goff.push_back(gstart[v] + gstart[v + 1]);
                    }
                    gstart[v + 1] += gstart[v];
                }
                for (const GatherE &g : gather) gidx[gstart[g.v]++] = g.idx;
            }
            lap("m2l slots and gather lists");
            P.m2l_ngather = (int)gt.size();
            P.m2l_pair_tiles = (int)std::count(pair_tile.begin(), pair_tile.end(), 1);
            if (P.m2l_ngather > 0) {
                P.m2l_gt = upload(gt, s);
                P.m2l_goff = upload(goff, s);
                P.m2l_gidx = upload(gidx, s);
            }
        }
        lap("m2l uploads");
        P.m2l_ntile = ntile;
        P.m2l_steps = (int64_t)tdir.size();
        P.m2l_ncol = nc;
        P.m2l_toff = upload(toff, s);
        P.m2l_dir = upload(tdir, s);
        P.m2l_cols = upload(cols, s);
        // the source vector of every (step, column), filled on the device
        {
            std::vector<int32_t> item(tdir.size());
            for (int k = 0; k < ntile; ++k)
                std::fill(item.begin() + toff[k], item.begin() + toff[k + 1], (int32_t)k);
            DBuf<int32_t> ditem = upload(item, s);
            P.m2l_src.alloc(tdir.size() * (size_t)nc);
            const int64_t n = (int64_t)tdir.size() * nc;
            if (n > 0) {
                hipLaunchKernelGGL(k_m2l_sources, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, ditem.p,
                                   P.m2l_dir.p, (int64_t)tdir.size(), P.m2l_cols.p, nc, t.vdense.p, t.sbeg.p,
                                   t.send.p, nrhs, P.m2l_src.p);
                FMM_HIP(hipGetLastError());
            }
            FMM_HIP(hipStreamSynchronize(s));
        }
        P.m2l_zero = upload(std::vector<float>(48, 0.f), s);
        lap("m2l sources");
    }
    phase_end(5);
    wl("M2L schedule");

    // P2L (X lists of boxes holding more than n_s targets)
    {
        std::vector<int32_t> items, roff{0}, rng;
        for (int64_t b = 0; b < nb; ++b) {
            if (ntrg(b) <= ns) continue;
            size_t from = rng.size();
            for (int32_t k = X.h_off[b]; k < X.h_off[b + 1]; ++k) {
                int32_t a = X.h_idx[k];
                add_range(rng, t.h_sbeg[a], t.h_send[a]);
            }
            if (rng.size() == from) continue;
            merge_ranges(rng, from);
            for (size_t e = from; e < rng.size(); e += 2) P.p2l_evals += (int64_t)(rng[e + 1] - rng[e]) * ns;
            items.push_back((int32_t)b);
            roff.push_back((int32_t)(rng.size() / 2));
        }
        P.n_p2l = (int)items.size();
        if (P.cheb) {
            // the Chebyshev expansion out of the M2L basis adds to the node
            // values P2L wrote and overwrites every other box's
            std::vector<int8_t> add((size_t)nb * nrhs, 0);
            for (int32_t b : items)
                for (int r = 0; r < nrhs; ++r) add[(size_t)b * nrhs + r] = 1;
            P.expand_add = upload(add, s);
        }
        P.p2l_items = upload(items, s);
        P.p2l_roff = upload(roff, s);
        P.p2l_rng = upload(rng, s);
        GemmJob &j = P.p2l_proj;
        std::vector<int32_t> cols = tile_columns(items, nrhs, kGemmCols, j.ntile);
        j.nterm = 1;
        j.cols = upload(cols, s);
        j.src = upload(cols, s);
    }

    wl("P2L lists");
    // L2L, top-down, float64 tiles grouped by octant (one matrix per tile)
    for (int l = 3; l < t.nlev; ++l) {
        std::vector<int32_t> by_oct[8];
        for (int64_t b = t.lvl_off[l]; b < t.lvl_off[l + 1]; ++b) {
            if (ntrg(b) == 0) continue;
            const int32_t *a = &t.h_anchor[3 * b];
            int o = ((a[0] & 1) << 2) | ((a[1] & 1) << 1) | (a[2] & 1);
            by_oct[o].push_back((int32_t)b);
        }
        GemmJob j;
        j.nterm = 1;
        j.use_mat = true;
        std::vector<int32_t> cols, src, mat;
        for (int o = 0; o < 8; ++o) {
            if (by_oct[o].empty()) continue;
            int nt = 0;
            std::vector<int32_t> c = tile_columns(by_oct[o], nrhs, ncol64, nt);
            for (int tl = 0; tl < nt; ++tl) {
                mat.push_back(o);
                for (int k = 0; k < ncol64; ++k) {
                    int32_t v = c[(size_t)tl * ncol64 + k];
                    cols.push_back(v);
                    src.push_back(v < 0 ? -1 : t.h_parent[v / nrhs] * nrhs + v % nrhs);
                }
            }
            j.ntile += nt;
        }
        if (j.ntile == 0) continue;
        j.cols = upload(cols, s);
        j.src = upload(src, s);
        j.mat = upload(mat, s);
        P.l2l_jobs.push_back(std::move(j));
    }

    wl("L2L lists");
    // check-to-equivalent maps and the leaf evaluation lists
    std::vector<int32_t> down_boxes;
    std::vector<uint8_t> up_needed(nb, 0);
    std::vector<int32_t> wleaf, wt0, soff{0}, sbox, poff{0}, prng, pmid;
    std::vector<int8_t> skind;
    // Which point ranges need the r < delta test: tight bounding boxes of the
    // target points of every target leaf and of the source points of every
    // box that supplies points to one; a range is tested when it is the
    // leaf's own box or the two boxes come within sqrt(1.1) delta (the margin
    // covers the float32 rounding of r^2).
    std::vector<int32_t> tb_index(nb, -1), sb_index(nb, -1);
    std::vector<float> tbox, sboxes;
    {
        std::vector<int32_t> tl, sl;
        std::vector<uint8_t> is_src(nb, 0);
        auto mark_src = [&](int32_t a) {
            if (!is_src[a] && nsrc(a) > 0) {
                is_src[a] = 1;
                sb_index[a] = (int32_t)sl.size();
                sl.push_back(a);
            }
        };
        for (int64_t b = 0; b < nb; ++b) {
            if (!leaf(b) || ntrg(b) == 0) continue;
            tb_index[b] = (int32_t)tl.size();
            tl.push_back((int32_t)b);
            for (int32_t k = U.h_off[b]; k < U.h_off[b + 1]; ++k) mark_src(U.h_idx[k]);
            for (int32_t k = W.h_off[b]; k < W.h_off[b + 1]; ++k)
                if (nsrc(W.h_idx[k]) <= ns) mark_src(W.h_idx[k]);
            for (int64_t anc = b; anc >= 0; anc = t.h_parent[anc]) {
                if (ntrg(anc) > ns) continue;
                for (int32_t k = X.h_off[anc]; k < X.h_off[anc + 1]; ++k) mark_src(X.h_idx[k]);
            }
        }
        auto boxes_of = [&](const std::vector<int32_t> &list, const DBuf<int64_t> &beg, const DBuf<int64_t> &end,
                            const DBuf<float> &x, const DBuf<float> &y, const DBuf<float> &z) {
            std::vector<float> h(6 * list.size());
            if (list.empty()) return h;
            DBuf<int32_t> dl = upload(list, s);
            DBuf<float> out(h.size());
            hipLaunchKernelGGL(k_point_boxes, dim3((unsigned)list.size()), dim3(64), 0, s, dl.p, beg.p, end.p, x.p,
                               y.p, z.p, out.p);
            FMM_HIP(hipGetLastError());
            d2h(h.data(), out.p, h.size(), s);
            return h;
        };
        tbox = t.tsm ? boxes_of(tl, t.tbeg, t.tend, t.tx, t.ty, t.tz) : boxes_of(tl, t.sbeg, t.send, t.sx, t.sy, t.sz);
        sboxes = boxes_of(sl, t.sbeg, t.send, t.sx, t.sy, t.sz);
    }
    wl("leaf bounding boxes");
    const double delta2 = std::max((double)P.opt.cutoff * P.opt.cutoff, (double)std::numeric_limits<float>::min());
    auto needs_test = [&](int64_t b, int32_t a) {
        if (a == b) return true;
        const float *tb = &tbox[6 * (size_t)tb_index[b]], *sb = &sboxes[6 * (size_t)sb_index[a]];
        double g2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double gap = std::max(0.0, std::max((double)sb[c] - tb[3 + c], (double)tb[c] - sb[3 + c]));
            g2 += gap * gap;
        }
        return g2 <= 1.1 * delta2;
    };
    // per target leaf, in parallel: its point ranges that need the test and
    // those that do not (each merged), and its W partners evaluated through
    // their upward surfaces; then concatenated in leaf order
    std::vector<int32_t> tleaves;
    for (int64_t b = 0; b < nb; ++b)
        if (leaf(b) && ntrg(b) > 0) tleaves.push_back((int32_t)b);
    struct LeafLists {
        std::vector<int32_t> rt, rf, wsurf;
    };
    std::vector<LeafLists> ll(tleaves.size());
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < (int64_t)tleaves.size(); ++i) {
        const int32_t b = tleaves[i];
        LeafLists &o = ll[i];
        auto add_src = [&](int32_t a) {
            if (nsrc(a) > 0) add_range(needs_test(b, a) ? o.rt : o.rf, t.h_sbeg[a], t.h_send[a]);
        };
        for (int32_t k = U.h_off[b]; k < U.h_off[b + 1]; ++k) add_src(U.h_idx[k]);
        for (int32_t k = W.h_off[b]; k < W.h_off[b + 1]; ++k) {
            const int32_t a = W.h_idx[k];
            if (nsrc(a) == 0) continue;
            if (nsrc(a) <= ns)
                add_src(a);
            else
                o.wsurf.push_back(a);
        }
        for (int64_t anc = b; anc >= 0; anc = t.h_parent[anc]) {
            if (ntrg(anc) > ns) continue;
            for (int32_t k = X.h_off[anc]; k < X.h_off[anc + 1]; ++k) add_src(X.h_idx[k]);
        }
        merge_ranges(o.rt, 0);
        merge_ranges(o.rf, 0);
    }
    int64_t tested_pairs = 0;
    for (size_t i = 0; i < tleaves.size(); ++i) {
        const int32_t b = tleaves[i];
        const LeafLists &o = ll[i];
        if (lvl(b) >= 2) {
            down_boxes.push_back(b);
            if (!P.cheb) {  // the Chebyshev L2P is an interpolation (nodes_to_points), not a kernel sum
                sbox.push_back(b);
                skind.push_back(0);
                P.surf_evals += ntrg(b) * ns;
            }
        }
        for (int32_t a : o.wsurf) {
            sbox.push_back(a);
            skind.push_back(1);
            up_needed[a] = 1;
            P.surf_evals += ntrg(b) * ns;
        }
        prng.insert(prng.end(), o.rt.begin(), o.rt.end());
        pmid.push_back((int32_t)(prng.size() / 2));
        prng.insert(prng.end(), o.rf.begin(), o.rf.end());
        int64_t npts = 0, ntest = 0;
        for (size_t e = 0; e < o.rt.size(); e += 2) ntest += o.rt[e + 1] - o.rt[e];
        npts = ntest;
        for (size_t e = 0; e < o.rf.size(); e += 2) npts += o.rf[e + 1] - o.rf[e];
        P.p2p_pairs += npts * ntrg(b);
        tested_pairs += ntest * ntrg(b);
        soff.push_back((int32_t)sbox.size());
        poff.push_back((int32_t)(prng.size() / 2));
        for (int64_t t0 = 0; t0 < ntrg(b); t0 += 64) {
            wleaf.push_back(b);
            wt0.push_back((int32_t)t0);
        }
    }
    ll.clear();
    wl("evaluation lists");
    // soff/poff are indexed by leaf id: expand to all boxes
    {
        std::vector<int32_t> so(nb + 1, 0), po(nb + 1, 0), pm(nb, 0);
        size_t li = 0;
        int32_t cs = 0, cp = 0;
        for (int64_t b = 0; b < nb; ++b) {
            so[b] = cs;
            po[b] = cp;
            pm[b] = cp;
            if (leaf(b) && ntrg(b) > 0) {
                pm[b] = pmid[li];
                cs = soff[li + 1];
                cp = poff[li + 1];
                ++li;
            }
        }
        so[nb] = cs;
        po[nb] = cp;
        P.soff = upload(so, s);
        P.poff = upload(po, s);
        P.pmid = upload(pm, s);
        P.p2p_tested = tested_pairs;
    }
    wl("evaluation offsets");
    P.nwork = (int)wleaf.size();
    P.wleaf = upload(wleaf, s);
    P.wt0 = upload(wt0, s);
    P.sbox = upload(sbox, s);
    P.skind = upload(skind, s);
    prng.insert(prng.end(), 8, 0);  // the evaluation reads bounds up to 8 entries ahead
    P.prng = upload(prng, s);
    {
        GemmJob &j = P.c2e_down;
        std::vector<int32_t> cols = tile_columns(down_boxes, nrhs, ncol64, j.ntile);
        j.nterm = 1;
        j.cols = upload(cols, s);
        j.src = upload(cols, s);
    }
    {
        std::vector<int32_t> ub;
        for (int64_t b = 0; b < nb; ++b)
            if (up_needed[b]) ub.push_back((int32_t)b);
        GemmJob &j = P.c2e_up;
        std::vector<int32_t> cols = tile_columns(ub, nrhs, ncol64, j.ntile);
        j.nterm = 1;
        j.cols = upload(cols, s);
        j.src = upload(cols, s);
    }
    if (P.cheb) {
        for (int l = t.nlev - 2; l >= 2; --l) {
            std::vector<int32_t> dst, src;
            for (int64_t b = t.lvl_off[l]; b < t.lvl_off[l + 1]; ++b) {
                if (leaf(b) || nsrc(b) == 0) continue;
                dst.push_back((int32_t)b);
                for (int o = 0; o < 8; ++o) {
                    const int32_t ch = t.h_child[8 * (size_t)b + o];
                    src.push_back(ch >= 0 && nsrc(ch) > 0 ? ch : -1);
                }
            }
            if (dst.empty()) continue;
            ChebJob j;
            j.n = (int)dst.size();
            j.dst = upload(dst, s);
            j.src = upload(src, s);
            P.cheb_m2m.push_back(std::move(j));
        }
        for (int l = 3; l < t.nlev; ++l) {
            std::vector<int32_t> dst, src;
            std::vector<int8_t> oct;
            for (int64_t b = t.lvl_off[l]; b < t.lvl_off[l + 1]; ++b) {
                if (ntrg(b) == 0) continue;
                const int32_t *a = &t.h_anchor[3 * b];
                dst.push_back((int32_t)b);
                src.push_back(t.h_parent[b]);
                oct.push_back((int8_t)(((a[0] & 1) << 2) | ((a[1] & 1) << 1) | (a[2] & 1)));
            }
            if (dst.empty()) continue;
            ChebJob j;
            j.n = (int)dst.size();
            j.dst = upload(dst, s);
            j.src = upload(src, s);
            j.oct = upload(oct, s);
            P.cheb_l2l.push_back(std::move(j));
        }
        std::vector<int32_t> with_src, with_trg;
        for (int64_t b = 0; b < nb; ++b) {
            if (lvl(b) < 2) continue;
            if (nsrc(b) > 0) with_src.push_back((int32_t)b);
            if (ntrg(b) > 0) with_trg.push_back((int32_t)b);
        }
        for (auto *jb : {&P.cheb_compress, &P.cheb_expand}) {
            GemmJob &j = *jb;
            std::vector<int32_t> cols = tile_columns(jb == &P.cheb_compress ? with_src : with_trg, nrhs, ncol64, j.ntile);
            j.nterm = 1;
            j.cols = upload(cols, s);
            j.src = upload(cols, s);
        }
    }
    wl("evaluation uploads, expansion and Chebyshev lists");
    phase_end(6);
}

static void run_gemm(GemmJob &j, const double *mats, int m_pad, int k_pad, const float *in, float *out,
                     const double *scale, bool accumulate, hipStream_t s) {
    if (j.ntile == 0) return;
    GemmLaunch a;
    a.m_pad = m_pad;
    a.k_pad = k_pad;
    a.ntile = j.ntile;
    a.nterm = j.nterm;
    a.tile_cols = j.cols.p;
    a.term_src = j.src.p;
    a.term_mat = j.use_mat ? j.mat.p : nullptr;
    a.mats = mats;
    a.mat_elems = (size_t)m_pad * k_pad;
    a.in = in;
    a.out = out;
    a.col_scale = scale;
    a.accumulate = accumulate ? 1 : 0;
    box_gemm_f64(a, s);
}

// adds one timed apply's stage times (its events, once they have completed) to the sums
static void collect_slot(Plan &P, Plan::TimeSlot &ts) {
    FMM_HIP(hipEventSynchronize(ts.ev[ST_COUNT]));
    double ms_k[ST_COUNT];
    for (int k = 0; k < ST_COUNT; ++k) {
        float ms = 0.f;
        FMM_HIP(hipEventElapsedTime(&ms, ts.ev[k], ts.ev[k + 1]));
        ms_k[k] = ms;
    }
    float ms = 0.f;
    if (P.cheb) {
        // L2L ends before the join; P2L and the evaluation ran on the side stream
        FMM_HIP(hipEventElapsedTime(&ms, ts.ev[ST_L2L], ts.l2l_end));
        ms_k[ST_L2L] = ms;
        FMM_HIP(hipEventElapsedTime(&ms, ts.side[0], ts.side[1]));
        ms_k[ST_P2L] = ms;
        FMM_HIP(hipEventElapsedTime(&ms, ts.side[2], ts.side[3]));
        ms_k[ST_EVAL] = ms;
    } else {
        // the near field ran on the side stream; EVAL is it plus the L2P pass
        FMM_HIP(hipEventElapsedTime(&ms, ts.side[2], ts.side[3]));
        ms_k[ST_EVAL] += ms;
    }
    for (int k = 0; k < ST_COUNT; ++k) P.stage_sum[k] += ms_k[k];
    ++P.stage_n;
    ts.pending = false;
}

void plan_apply(Plan &P, const float *q, const float *mu, float *pot, float *field, hipStream_t s, bool capturing) {
    Tree &t = P.t;
    const int nrhs = P.nrhs;
    const Operators &op = *P.ops;
    // a timed apply records its stage events in the next slot (created on
    // first use, from whichever entry point applies)
    Plan::TimeSlot *ts = nullptr;
    if (P.timing && !capturing) {
        ts = &P.tslot[P.tnext];
        if (!ts->ev[0]) {
            for (auto &e : ts->ev) FMM_HIP(hipEventCreate(&e));
            for (auto &e : ts->side) FMM_HIP(hipEventCreate(&e));
            FMM_HIP(hipEventCreate(&ts->l2l_end));
        }
        if (ts->pending) collect_slot(P, *ts);
        P.tnext = (P.tnext + 1) % Plan::kTimeSlots;
    }
    auto mark = [&](int k) {
        if (ts) FMM_HIP(hipEventRecord(ts->ev[k], s));
    };
    const bool sl = q != nullptr, dl = mu != nullptr;
    if (sl && dl && P.qm.n) {
        const int64_t total = (int64_t)nrhs * t.n_src;
        hipLaunchKernelGGL(k_pair_densities, dim3(grid_for(total, kBlock)), dim3(kBlock), 0, s, total, q, mu,
                           (float2 *)P.qm.p);
        hipLaunchKernelGGL(k_sort_density_pairs, dim3(grid_for(t.n_src, kBlock)), dim3(kBlock), 0, s, t.src_perm.p,
                           t.n_src, nrhs, (const float2 *)P.qm.p, t.snx.p, t.sny.p, t.snz.p, P.q_sorted.p, P.mx.p,
                           P.my.p, P.mz.p);
    } else {
        hipLaunchKernelGGL(k_sort_densities, dim3(grid_for(t.n_src, kBlock)), dim3(kBlock), 0, s, t.src_perm.p,
                           t.n_src, nrhs, q, mu, t.snx.p, t.sny.p, t.snz.p, P.q_sorted.p, P.mx.p, P.my.p, P.mz.p);
    }
    FMM_HIP(hipGetLastError());
    // the M2L output accumulates (translation, reduction, gather and, in the
    // surface form, the P2L projection): cleared once per apply, in the
    // Chebyshev form only after the fork, where it waits behind the
    // evaluation's workgroups instead of ahead of P2M
    auto clear_dt = [&]() {
        if (!P.dt.n) return;
        hipLaunchKernelGGL(k_zero, dim3(grid_for((int64_t)P.dt.n, kBlock)), dim3(kBlock), 0, s, P.dt.p, (int64_t)P.dt.n);
        FMM_HIP(hipGetLastError());
    };
    if (!P.cheb) clear_dt();
    const int np = P.n_pad, rp = P.r_pad;

    PointSrc src;
    src.x = t.sx.p;
    src.y = t.sy.p;
    src.z = t.sz.p;
    src.q = P.q_sorted.p;
    src.mx = P.mx.p;
    src.my = P.my.p;
    src.mz = P.mz.p;
    src.n = t.n_src;
    SurfaceGeom g;
    g.Y = op.dY.p;
    g.ns = op.ns;
    g.n_pad = op.n_pad;
    g.centre = t.centre.p;
    g.half = t.half.p;

    auto split_m2l_input = [&] {
        if (P.m2l_form) m2l_split_vecs(P.ut.p, rp, t.nb * nrhs, m2l_form_parts(P.m2l_form), P.ut_bf.p, s);
    };
    auto run_m2l = [&] {
        M2LLaunch m;
        m.r_pad = rp;
        m.ntile = P.m2l_ntile;
        m.ncol = P.m2l_ncol;
        m.tile_term_off = P.m2l_toff.p;
        m.term_dir = P.m2l_dir.p;
        m.term_src = P.m2l_src.p;
        m.tile_cols = P.m2l_cols.p;
        m.mats = op.m2l_f32.p;
        m.in = P.ut.p;
        m.mats_bf = m2l_form_parts(P.m2l_form) == 3 ? op.m2l_bf.p : op.m2l_bf2.p;
        m.in_bf = P.ut_bf.p;
        m.zero = P.m2l_zero.p;
        m.piece_slot = P.m2l_slot.p;
        m.partial = P.m2l_partial.p;
        m.out = P.dt.p;
        m2l_run(P.m2l_form, m, s);
        if (P.m2l_nsplit > 0)
            m2l_reduce(rp, P.m2l_nsplit, P.m2l_ncol, P.m2l_red_cols.p, P.m2l_red_slot0.p, P.m2l_red_k.p, P.m2l_partial.p,
                       P.dt.p, s);
        if (P.m2l_ngather > 0)
            m2l_gather(rp, P.m2l_ngather, P.m2l_gt.p, P.m2l_goff.p, P.m2l_gidx.p, P.m2l_partial.p, P.dt.p, s);
    };

    EvalArgs e;
    e.wleaf = P.wleaf.p;
    e.wt0 = P.wt0.p;
    e.nwork = P.nwork;
    e.soff = P.soff.p;
    e.sbox = P.sbox.p;
    e.skind = P.skind.p;
    e.poff = P.poff.p;
    e.prng = P.prng.p;
    e.pmid = P.pmid.p;
    e.tbeg = t.tbeg.p;
    e.tend = t.tend.p;
    if (t.tsm) {
        e.tx = t.tx.p;
        e.ty = t.ty.p;
        e.tz = t.tz.p;
        e.trg_perm = t.trg_perm.p;
    } else {
        e.tx = t.sx.p;
        e.ty = t.sy.p;
        e.tz = t.sz.p;
        e.trg_perm = t.src_perm.p;
    }
    e.n_trg = t.n_trg;
    e.phi_d = P.phi_d.p;
    e.phi_u = P.phi_u.p;
    e.rad_down = kRadOut;
    e.rad_up = P.cheb ? 1.0 : kRadIn;
    // r < cutoff is excluded; a positive floor also excludes r = 0 when cutoff = 0
    e.delta2 = std::max(P.opt.cutoff * P.opt.cutoff, std::numeric_limits<float>::min());
    e.pot = pot;
    e.field = field;
    if (P.cheb) {
        // Chebyshev form (Sec. III.A.1 Eq. p2m): node weights W (phi_u) up the
        // tree, node values L (phi_d) down; M2L in the shared compressed basis.
        // The leaf evaluation needs W only (M2P), so it runs on the side stream
        // from the end of the upward pass, beside P2L, M2L and L2L, and writes
        // the outputs; L2P adds to them after the join. The node values need
        // no clearing: P2L writes its boxes', the expansion overwrites every
        // other box the downward pass reads (all boxes with targets from
        // level 2) and adds to P2L's, and the rest stay zero from the setup.
        // side stream, first: P2L at the nodes, beside P2M and M2M
        FMM_HIP(hipEventRecord(P.fork0, s));
        FMM_HIP(hipStreamWaitEvent(P.side, P.fork0, 0));
        if (ts) FMM_HIP(hipEventRecord(ts->side[0], P.side));
        points_to_surface(nrhs, sl, dl, P.p2l_items.p, P.n_p2l, P.p2l_roff.p, P.p2l_rng.p, 1.0, g, src, P.phi_d.p,
                          false, P.side);
        if (ts) FMM_HIP(hipEventRecord(ts->side[1], P.side));
        FMM_HIP(hipEventRecord(P.p2l_done, P.side));
        mark(ST_P2M);
        points_to_nodes(nrhs, sl, dl, op.p, op.cheb_coef.p, P.p2m_items.p, P.n_p2m, P.p2m_roff.p, P.p2m_rng.p, g, src,
                        P.phi_u.p, s);
        mark(ST_M2M);
        for (auto &j : P.cheb_m2m)
            cheb_tensor(nrhs, op.p, false, op.cheb_s1.p, j.n, j.dst.p, j.src.p, nullptr, P.phi_u.p, P.phi_u.p, np, s);
        // the upward pass ends with the weights in the M2L basis
        dense_gemm_f32(rp, np, P.cheb_compress.ntile, P.cheb_compress.cols.p, op.pv_f32.p, P.phi_u.p, P.ut.p,
                       nullptr, 0, s);
        // side stream, second: the leaf evaluation, beside M2L and L2L
        FMM_HIP(hipEventRecord(P.fork, s));
        FMM_HIP(hipStreamWaitEvent(P.side, P.fork, 0));
        if (ts) FMM_HIP(hipEventRecord(ts->side[2], P.side));
        eval_leaves(nrhs, sl, dl, e, g, src, P.side);
        if (ts) FMM_HIP(hipEventRecord(ts->side[3], P.side));
        FMM_HIP(hipEventRecord(P.join, P.side));
        mark(ST_P2L);  // (P2L runs on the side stream; timed there)
        // the clearing of the M2L output and the split of its input queue
        // behind the evaluation's workgroups; they stay out of the M2L
        // stage, which times the translation kernel, the reduction and the
        // gather
        clear_dt();
        split_m2l_input();
        mark(ST_M2L);
        run_m2l();
        mark(ST_L2L);
        // the downward pass starts by expanding the M2L result onto the nodes,
        // adding to the P2L values
        FMM_HIP(hipStreamWaitEvent(s, P.p2l_done, 0));
        dense_gemm_f32(np, rp, P.cheb_expand.ntile, P.cheb_expand.cols.p, op.cd_f32.p, P.dt.p, P.phi_d.p,
                       P.col_iscale.p, 0, s, P.expand_add.p);
        for (auto &j : P.cheb_l2l)
            cheb_tensor(nrhs, op.p, true, op.cheb_s1.p, j.n, j.dst.p, j.src.p, j.oct.p, P.phi_d.p, P.phi_d.p, np, s);
        if (ts) FMM_HIP(hipEventRecord(ts->l2l_end, s));
        FMM_HIP(hipStreamWaitEvent(s, P.join, 0));
        mark(ST_C2E);  // the Chebyshev L2P takes the slot of the surface form's check-to-equivalent maps
        EvalArgs el = e;
        el.accumulate = 1;
        nodes_to_points(nrhs, op.p, op.cheb_coef.p, el, g, P.phi_d.p, s);
        mark(ST_EVAL);  // the evaluation itself is timed on the side stream
    } else {
        // Surface form: the near field and M2P (the leaf evaluation without
        // L2P) need only the upward equivalent densities, so after the upward
        // pass they run on the side stream beside P2L, M2L, L2L and the
        // downward expansion; L2P adds to the outputs after the join.
        mark(ST_P2M);
        points_to_surface(nrhs, sl, dl, P.p2m_items.p, P.n_p2m, P.p2m_roff.p, P.p2m_rng.p, kRadOut, g, src, P.chk.p,
                          false, s);
        run_gemm(P.p2m_proj, op.pu_f64.p, rp, np, P.chk.p, P.ut.p, nullptr, false, s);
        mark(ST_M2M);
        for (auto &j : P.m2m_jobs) run_gemm(j, op.m2m_f64.p, rp, rp, P.ut.p, P.ut.p, nullptr, false, s);
        run_gemm(P.c2e_up, op.cu_f64.p, np, rp, P.ut.p, P.phi_u.p, P.col_scale.p, false, s);
        FMM_HIP(hipEventRecord(P.fork, s));
        FMM_HIP(hipStreamWaitEvent(P.side, P.fork, 0));
        if (ts) FMM_HIP(hipEventRecord(ts->side[2], P.side));
        EvalArgs en = e;
        en.surf_mask = 2;  // M2P surfaces and the point ranges
        eval_leaves(nrhs, sl, dl, en, g, src, P.side);
        if (ts) FMM_HIP(hipEventRecord(ts->side[3], P.side));
        FMM_HIP(hipEventRecord(P.join, P.side));
        mark(ST_P2L);
        points_to_surface(nrhs, sl, dl, P.p2l_items.p, P.n_p2l, P.p2l_roff.p, P.p2l_rng.p, kRadIn, g, src, P.chk.p,
                          false, s);
        run_gemm(P.p2l_proj, op.pv_f64.p, rp, np, P.chk.p, P.dt.p, nullptr, true, s);
        mark(ST_M2L);
        split_m2l_input();
        run_m2l();
        mark(ST_L2L);
        for (auto &j : P.l2l_jobs) run_gemm(j, op.l2l_f64.p, rp, rp, P.dt.p, P.dt.p, nullptr, true, s);
        mark(ST_C2E);
        run_gemm(P.c2e_down, op.cd_f64.p, np, rp, P.dt.p, P.phi_d.p, P.col_scale.p, false, s);
        FMM_HIP(hipStreamWaitEvent(s, P.join, 0));
        mark(ST_EVAL);
        EvalArgs ef = e;
        ef.surf_mask = 1;  // L2P: the leaf's own downward surface, added to the near field
        ef.points = 0;
        ef.accumulate = 1;
        eval_leaves(nrhs, sl, dl, ef, g, src, s);
    }
    mark(ST_COUNT);
    if (ts) ts->pending = true;
}

void plan_report_times(Plan &P) {
    for (int i = 0; i < Plan::kTimeSlots; ++i) {
        Plan::TimeSlot &ts = P.tslot[(P.tnext + i) % Plan::kTimeSlots];  // oldest first
        if (ts.pending) collect_slot(P, ts);
    }
    if (P.stage_n == 0) return;
    for (int k = 0; k < ST_COUNT; ++k) {
        P.stage_ms[k] = P.stage_sum[k] / P.stage_n;
        P.stage_sum[k] = 0.0;
    }
    P.stage_n = 0;
    P.have_times = true;
}

void plan_create_side(Plan &P) {
    if (P.side) return;
    FMM_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));  // default priority
    for (hipEvent_t *e : {&P.fork0, &P.p2l_done, &P.fork, &P.join})
        FMM_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
}

void plan_release_events(Plan &P) {
    if (P.side) {
        (void)hipStreamSynchronize(P.side);
        (void)hipStreamDestroy(P.side);
        P.side = nullptr;
    }
    for (hipEvent_t *e : {&P.fork0, &P.p2l_done, &P.fork, &P.join})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    for (auto &ts : P.tslot) {
        for (auto &e : ts.ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : ts.side)
            if (e) (void)hipEventDestroy(e);
        if (ts.l2l_end) (void)hipEventDestroy(ts.l2l_end);
        ts = Plan::TimeSlot{};
    }
}

void plan_apply_graph(Plan &P, const float *q, const float *mu, float *pot, float *field, hipStream_t s) {
    auto &G = P.graph;
    const std::array<const void *, 4> key = {q, mu, pot, field};
    if (!G.stream) {
        FMM_HIP(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
        FMM_HIP(hipEventCreateWithFlags(&G.in, hipEventDisableTiming));
        FMM_HIP(hipEventCreateWithFlags(&G.out, hipEventDisableTiming));
    }
    if (!G.exec || G.key != key) {
        if (G.exec) {
            FMM_HIP(hipGraphExecDestroy(G.exec));
            G.exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        FMM_HIP(hipStreamBeginCapture(G.stream, hipStreamCaptureModeThreadLocal));
        try {
            plan_apply(P, q, mu, pot, field, G.stream, true);
        } catch (...) {
            (void)hipStreamEndCapture(G.stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        FMM_HIP(hipStreamEndCapture(G.stream, &graph));
        const hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        FMM_HIP(e);
        G.key = key;
    }
    // the graph runs on the plan's stream, ordered after the caller's work
    // and before whatever the caller queues next
    FMM_HIP(hipEventRecord(G.in, s));
    FMM_HIP(hipStreamWaitEvent(G.stream, G.in, 0));
    FMM_HIP(hipGraphLaunch(G.exec, G.stream));
    FMM_HIP(hipEventRecord(G.out, G.stream));
    FMM_HIP(hipStreamWaitEvent(s, G.out, 0));
}

void plan_release_graph(Plan &P) {
    auto &G = P.graph;
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.stream) {
        (void)hipStreamSynchronize(G.stream);
        (void)hipStreamDestroy(G.stream);
    }
    if (G.in) (void)hipEventDestroy(G.in);
    if (G.out) (void)hipEventDestroy(G.out);
    G = Plan::Graph{};
}

}  // namespace fmm
