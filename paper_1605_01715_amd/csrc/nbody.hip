// n-body shaped kernels of the FMM: P2M, P2L, L2P, M2P, P2P and the
// all-pairs direct sum.
//
// The kernels are the Laplace single layer q / (4 pi r), the double layer
// m . (x - y) / (4 pi r^3) with m = mu n_y (the normal derivative applied at
// the source side, Sec. III.A.1 Eq. p2m), and the field q (x - y) / (4 pi r^3)
// (Sec. III.A.2 Eq. kernel_pol). Pairs closer than the tolerance radius are
// excluded in the near field (Sec. III.A.1).
//
// One wave (64 lanes) handles one box. Sources are staged in LDS, 64 at a
// time, and every lane reads them by broadcast. Surface points and the
// sources seen from a box surface are expressed relative to the box centre in
// float64 before rounding to float32, so the rounding error of a coordinate
// is relative to the box size, not to the distance from the origin. The
// near field uses the float32 input coordinates directly (x - y of two close
// float32 values is exact). Per-target sums are accumulated per LDS tile in
// float32 and folded into a (hi, lo) pair with Knuth's TwoSum.
#include <type_traits>

#include "nbody.hpp"

namespace fmm {

namespace {

constexpr float kInv4Pi = 0.079577471545947667884f;

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ inline void two_sum_into(float &hi, float &lo, float p) {
    float s = hi + p;
    float bb = s - hi;
    float err = (hi - (s - bb)) + (p - bb);
    hi = s;
    lo += err;
}

// ------------------------------------------------------------ P2M / P2L

// q / r + (m . d) / r^3 = (q + (m . d) / r^2) / r for one (surface point,
// source) pair; v holds the source's offset from the box centre, then its
// strengths. Check points lie outside every box that feeds them (P2M: radius
// 2.95 around the sources' own box; P2L: X-list boxes are a box width away),
// so r > 0; the floor only keeps a degenerate input finite.
template <int NRHS, bool SL, bool DL>
__device__ inline void pair_terms(float x, float y, float z, const float *v, float *t) {
    const float dx = x - v[0], dy = y - v[1], dz = z - v[2];
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float inv = rsq(fmaxf(r2, 1e-30f));
    const float inv2 = inv * inv;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) {
        float u = SL ? v[3 + r] : 0.f;
        if (DL) {
            const int o = 3 + (SL ? NRHS : 0) + 3 * r;
            u += (v[o] * dx + v[o + 1] * dy + v[o + 2] * dz) * inv2;
        }
        t[r] = u * inv;
    }
}

template <int NRHS, bool SL, bool DL>
__global__ __launch_bounds__(64) void k_points_to_surface(const int32_t *items, const int32_t *roff,
                                                         const int32_t *rng, double rfac, SurfaceGeom g,
                                                         PointSrc src, float *out, int accumulate) {
    constexpr int TPL = 8;        // surface points per lane (n_s <= 512)
    constexpr int W = 3 + (SL ? NRHS : 0) + (DL ? 3 * NRHS : 0);
    __shared__ float sh[64 * W];
    const int lane = threadIdx.x;
    const int b = items[blockIdx.x];
    const double cx = g.centre[3 * b], cy = g.centre[3 * b + 1], cz = g.centre[3 * b + 2];
    const double rr = rfac * g.half[b];
    float xm[TPL], ym[TPL], zm[TPL];
    // float64 sums (of float32 sums of two pairs): check potentials feed every translation
    double acc[TPL][NRHS];
    for (int i = 0; i < TPL; ++i) {
        int m = lane + 64 * i;
        bool ok = m < g.ns;
        xm[i] = ok ? (float)(rr * g.Y[3 * m]) : 0.f;
        ym[i] = ok ? (float)(rr * g.Y[3 * m + 1]) : 0.f;
        zm[i] = ok ? (float)(rr * g.Y[3 * m + 2]) : 0.f;
        for (int r = 0; r < NRHS; ++r) acc[i][r] = 0.0;
    }
    const int ntpl = (g.ns + 63) / 64;
    for (int e = roff[blockIdx.x]; e < roff[blockIdx.x + 1]; ++e) {
        const int s0 = rng[2 * e], s1 = rng[2 * e + 1];
        for (int j0 = s0; j0 < s1; j0 += 64) {
            const int j = j0 + lane;
            const int cnt = min(64, s1 - j0);
            {
                // lanes past the range stage a zero-strength source at the box centre (r > 0 from
                // every check point), so the pair loop below can run over an even count
                float *p = sh + lane * W;
#pragma unroll
                for (int k = 0; k < W; ++k) p[k] = 0.f;
                if (j < s1) {
                    p[0] = (float)((double)src.x[j] - cx);
                    p[1] = (float)((double)src.y[j] - cy);
                    p[2] = (float)((double)src.z[j] - cz);
                    int o = 3;
                    if (SL)
                        for (int r = 0; r < NRHS; ++r) p[o++] = src.q[r * src.n + j];
                    if (DL)
                        for (int r = 0; r < NRHS; ++r) {
                            p[o++] = src.mx[r * src.n + j];
                            p[o++] = src.my[r * src.n + j];
                            p[o++] = src.mz[r * src.n + j];
                        }
                }
            }
            __syncthreads();
            for (int jj = 0; jj < cnt; jj += 2) {
                // two sources per step, read into registers once for all surface points
                float v0[W], v1[W];
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    v0[k] = sh[jj * W + k];
                    v1[k] = sh[(jj + 1) * W + k];
                }
#pragma unroll
                for (int i = 0; i < TPL; ++i) {
                    if (i >= ntpl) continue;  // static index keeps acc in registers
                    float t0[NRHS], t1[NRHS];
                    pair_terms<NRHS, SL, DL>(xm[i], ym[i], zm[i], v0, t0);
                    pair_terms<NRHS, SL, DL>(xm[i], ym[i], zm[i], v1, t1);
#pragma unroll
                    for (int r = 0; r < NRHS; ++r) acc[i][r] += (double)(t0[r] + t1[r]);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < TPL; ++i) {
        int m = lane + 64 * i;
        if (m >= g.ns) continue;
        for (int r = 0; r < NRHS; ++r) {
            float *op = out + ((int64_t)b * NRHS + r) * g.n_pad + m;
            double v = acc[i][r] * (1.0 / kFourPi);
            *op = accumulate ? (float)((double)*op + v) : (float)v;
        }
    }
}

// ------------------------------------------------------------ leaf evaluation
//
// One wave per work item (up to 64 targets of a leaf). Lanes are laid out as
// S source slices x L lane-targets, each lane holding TPL targets (1 to 4
// with one output and one right-hand side, else 1 or 2), chosen per item to
// keep most lane-slots busy: a 45-target item runs as 15 lanes x 3 targets x
// 4 slices (94% of the slots) instead of 45 of 64 lanes, or 23 x 2 x 2 (70%).
// More targets per lane also read each staged source once for more pairs.
// Sources are staged in
// LDS 64 at a time (records padded to 16 bytes, the tail of a tile filled
// with zero-density sources far away), so the loop over a tile has the same
// trip count in every lane and no per-pair validity test. Slices are summed
// through LDS at the end.
constexpr int kFar = 1000000000;  // far-away coordinate of padding records (1e9)

template <int NRHS, bool SL, bool DL, bool FIELD>
struct EvalShape {
    static constexpr int NOUT = FIELD ? 4 : 1;
    static constexpr int WP = 3 + (SL ? NRHS : 0) + (DL ? 3 * NRHS : 0);  // point source record
    static constexpr int WS = 3 + NRHS;                                   // surface source record
    static constexpr int W = ((WP > WS ? WP : WS) + 3) / 4 * 4;           // floats, 16-byte aligned
    static constexpr int NREC = 128;                                      // 64 + room for slice overrun
};

template <int TPL, int NRHS, bool SL, bool DL, bool FIELD>
__device__ void eval_item(const EvalArgs &a, const SurfaceGeom &g, const PointSrc &src, int leaf, int64_t t_first,
                          int nt, float *sh, float *red) {
    using E = EvalShape<NRHS, SL, DL, FIELD>;
    constexpr int NOUT = E::NOUT, W = E::W, NREC = E::NREC;
    const int lane = threadIdx.x;
    const int L = (nt + TPL - 1) / TPL;      // lanes per slice
    const int S = 64 / L;                    // slices
    const int slice = lane / L, tl = lane % L;
    const int niter = (64 + S - 1) / S;      // uniform trip count over a tile
    const bool active = slice < S;

    float xg[TPL], yg[TPL], zg[TPL], xl[TPL], yl[TPL], zl[TPL];
    const double cx = g.centre[3 * leaf], cy = g.centre[3 * leaf + 1], cz = g.centre[3 * leaf + 2];
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const int t = tl + u * L;
        const int64_t k = t_first + (t < nt ? t : 0);
        xg[u] = a.tx[k];
        yg[u] = a.ty[k];
        zg[u] = a.tz[k];
        xl[u] = (float)((double)xg[u] - cx);
        yl[u] = (float)((double)yg[u] - cy);
        zl[u] = (float)((double)zg[u] - cz);
    }
    float hi[TPL][NRHS][NOUT], lo[TPL][NRHS][NOUT];
#pragma unroll
    for (int u = 0; u < TPL; ++u)
        for (int r = 0; r < NRHS; ++r)
            for (int o = 0; o < NOUT; ++o) hi[u][r][o] = lo[u][r][o] = 0.f;

    // padding records: slots 64..127 once (every tile's overrun), slots
    // [cnt, 64) per tile
    auto pad = [&](int slot) {
        float *p = sh + slot * W;
        p[0] = p[1] = p[2] = (float)kFar;
        for (int c = 3; c < W; ++c) p[c] = 0.f;
    };
    pad(64 + lane);

    // surfaces: L2P (own downward equivalent density) and M2P (W-list boxes);
    // surface points never coincide with targets (they lie outside the box)
    for (int e = a.soff[leaf]; e < a.soff[leaf + 1]; ++e) {
        if (!(a.surf_mask & (1 << a.skind[e]))) continue;  // the same for every lane
        const int box = a.sbox[e];
        const bool down = a.skind[e] == 0;
        const double rr = (down ? a.rad_down : a.rad_up) * g.half[box];
        const double ox = g.centre[3 * box] - cx, oy = g.centre[3 * box + 1] - cy, oz = g.centre[3 * box + 2] - cz;
        const float *phi = (down ? a.phi_d : a.phi_u) + (int64_t)box * NRHS * g.n_pad;
        for (int m0 = 0; m0 < g.ns; m0 += 64) {
            const int m = m0 + lane;
            if (m < g.ns) {
                float *p = sh + lane * W;
                p[0] = (float)(ox + rr * g.Y[3 * m]);
                p[1] = (float)(oy + rr * g.Y[3 * m + 1]);
                p[2] = (float)(oz + rr * g.Y[3 * m + 2]);
                for (int r = 0; r < NRHS; ++r) p[3 + r] = phi[r * g.n_pad + m];
            } else {
                pad(lane);
            }
            __syncthreads();
            float part[TPL][NRHS][NOUT];
#pragma unroll
            for (int u = 0; u < TPL; ++u)
                for (int r = 0; r < NRHS; ++r)
                    for (int o = 0; o < NOUT; ++o) part[u][r][o] = 0.f;
            for (int i = 0; i < niter; ++i) {
                const float4 *p4 = (const float4 *)(sh + (slice + i * S) * W);
                const float4 r0 = p4[0];
                float ph[NRHS];
                ph[0] = r0.w;
                if (NRHS > 1) {
                    const float4 r1 = p4[1];
                    const float rest[3] = {r1.x, r1.y, r1.z};
                    for (int r = 1; r < NRHS; ++r) ph[r] = rest[r - 1];
                }
#pragma unroll
                for (int u = 0; u < TPL; ++u) {
                    const float dx = xl[u] - r0.x, dy = yl[u] - r0.y, dz = zl[u] - r0.z;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float inv = rsq(r2);
                    if constexpr (FIELD) {
                        const float inv3 = inv * inv * inv;
                        for (int r = 0; r < NRHS; ++r) {
                            part[u][r][0] += ph[r] * inv;
                            const float di3 = ph[r] * inv3;
                            part[u][r][1] += di3 * dx;
                            part[u][r][2] += di3 * dy;
                            part[u][r][3] += di3 * dz;
                        }
                    } else {
                        for (int r = 0; r < NRHS; ++r) part[u][r][0] += ph[r] * inv;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < TPL; ++u)
                for (int r = 0; r < NRHS; ++r)
                    for (int o = 0; o < NOUT; ++o) two_sum_into(hi[u][r][o], lo[u][r][o], part[u][r][o]);
            __syncthreads();
        }
    }

    // points: P2P (U list) and the direct W / X pairs; r < delta excluded
    // (delta2 > 0 also excludes r = 0). Ranges [poff, pmid) may hold a pair
    // closer than delta and are tested pair by pair; for ranges [pmid,
    // poff + 1) the setup has shown that the points' bounding boxes are
    // farther apart than delta, and the test is skipped.
    const float delta2 = a.delta2;
    // The ranges e0 .. e1 - 1 as one sequence of sources, staged 64 at a
    // time: a tile runs across range boundaries, so only the sequence's last
    // tile is padded (per-range tiles left a quarter of the slots padding on
    // the clustered cloud, whose leaves have about ten merged ranges each).
    // (e, off) is the wave-uniform position of the tile's first source.
    // Range bounds are wave-uniform: read through the constant address space
    // they become scalar loads, and the four bounds pairs a tile looks at
    // first are read together (the array is padded by 8 entries, so reads
    // past the last range stay inside it).
    const int32_t __attribute__((address_space(4))) *rng =
        (const int32_t __attribute__((address_space(4))) *)a.prng;
    auto stream = [&](auto test_tag, int e0, int e1) {
        constexpr bool TEST = decltype(test_tag)::value;
        int e = e0, off = 0;
        while (e < e1) {
            // this lane's source: the tile covers the rest of range e and,
            // past its end, the next ranges (a tile rarely spans more than four)
            int j = -1;
            {
                int bnd[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) bnd[u] = rng[2 * e + u];
                int base = 0, k = e;  // base: tile position where range k starts
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r0 = bnd[2 * u] + (u == 0 ? off : 0);
                    const int len = (k < e1) ? bnd[2 * u + 1] - r0 : 0;
                    if (lane >= base && lane < base + len) j = r0 + (lane - base);
                    base += len;
                    k += k < e1 ? 1 : 0;
                }
                while (k < e1 && base < 64) {
                    const int r0 = rng[2 * k], len = rng[2 * k + 1] - r0;
                    if (lane >= base && lane < base + len) j = r0 + (lane - base);
                    base += len;
                    ++k;
                }
            }
            if (j >= 0) {
                float *p = sh + lane * W;
                p[0] = src.x[j];
                p[1] = src.y[j];
                p[2] = src.z[j];
                int o = 3;
                if (SL)
                    for (int r = 0; r < NRHS; ++r) p[o++] = src.q[r * src.n + j];
                if (DL)
                    for (int r = 0; r < NRHS; ++r) {
                        p[o++] = src.mx[r * src.n + j];
                        p[o++] = src.my[r * src.n + j];
                        p[o++] = src.mz[r * src.n + j];
                    }
            } else {
                pad(lane);
            }
            __syncthreads();
            float part[TPL][NRHS][NOUT];
#pragma unroll
            for (int u = 0; u < TPL; ++u)
                for (int r = 0; r < NRHS; ++r)
                    for (int o = 0; o < NOUT; ++o) part[u][r][o] = 0.f;
            for (int i = 0; i < niter; ++i) {
                const float *p = sh + (slice + i * S) * W;
                float rec[W];
#pragma unroll
                for (int c = 0; c < W; c += 4) {
                    const float4 v = *(const float4 *)(p + c);
                    rec[c] = v.x;
                    rec[c + 1] = v.y;
                    rec[c + 2] = v.z;
                    rec[c + 3] = v.w;
                }
#pragma unroll
                for (int u = 0; u < TPL; ++u) {
                    const float dx = xg[u] - rec[0], dy = yg[u] - rec[1], dz = zg[u] - rec[2];
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float inv = TEST ? (r2 >= delta2 ? rsq(r2) : 0.f) : rsq(r2);
                    const float inv2 = inv * inv;
                    int o = 3;
                    float sl[NRHS];
                    for (int r = 0; r < NRHS; ++r) sl[r] = SL ? rec[o + r] : 0.f;
                    if (SL) o += NRHS;
                    if constexpr (FIELD) {
                        const float inv3 = inv2 * inv;
                        for (int r = 0; r < NRHS; ++r) {
                            part[u][r][0] += sl[r] * inv;
                            const float di3 = sl[r] * inv3;
                            part[u][r][1] += di3 * dx;
                            part[u][r][2] += di3 * dy;
                            part[u][r][3] += di3 * dz;
                        }
                    } else {
                        for (int r = 0; r < NRHS; ++r) {
                            // q / r + (m . d) / r^3 = (q + (m . d) / r^2) / r
                            float t = sl[r];
                            if (DL) {
                                const float md = rec[o + 3 * r] * dx + rec[o + 3 * r + 1] * dy + rec[o + 3 * r + 2] * dz;
                                t += md * inv2;
                            }
                            part[u][r][0] += t * inv;
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < TPL; ++u)
                for (int r = 0; r < NRHS; ++r)
                    for (int o = 0; o < NOUT; ++o) two_sum_into(hi[u][r][o], lo[u][r][o], part[u][r][o]);
            __syncthreads();
            // advance the position by 64 sources
            int adv = 64;
            while (e < e1) {
                const int rest = rng[2 * e + 1] - rng[2 * e] - off;
                if (adv < rest) {
                    off += adv;
                    break;
                }
                adv -= rest;
                ++e;
                off = 0;
            }
        }
    };
    if (a.points) {
        const int pmid = a.pmid ? a.pmid[leaf] : a.poff[leaf + 1];
        stream(std::true_type{}, a.poff[leaf], pmid);
        stream(std::false_type{}, pmid, a.poff[leaf + 1]);
    }

    // sum the slices of each target through LDS, then slice 0 writes
    constexpr int NV = TPL * NRHS * NOUT;
    if (active && slice > 0) {
        float *q = red + (size_t)lane * NV * 2;
        int v = 0;
#pragma unroll
        for (int u = 0; u < TPL; ++u)
            for (int r = 0; r < NRHS; ++r)
                for (int o = 0; o < NOUT; ++o, ++v) {
                    q[2 * v] = hi[u][r][o];
                    q[2 * v + 1] = lo[u][r][o];
                }
    }
    __syncthreads();
    if (active && slice == 0) {
        for (int sl2 = 1; sl2 < S; ++sl2) {
            const float *q = red + (size_t)(sl2 * L + tl) * NV * 2;
            int v = 0;
#pragma unroll
            for (int u = 0; u < TPL; ++u)
                for (int r = 0; r < NRHS; ++r)
                    for (int o = 0; o < NOUT; ++o, ++v) {
                        two_sum_into(hi[u][r][o], lo[u][r][o], q[2 * v]);
                        lo[u][r][o] += q[2 * v + 1];
                    }
        }
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
            const int t = tl + u * L;
            if (t >= nt) continue;
            const int64_t k = t_first + t;
            const int64_t dst = a.trg_perm ? a.trg_perm[k] : k;
            for (int r = 0; r < NRHS; ++r) {
                if (a.pot) {
                    float *pp = a.pot + r * a.n_trg + dst;
                    const float v = (hi[u][r][0] + lo[u][r][0]) * kInv4Pi;
                    *pp = a.accumulate ? *pp + v : v;
                }
                if (FIELD && a.field) {
                    float *f = a.field + ((int64_t)r * a.n_trg + dst) * 3;
                    for (int c = 0; c < 3; ++c) {
                        const float v = (hi[u][r][1 + c] + lo[u][r][1 + c]) * kInv4Pi;
                        f[c] = a.accumulate ? f[c] + v : v;
                    }
                }
            }
        }
    }
}

template <int NRHS, bool SL, bool DL, bool FIELD>
__global__ __launch_bounds__(64) void k_eval(EvalArgs a, SurfaceGeom g, PointSrc src) {
    using E = EvalShape<NRHS, SL, DL, FIELD>;
    // up to 4 targets per lane where one output and one right-hand side
    // keep the accumulators few; 2 otherwise
    constexpr int MAXTPL = (E::NOUT == 1 && NRHS == 1) ? 4 : 2;
    constexpr int NSH = E::NREC * E::W, NRED = 64 * MAXTPL * NRHS * E::NOUT * 2;
    // the slice sums of the end reuse the source records' LDS
    __shared__ __align__(16) float sh[NSH > NRED ? NSH : NRED];
    const int leaf = a.wleaf[blockIdx.x];
    const int64_t t_first = a.tbeg[leaf] + a.wt0[blockIdx.x];
    const int nt = (int)min((int64_t)64, a.tend[leaf] - t_first);
    // targets per lane (TPL): the count that keeps the most lane-slots busy,
    // nt * S / (64 TPL) with S = 64 / ceil(nt / TPL) slices; ties to the larger
    // (fewer LDS reads per pair)
    int best = 1, bnum = nt * (64 / nt), bden = 64;
#pragma unroll
    for (int tpl = 2; tpl <= MAXTPL; ++tpl) {
        const int num = nt * (64 / ((nt + tpl - 1) / tpl)), den = 64 * tpl;
        if (num * bden >= bnum * den) {
            best = tpl;
            bnum = num;
            bden = den;
        }
    }
    if constexpr (MAXTPL == 4) {
        if (best == 4) return eval_item<4, NRHS, SL, DL, FIELD>(a, g, src, leaf, t_first, nt, sh, sh);
        if (best == 3) return eval_item<3, NRHS, SL, DL, FIELD>(a, g, src, leaf, t_first, nt, sh, sh);
    }
    if (best >= 2)
        eval_item<2, NRHS, SL, DL, FIELD>(a, g, src, leaf, t_first, nt, sh, sh);
    else
        eval_item<1, NRHS, SL, DL, FIELD>(a, g, src, leaf, t_first, nt, sh, sh);
}

// ------------------------------------------------------------ all pairs
__global__ __launch_bounds__(256) void k_direct(const float *trg, int64_t n_trg, const float *src, const float *nrm,
                                               int64_t n_src, const float *q, const float *mu, float delta2,
                                               float *pot, float *field) {
    __shared__ float sh[256][8];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < n_trg;
    const float x = valid ? trg[3 * i] : 0.f, y = valid ? trg[3 * i + 1] : 0.f, z = valid ? trg[3 * i + 2] : 0.f;
    float hp = 0.f, lp = 0.f, hf[3] = {0.f, 0.f, 0.f}, lf[3] = {0.f, 0.f, 0.f};
    for (int64_t j0 = 0; j0 < n_src; j0 += 256) {
        const int64_t j = j0 + threadIdx.x;
        if (j < n_src) {
            sh[threadIdx.x][0] = src[3 * j];
            sh[threadIdx.x][1] = src[3 * j + 1];
            sh[threadIdx.x][2] = src[3 * j + 2];
            sh[threadIdx.x][3] = q ? q[j] : 0.f;
            float m = mu ? mu[j] : 0.f;
            sh[threadIdx.x][4] = mu ? m * nrm[3 * j] : 0.f;
            sh[threadIdx.x][5] = mu ? m * nrm[3 * j + 1] : 0.f;
            sh[threadIdx.x][6] = mu ? m * nrm[3 * j + 2] : 0.f;
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)256, n_src - j0);
        float pp = 0.f, pf[3] = {0.f, 0.f, 0.f};
        for (int jj = 0; jj < cnt; ++jj) {
            float dx = x - sh[jj][0], dy = y - sh[jj][1], dz = z - sh[jj][2];
            float r2 = dx * dx + dy * dy + dz * dz;
            float inv = (r2 >= delta2 && r2 > 0.f) ? rsq(r2) : 0.f;
            float inv3 = inv * inv * inv;
            float qq = sh[jj][3];
            pp += qq * inv + (sh[jj][4] * dx + sh[jj][5] * dy + sh[jj][6] * dz) * inv3;
            pf[0] += qq * inv3 * dx;
            pf[1] += qq * inv3 * dy;
            pf[2] += qq * inv3 * dz;
        }
        two_sum_into(hp, lp, pp);
        for (int c = 0; c < 3; ++c) two_sum_into(hf[c], lf[c], pf[c]);
        __syncthreads();
    }
    if (!valid) return;
    if (pot) pot[i] = (hp + lp) * kInv4Pi;
    if (field)
        for (int c = 0; c < 3; ++c) field[3 * i + c] = (hf[c] + lf[c]) * kInv4Pi;
}

}  // namespace

#define FMM_NRHS_SWITCH(NRHS_VAR, CALL)                                                        \
    switch (NRHS_VAR) {                                                                        \
    case 1: { constexpr int R = 1; CALL; } break;                                              \
    case 2: { constexpr int R = 2; CALL; } break;                                              \
    case 3: { constexpr int R = 3; CALL; } break;                                              \
    case 4: { constexpr int R = 4; CALL; } break;                                              \
    default: throw Error(FMM_ERR_ARG, "nrhs must be 1..4");                                    \
    }

void points_to_surface(int nrhs, bool sl, bool dl, const int32_t *items, int nitems, const int32_t *roff,
                       const int32_t *rng, double rfac, const SurfaceGeom &g, const PointSrc &src, float *out,
                       bool accumulate, hipStream_t s) {
    if (nitems <= 0) return;
    FMM_REQUIRE(g.ns <= 512, "points_to_surface: surface too large");
    dim3 gr(nitems), bl(64);
    int acc = accumulate ? 1 : 0;
    if (sl && dl) {
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_points_to_surface<R, true, true>), gr, bl, 0, s, items, roff, rng,
                                                 rfac, g, src, out, acc));
    } else if (dl) {
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_points_to_surface<R, false, true>), gr, bl, 0, s, items, roff,
                                                 rng, rfac, g, src, out, acc));
    } else {
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_points_to_surface<R, true, false>), gr, bl, 0, s, items, roff,
                                                 rng, rfac, g, src, out, acc));
    }
    FMM_HIP(hipGetLastError());
}

void eval_leaves(int nrhs, bool sl, bool dl, const EvalArgs &a, const SurfaceGeom &g, const PointSrc &src,
                 hipStream_t s) {
    if (a.nwork <= 0) return;
    dim3 gr(a.nwork), bl(64);
    const bool field = a.field != nullptr;
    if (field) {
        FMM_REQUIRE(sl && !dl, "field output is defined for the single layer only");
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_eval<R, true, false, true>), gr, bl, 0, s, a, g, src));
    } else if (sl && dl) {
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_eval<R, true, true, false>), gr, bl, 0, s, a, g, src));
    } else if (dl) {
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_eval<R, false, true, false>), gr, bl, 0, s, a, g, src));
    } else {
        FMM_NRHS_SWITCH(nrhs, hipLaunchKernelGGL((k_eval<R, true, false, false>), gr, bl, 0, s, a, g, src));
    }
    FMM_HIP(hipGetLastError());
}

void direct_all_pairs(const float *trg, int64_t n_trg, const float *src, const float *nrm, int64_t n_src,
                      const float *q, const float *mu, float delta, float *pot, float *field, hipStream_t s) {
    if (n_trg <= 0) return;
    hipLaunchKernelGGL(k_direct, dim3(grid_for(n_trg, 256)), dim3(256), 0, s, trg, n_trg, src, nrm, n_src, q, mu,
                       delta * delta, pot, field);
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
