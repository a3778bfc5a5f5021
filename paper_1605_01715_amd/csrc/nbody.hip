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
    double acc[TPL][NRHS];  // float64 sums: check potentials feed every translation
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
            if (j < s1) {
                float *p = sh + lane * W;
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
            __syncthreads();
            for (int jj = 0; jj < cnt; ++jj) {
                const float *p = sh + jj * W;
                const float sx = p[0], sy = p[1], sz = p[2];
#pragma unroll
                for (int i = 0; i < TPL; ++i) {
                    if (i >= ntpl) continue;  // static index keeps acc in registers
                    float dx = xm[i] - sx, dy = ym[i] - sy, dz = zm[i] - sz;
                    float r2 = dx * dx + dy * dy + dz * dz;
                    float inv = r2 > 0.f ? rsq(r2) : 0.f;
                    int o = 3;
                    if (SL)
                        for (int r = 0; r < NRHS; ++r) acc[i][r] += (double)(p[o++] * inv);
                    if (DL) {
                        float inv3 = inv * inv * inv;
                        for (int r = 0; r < NRHS; ++r) {
                            float md = p[o] * dx + p[o + 1] * dy + p[o + 2] * dz;
                            o += 3;
                            acc[i][r] += (double)(md * inv3);
                        }
                    }
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
template <int NRHS, bool SL, bool DL, bool FIELD>
__global__ __launch_bounds__(64) void k_eval(EvalArgs a, SurfaceGeom g, PointSrc src) {
    constexpr int NOUT = FIELD ? 4 : 1;
    constexpr int WS = 3 + NRHS;  // surface source record
    constexpr int WP = 3 + (SL ? NRHS : 0) + (DL ? 3 * NRHS : 0);
    constexpr int W = WP > WS ? WP : WS;
    __shared__ float sh[64 * W];
    const int lane = threadIdx.x;
    const int leaf = a.wleaf[blockIdx.x];
    const int64_t t_first = a.tbeg[leaf] + a.wt0[blockIdx.x];
    const int nt = (int)min((int64_t)64, a.tend[leaf] - t_first);
    int tp = 1;
    while (tp < nt) tp <<= 1;
    const int grp = lane / tp, ngrp = 64 / tp;
    const int tl = lane % tp;
    const bool tvalid = tl < nt;
    const int64_t k = t_first + (tvalid ? tl : 0);
    const float xg = a.tx[k], yg = a.ty[k], zg = a.tz[k];
    const double cx = g.centre[3 * leaf], cy = g.centre[3 * leaf + 1], cz = g.centre[3 * leaf + 2];
    const float xl = (float)((double)xg - cx), yl = (float)((double)yg - cy), zl = (float)((double)zg - cz);
    float hi[NRHS][NOUT], lo[NRHS][NOUT];
    for (int r = 0; r < NRHS; ++r)
        for (int o = 0; o < NOUT; ++o) hi[r][o] = lo[r][o] = 0.f;

    // surfaces: L2P (own downward equivalent density) and M2P (W-list boxes)
    for (int e = a.soff[leaf]; e < a.soff[leaf + 1]; ++e) {
        const int box = a.sbox[e];
        const bool down = a.skind[e] == 0;
        const double rr = (down ? kRadOut : kRadIn) * g.half[box];
        const double ox = g.centre[3 * box] - cx, oy = g.centre[3 * box + 1] - cy, oz = g.centre[3 * box + 2] - cz;
        const float *phi = (down ? a.phi_d : a.phi_u) + (int64_t)box * NRHS * g.n_pad;
        for (int m0 = 0; m0 < g.ns; m0 += 64) {
            const int m = m0 + lane;
            const int cnt = min(64, g.ns - m0);
            if (m < g.ns) {
                float *p = sh + lane * W;
                p[0] = (float)(ox + rr * g.Y[3 * m]);
                p[1] = (float)(oy + rr * g.Y[3 * m + 1]);
                p[2] = (float)(oz + rr * g.Y[3 * m + 2]);
                for (int r = 0; r < NRHS; ++r) p[3 + r] = phi[r * g.n_pad + m];
            }
            __syncthreads();
            float part[NRHS][NOUT];
            for (int r = 0; r < NRHS; ++r)
                for (int o = 0; o < NOUT; ++o) part[r][o] = 0.f;
            for (int jj = grp; jj < cnt; jj += ngrp) {
                const float *p = sh + jj * W;
                float dx = xl - p[0], dy = yl - p[1], dz = zl - p[2];
                float r2 = dx * dx + dy * dy + dz * dz;
                float inv = r2 > 0.f ? rsq(r2) : 0.f;
                float inv3 = inv * inv * inv;
                for (int r = 0; r < NRHS; ++r) {
                    float d = p[3 + r];
                    part[r][0] += d * inv;
                    if (FIELD) {
                        float di3 = d * inv3;
                        part[r][1] += di3 * dx;
                        part[r][2] += di3 * dy;
                        part[r][3] += di3 * dz;
                    }
                }
            }
            for (int r = 0; r < NRHS; ++r)
                for (int o = 0; o < NOUT; ++o) two_sum_into(hi[r][o], lo[r][o], part[r][o]);
            __syncthreads();
        }
    }

    // points: P2P (U list) and the direct W / X pairs
    for (int e = a.poff[leaf]; e < a.poff[leaf + 1]; ++e) {
        const int s0 = a.prng[2 * e], s1 = a.prng[2 * e + 1];
        for (int j0 = s0; j0 < s1; j0 += 64) {
            const int j = j0 + lane;
            const int cnt = min(64, s1 - j0);
            if (j < s1) {
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
            }
            __syncthreads();
            float part[NRHS][NOUT];
            for (int r = 0; r < NRHS; ++r)
                for (int o = 0; o < NOUT; ++o) part[r][o] = 0.f;
            for (int jj = grp; jj < cnt; jj += ngrp) {
                const float *p = sh + jj * W;
                float dx = xg - p[0], dy = yg - p[1], dz = zg - p[2];
                float r2 = dx * dx + dy * dy + dz * dz;
                float inv = (r2 >= a.delta2 && r2 > 0.f) ? rsq(r2) : 0.f;
                float inv3 = inv * inv * inv;
                int o = 3;
                for (int r = 0; r < NRHS; ++r) {
                    if (SL) {
                        float d = p[o++];
                        part[r][0] += d * inv;
                        if (FIELD) {
                            float di3 = d * inv3;
                            part[r][1] += di3 * dx;
                            part[r][2] += di3 * dy;
                            part[r][3] += di3 * dz;
                        }
                    }
                }
                if (DL) {
                    int od = 3 + (SL ? NRHS : 0);
                    for (int r = 0; r < NRHS; ++r) {
                        float md = p[od] * dx + p[od + 1] * dy + p[od + 2] * dz;
                        od += 3;
                        part[r][0] += md * inv3;
                    }
                }
            }
            for (int r = 0; r < NRHS; ++r)
                for (int o = 0; o < NOUT; ++o) two_sum_into(hi[r][o], lo[r][o], part[r][o]);
            __syncthreads();
        }
    }

    // combine the lane groups that share a target
    for (int off = tp; off < 64; off <<= 1) {
        for (int r = 0; r < NRHS; ++r)
            for (int o = 0; o < NOUT; ++o) {
                float h2 = __shfl_xor(hi[r][o], off);
                float l2 = __shfl_xor(lo[r][o], off);
                two_sum_into(hi[r][o], lo[r][o], h2);
                lo[r][o] += l2;
            }
    }
    if (grp == 0 && tvalid) {
        const int64_t dst = a.trg_perm ? a.trg_perm[k] : k;
        for (int r = 0; r < NRHS; ++r) {
            if (a.pot) a.pot[r * a.n_trg + dst] = (hi[r][0] + lo[r][0]) * kInv4Pi;
            if (FIELD && a.field) {
                float *f = a.field + ((int64_t)r * a.n_trg + dst) * 3;
                f[0] = (hi[r][1] + lo[r][1]) * kInv4Pi;
                f[1] = (hi[r][2] + lo[r][2]) * kInv4Pi;
                f[2] = (hi[r][3] + lo[r][3]) * kInv4Pi;
            }
        }
    }
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
