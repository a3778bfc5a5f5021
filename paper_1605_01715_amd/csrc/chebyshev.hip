// Interpolation kernels of the Chebyshev far field (Sec. III.A.1 Eq. p2m).
//
// Both kernels use the tensor-product structure of the interpolant,
// S(xbar_m, t) = S_x(i, t_x) S_y(j, t_y) S_z(k, t_z) for node m = (i n + j) n + k,
// with the 1D Lagrange polynomial of node i written as
// S(i, t) = sum_k coef[i][k] T_k(t) (T_k by the three-term recurrence, its
// derivative as k U_{k-1}). One wave handles one box.
//
// P2M: lane (j, k) owns the n nodes (0..n-1, j, k) and keeps their n sums in
// registers; each source is reduced once to the 3n values S_c(i, t_c) (and
// 3n derivatives for the double layer) when it is staged in LDS, so the
// inner loop costs 2 LDS reads and about 2n + 8 FMAs per (source, lane).
// The double layer uses
//   sum_j m . grad S = dS_x (m_x S_y S_z) + S_x (m_y dS_y S_z + m_z S_y dS_z).
//
// L2P: lane = target. The contraction over the n^3 node values (staged in
// LDS, read by broadcast) runs axis by axis: z inside, then y, then x.
#include "chebyshev.hpp"

namespace fmm {

namespace {

// T_k(t), k < N, and (if D) T_k'(t) = k U_{k-1}(t), into registers. The
// interpolation weights are formed in float64: a float32 weight is off by
// about 1e-7 absolute, and n^3 such errors against a smooth kernel do not
// cancel (they would cap the far field near 1e-6).
template <int N, bool D>
__device__ inline void cheb_basis(double t, double *tk, double *dtk) {
    tk[0] = 1.0;
    if (N > 1) tk[1] = t;
#pragma unroll
    for (int k = 2; k < N; ++k) tk[k] = 2.0 * t * tk[k - 1] - tk[k - 2];
    if (D) {
        double u0 = 1.0, u1 = 2.0 * t;  // U_0, U_1
        dtk[0] = 0.0;
        if (N > 1) dtk[1] = 1.0;
#pragma unroll
        for (int k = 2; k < N; ++k) {
            dtk[k] = k * u1;
            const double u2 = 2.0 * t * u1 - u0;
            u0 = u1;
            u1 = u2;
        }
    }
}

// S(i, t) and (if D) dS/dt for every node i of one axis; cf [N][N] float64.
template <int N, bool D, typename T>
__device__ inline void cheb_lagrange_1d(const double *cf, double t, T *s, T *ds) {
    double tk[N], dtk[N];
    cheb_basis<N, D>(t, tk, dtk);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double v = 0.0, dv = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            v += cf[i * N + k] * tk[k];
            if (D) dv += cf[i * N + k] * dtk[k];
        }
        s[i] = (T)v;
        if (D) ds[i] = (T)dv;
    }
}

template <int N, int NRHS, bool SL, bool DL>
__global__ __launch_bounds__(64) void k_points_to_nodes(const double *coef, const int32_t *items, const int32_t *roff,
                                                       const int32_t *rng, SurfaceGeom g, PointSrc src, float *out) {
    // per staged source: S_c(i) for c = x, y, z; dS_c(i) (DL); then q, m / h
    constexpr int OS = 0, OD = 3 * N, OQ = DL ? 6 * N : 3 * N, OM = OQ + (SL ? NRHS : 0);
    constexpr int W = OM + (DL ? 3 * NRHS : 0);
    __shared__ float sh[64 * W];
    __shared__ double cf[N * N];
    const int lane = threadIdx.x;
    const int b = items[blockIdx.x];
    if (lane < N * N) cf[lane] = coef[lane];
    const double cx = g.centre[3 * b], cy = g.centre[3 * b + 1], cz = g.centre[3 * b + 2];
    const double ih = 1.0 / g.half[b];
    const bool act = lane < N * N;
    const int jy = act ? lane / N : 0, kz = act ? lane % N : 0;
    // float64 sums: the Lagrange weights take both signs and cancel
    double acc[N][NRHS];
#pragma unroll
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < NRHS; ++r) acc[i][r] = 0.0;
    __syncthreads();
    for (int e = roff[blockIdx.x]; e < roff[blockIdx.x + 1]; ++e) {
        const int s0 = rng[2 * e], s1 = rng[2 * e + 1];
        for (int j0 = s0; j0 < s1; j0 += 64) {
            const int j = j0 + lane;
            const int cnt = min(64, s1 - j0);
            if (j >= s1 && lane < ((cnt + 1) & ~1)) {
                // the odd tail slot: a zero-strength record, so the loop below takes sources in pairs
                float *p = sh + lane * W;
                for (int k = 0; k < W; ++k) p[k] = 0.f;
            }
            if (j < s1) {
                float *p = sh + lane * W;
                const double t[3] = {((double)src.x[j] - cx) * ih, ((double)src.y[j] - cy) * ih,
                                     ((double)src.z[j] - cz) * ih};
#pragma unroll
                for (int c = 0; c < 3; ++c) cheb_lagrange_1d<N, DL>(cf, t[c], p + OS + c * N, p + OD + c * N);
                if (SL)
                    for (int r = 0; r < NRHS; ++r) p[OQ + r] = src.q[r * src.n + j];
                if (DL)
                    for (int r = 0; r < NRHS; ++r) {
                        p[OM + 3 * r] = (float)(src.mx[r * src.n + j] * ih);
                        p[OM + 3 * r + 1] = (float)(src.my[r * src.n + j] * ih);
                        p[OM + 3 * r + 2] = (float)(src.mz[r * src.n + j] * ih);
                    }
            }
            __syncthreads();
            // the weights of x-node i for one source: S_x(i) A + dS_x(i) B
            auto weights = [&](const float *p, float (&A)[NRHS], float (&B)[NRHS]) {
                const float sy = p[OS + N + jy], sz = p[OS + 2 * N + kz];
#pragma unroll
                for (int r = 0; r < NRHS; ++r) {
                    A[r] = SL ? p[OQ + r] * (sy * sz) : 0.f;
                    B[r] = 0.f;
                }
                if (DL) {
                    const float dsy = p[OD + N + jy], dsz = p[OD + 2 * N + kz];
#pragma unroll
                    for (int r = 0; r < NRHS; ++r) {
                        A[r] += p[OM + 3 * r + 1] * (dsy * sz) + p[OM + 3 * r + 2] * (sy * dsz);
                        B[r] = p[OM + 3 * r] * (sy * sz);
                    }
                }
            };
            for (int jj = 0; jj < cnt; jj += 2) {
                // two sources per step: their float32 terms are added, then one float64 add
                const float *p0 = sh + jj * W, *p1 = p0 + W;
                float A0[NRHS], B0[NRHS], A1[NRHS], B1[NRHS];
                weights(p0, A0, B0);
                weights(p1, A1, B1);
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const float sx0 = p0[OS + i], sx1 = p1[OS + i];
                    const float dsx0 = DL ? p0[OD + i] : 0.f, dsx1 = DL ? p1[OD + i] : 0.f;
#pragma unroll
                    for (int r = 0; r < NRHS; ++r) {
                        const float t0 = DL ? sx0 * A0[r] + dsx0 * B0[r] : sx0 * A0[r];
                        const float t1 = DL ? sx1 * A1[r] + dsx1 * B1[r] : sx1 * A1[r];
                        acc[i][r] += (double)(t0 + t1);
                    }
                }
            }
            __syncthreads();
        }
    }
    if (!act) return;
#pragma unroll
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < NRHS; ++r)
            out[((int64_t)b * NRHS + r) * g.n_pad + (i * N + jy) * N + kz] = (float)acc[i][r];
}

template <int N, int NRHS, bool FIELD>
__global__ __launch_bounds__(64) void k_nodes_to_points(const double *coef, EvalArgs a, SurfaceGeom g, const float *L) {
    constexpr int NN = N * N * N;
    // node values as stored (float32): every lane reads each of them, so LDS
    // return bandwidth, not arithmetic, bounds this kernel; float32 halves it
    // and the float64 arithmetic sees the same values
    __shared__ __align__(16) float sl[NRHS * NN];
    __shared__ double cf[N * N];
    const int lane = threadIdx.x;
    const int leaf = a.wleaf[blockIdx.x];
    const int64_t t_first = a.tbeg[leaf] + a.wt0[blockIdx.x];
    const int nt = (int)min((int64_t)64, a.tend[leaf] - t_first);
    if (lane < N * N) cf[lane] = coef[lane];
    {
        // all loads first, then the LDS writes (the loads overlap)
        constexpr int NV = (NN + 63) / 64;
        float lv[NRHS][NV];
#pragma unroll
        for (int r = 0; r < NRHS; ++r)
#pragma unroll
            for (int i = 0; i < NV; ++i)  // clamped index: no branch per load
                lv[r][i] = L[((int64_t)leaf * NRHS + r) * g.n_pad + min(lane + 64 * i, NN - 1)];
#pragma unroll
        for (int r = 0; r < NRHS; ++r)
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (lane + 64 * i < NN) sl[r * NN + lane + 64 * i] = lv[r][i];
    }
    __syncthreads();
    // SP lanes per target for short items (SP a power of two, nt SP <= 64):
    // lane part takes x-nodes i = part, part + SP, ..., and the SP partial
    // sums are added across the group's lanes at the end (a fixed order)
    int SP = 1;
    while (SP * 2 <= N && nt * SP * 2 <= 64) SP *= 2;
    const int part = lane & (SP - 1), tl = lane / SP;
    const bool valid = tl < nt;
    const int64_t k = t_first + (valid ? tl : 0);
    const double ih = 1.0 / g.half[leaf];
    const double tx = ((double)a.tx[k] - g.centre[3 * leaf]) * ih;
    const double ty = ((double)a.ty[k] - g.centre[3 * leaf + 1]) * ih;
    const double tz = ((double)a.tz[k] - g.centre[3 * leaf + 2]) * ih;
    double sy[N], sz[N], dsy[N], dsz[N], tk[N], dtk[N];
    cheb_lagrange_1d<N, FIELD>(cf, ty, sy, dsy);
    cheb_lagrange_1d<N, FIELD>(cf, tz, sz, dsz);
    cheb_basis<N, FIELD>(tx, tk, dtk);
    const int64_t dst = a.trg_perm ? a.trg_perm[k] : k;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) {
        const float *lr = sl + r * NN;
        double pot = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        // the x axis stays a loop (n^2 node values live at a time); S_x(i) is
        // formed from row i of the coefficients
#pragma unroll 1
        for (int i = part; i < N; i += SP) {
            double sxi = 0.0, dsxi = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                sxi += cf[i * N + q] * tk[q];
                if (FIELD) dsxi += cf[i * N + q] * dtk[q];
            }
            double bi = 0.0, biy = 0.0, biz = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                double az = 0.0, azd = 0.0;
#pragma unroll
                for (int kk = 0; kk < N; ++kk) {
                    const double l = (double)lr[(i * N + j) * N + kk];
                    az += sz[kk] * l;
                    if (FIELD) azd += dsz[kk] * l;
                }
                bi += sy[j] * az;
                if (FIELD) {
                    biy += dsy[j] * az;
                    biz += sy[j] * azd;
                }
            }
            pot += sxi * bi;
            if (FIELD) {
                gx += dsxi * bi;
                gy += sxi * biy;
                gz += sxi * biz;
            }
        }
        for (int o = 1; o < SP; o <<= 1) {
            pot += __shfl_xor(pot, o);
            if (FIELD) {
                gx += __shfl_xor(gx, o);
                gy += __shfl_xor(gy, o);
                gz += __shfl_xor(gz, o);
            }
        }
        if (!valid || part != 0) continue;
        if (a.pot) {
            float *pp = a.pot + r * a.n_trg + dst;
            *pp = a.accumulate ? (float)((double)*pp + pot) : (float)pot;
        }
        if (FIELD && a.field) {
            // field = -grad_x f = -(1/h) grad_t f
            float *f = a.field + ((int64_t)r * a.n_trg + dst) * 3;
            const double gr[3] = {-ih * gx, -ih * gy, -ih * gz};
            for (int c = 0; c < 3; ++c) f[c] = a.accumulate ? (float)((double)f[c] + gr[c]) : (float)gr[c];
        }
    }
}

// out (+)= (A_x (x) A_y (x) A_z) in with A_c = S[side_c] (M2M) or its
// transpose (L2L). Lane (q, s) = (lane / N, lane % N): the z pass gives
// T1[p'][q][s] (to LDS), the y pass T2[p'] for the lane's (q, s) in
// registers, the x pass accumulates out[p][q][s] for every p.
template <int N, int NRHS, bool L2L>
__global__ __launch_bounds__(64) void k_cheb_tensor(const double *s1, const int32_t *dst, const int32_t *src,
                                                   const int8_t *oct, const float *in, float *out, int n_pad) {
    constexpr int NN = N * N * N, NT = L2L ? 1 : 8;
    __shared__ double sm[2 * N * N];
    __shared__ double X[NN], T1[NN];
    const int lane = threadIdx.x, item = blockIdx.x;
    for (int e = lane; e < 2 * N * N; e += 64) sm[e] = s1[e];
    const bool act = lane < N * N;
    const int q = act ? lane / N : 0, sz = act ? lane % N : 0;
    // A_c[p][p'] from table side: S[side][p][p'] (M2M) or S[side][p'][p] (L2L)
    auto A = [&](int side, int p, int p2) { return L2L ? sm[(side * N + p2) * N + p] : sm[(side * N + p) * N + p2]; };
    const int64_t d = dst[item];
#pragma unroll 1
    for (int r = 0; r < NRHS; ++r) {
        double acc[N];
#pragma unroll
        for (int p = 0; p < N; ++p) acc[p] = 0.0;
#pragma unroll 1
        for (int t = 0; t < NT; ++t) {
            const int64_t sb = src[(int64_t)item * NT + t];
            if (sb < 0) continue;  // uniform across the wave
            const int o = L2L ? oct[item] : t;
            const int sx = (o >> 2) & 1, sy = (o >> 1) & 1, szd = o & 1;
            __syncthreads();  // sm loaded; the previous term is done with X and T1
            {
                // all loads first, then the LDS writes, so the loads are in
                // flight together rather than one latency each
                constexpr int NV = (NN + 63) / 64;
                float xv[NV];
#pragma unroll
                for (int i = 0; i < NV; ++i)  // clamped index: no branch per load
                    xv[i] = in[(sb * NRHS + r) * n_pad + min(lane + 64 * i, NN - 1)];
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    if (lane + 64 * i < NN) X[lane + 64 * i] = xv[i];
            }
            __syncthreads();
            if (act) {
                // z pass: T1[p'][q][s] = sum_s' A_z[s][s'] X[p'][q][s']
                double az[N];
#pragma unroll
                for (int s2 = 0; s2 < N; ++s2) az[s2] = A(szd, sz, s2);
#pragma unroll
                for (int p2 = 0; p2 < N; ++p2) {
                    double v = 0.0;
#pragma unroll
                    for (int s2 = 0; s2 < N; ++s2) v += az[s2] * X[(p2 * N + q) * N + s2];
                    T1[(p2 * N + q) * N + sz] = v;
                }
            }
            __syncthreads();
            if (act) {
                // y pass: T2[p'] = sum_q' A_y[q][q'] T1[p'][q'][s]
                double ay[N], t2[N];
#pragma unroll
                for (int q2 = 0; q2 < N; ++q2) ay[q2] = A(sy, q, q2);
#pragma unroll
                for (int p2 = 0; p2 < N; ++p2) {
                    double v = 0.0;
#pragma unroll
                    for (int q2 = 0; q2 < N; ++q2) v += ay[q2] * T1[(p2 * N + q2) * N + sz];
                    t2[p2] = v;
                }
                // x pass: acc[p] += sum_p' A_x[p][p'] T2[p']
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    double v = acc[p];
#pragma unroll
                    for (int p2 = 0; p2 < N; ++p2) v += A(sx, p, p2) * t2[p2];
                    acc[p] = v;
                }
            }
        }
        if (act) {
#pragma unroll
            for (int p = 0; p < N; ++p) {
                float *o = out + (d * NRHS + r) * n_pad + (p * N + q) * N + sz;
                *o = L2L ? (float)((double)*o + acc[p]) : (float)acc[p];
            }
        }
    }
}

#define FMM_CHEB_SWITCH(N_VAR, NRHS_VAR, CALL)                                      \
    switch ((N_VAR) * 8 + (NRHS_VAR)) {                                             \
    case 2 * 8 + 1: { constexpr int N = 2, R = 1; CALL; } break;                    \
    case 2 * 8 + 2: { constexpr int N = 2, R = 2; CALL; } break;                    \
    case 2 * 8 + 3: { constexpr int N = 2, R = 3; CALL; } break;                    \
    case 2 * 8 + 4: { constexpr int N = 2, R = 4; CALL; } break;                    \
    case 3 * 8 + 1: { constexpr int N = 3, R = 1; CALL; } break;                    \
    case 3 * 8 + 2: { constexpr int N = 3, R = 2; CALL; } break;                    \
    case 3 * 8 + 3: { constexpr int N = 3, R = 3; CALL; } break;                    \
    case 3 * 8 + 4: { constexpr int N = 3, R = 4; CALL; } break;                    \
    case 4 * 8 + 1: { constexpr int N = 4, R = 1; CALL; } break;                    \
    case 4 * 8 + 2: { constexpr int N = 4, R = 2; CALL; } break;                    \
    case 4 * 8 + 3: { constexpr int N = 4, R = 3; CALL; } break;                    \
    case 4 * 8 + 4: { constexpr int N = 4, R = 4; CALL; } break;                    \
    case 5 * 8 + 1: { constexpr int N = 5, R = 1; CALL; } break;                    \
    case 5 * 8 + 2: { constexpr int N = 5, R = 2; CALL; } break;                    \
    case 5 * 8 + 3: { constexpr int N = 5, R = 3; CALL; } break;                    \
    case 5 * 8 + 4: { constexpr int N = 5, R = 4; CALL; } break;                    \
    case 6 * 8 + 1: { constexpr int N = 6, R = 1; CALL; } break;                    \
    case 6 * 8 + 2: { constexpr int N = 6, R = 2; CALL; } break;                    \
    case 6 * 8 + 3: { constexpr int N = 6, R = 3; CALL; } break;                    \
    case 6 * 8 + 4: { constexpr int N = 6, R = 4; CALL; } break;                    \
    case 7 * 8 + 1: { constexpr int N = 7, R = 1; CALL; } break;                    \
    case 7 * 8 + 2: { constexpr int N = 7, R = 2; CALL; } break;                    \
    case 7 * 8 + 3: { constexpr int N = 7, R = 3; CALL; } break;                    \
    case 7 * 8 + 4: { constexpr int N = 7, R = 4; CALL; } break;                    \
    case 8 * 8 + 1: { constexpr int N = 8, R = 1; CALL; } break;                    \
    case 8 * 8 + 2: { constexpr int N = 8, R = 2; CALL; } break;                    \
    case 8 * 8 + 3: { constexpr int N = 8, R = 3; CALL; } break;                    \
    case 8 * 8 + 4: { constexpr int N = 8, R = 4; CALL; } break;                    \
    default: throw Error(FMM_ERR_ARG, "Chebyshev order must be 2..8 and nrhs 1..4"); \
    }

}  // namespace

void points_to_nodes(int nrhs, bool sl, bool dl, int n, const double *coef, const int32_t *items, int nitems,
                     const int32_t *roff, const int32_t *rng, const SurfaceGeom &g, const PointSrc &src, float *out,
                     hipStream_t s) {
    if (nitems <= 0) return;
    FMM_REQUIRE(g.ns == n * n * n && g.n_pad >= g.ns, "points_to_nodes: node count does not match the order");
    dim3 gr(nitems), bl(64);
    if (sl && dl) {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_points_to_nodes<N, R, true, true>), gr, bl, 0, s, coef, items,
                                                    roff, rng, g, src, out));
    } else if (dl) {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_points_to_nodes<N, R, false, true>), gr, bl, 0, s, coef, items,
                                                    roff, rng, g, src, out));
    } else {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_points_to_nodes<N, R, true, false>), gr, bl, 0, s, coef, items,
                                                    roff, rng, g, src, out));
    }
    FMM_HIP(hipGetLastError());
}

void cheb_tensor(int nrhs, int n, bool l2l, const double *s1, int nitems, const int32_t *dst, const int32_t *src,
                 const int8_t *oct, const float *in, float *out, int n_pad, hipStream_t s) {
    if (nitems <= 0) return;
    FMM_REQUIRE(n_pad >= n * n * n, "cheb_tensor: rows shorter than n^3");
    dim3 gr(nitems), bl(64);
    if (l2l) {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_cheb_tensor<N, R, true>), gr, bl, 0, s, s1, dst, src, oct, in,
                                                    out, n_pad));
    } else {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_cheb_tensor<N, R, false>), gr, bl, 0, s, s1, dst, src, oct, in,
                                                    out, n_pad));
    }
    FMM_HIP(hipGetLastError());
}

void nodes_to_points(int nrhs, int n, const double *coef, const EvalArgs &a, const SurfaceGeom &g, const float *L,
                     hipStream_t s) {
    if (a.nwork <= 0) return;
    FMM_REQUIRE(g.ns == n * n * n && g.n_pad >= g.ns, "nodes_to_points: node count does not match the order");
    dim3 gr(a.nwork), bl(64);
    if (a.field) {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_nodes_to_points<N, R, true>), gr, bl, 0, s, coef, a, g, L));
    } else {
        FMM_CHEB_SWITCH(n, nrhs, hipLaunchKernelGGL((k_nodes_to_points<N, R, false>), gr, bl, 0, s, coef, a, g, L));
    }
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
