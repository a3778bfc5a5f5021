// Matrix-free restarted GMRES on the device (gmres_solve in include/fmm.h).
//
// The paper solves its dense boundary-integral systems with GMRES in
// matrix-free form: only the action of A is defined, and the boundary integral
// inside it is the dominant cost (Sec. III, electrostatic problem). Here every
// iteration is one FMM apply plus float64 vector work on the device:
// classical Gram-Schmidt applied twice (CGS2) for the Arnoldi step, its dot
// products reduced on the device and brought back in one copy per step, the
// small Hessenberg least-squares problem kept triangular by Givens rotations
// on the host, and the true residual recomputed at every restart.
#include <cmath>

#include "plan.hpp"

namespace fmm {

namespace {

constexpr int kBlock = 256;
constexpr int kDotBlocks = 240;

// partial[k][blk] = sum over this block's share of V[k] . w, for k < nk
__global__ __launch_bounds__(kBlock) void k_multi_dot(const double *V, int64_t ldv, int nk, const double *w,
                                                      int64_t n, double *partial) {
    __shared__ double sh[kBlock];
    const int k = blockIdx.y;
    double acc = 0.0;
    const double *v = V + (int64_t)k * ldv;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        acc += v[i] * w[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)k * gridDim.x + blockIdx.x] = sh[0];
}

// out[k] = sum over blocks of partial[k][blk], reduced in a fixed tree order
// (one workgroup per k; deterministic)
__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double *partial, int nblk, double *out) {
    __shared__ double sh[kBlock];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) acc += partial[(int64_t)k * nblk + b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
}

// w -= sum_k h[k] V[k]
__global__ void k_multi_axpy(const double *V, int64_t ldv, int nk, const double *h, double *w, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double acc = w[i];
    for (int k = 0; k < nk; ++k) acc -= h[k] * V[(int64_t)k * ldv + i];
    w[i] = acc;
}

// v /= sqrt(*sumsq) unless sqrt(*sumsq) <= floor (Arnoldi breakdown: v is left as it is)
__global__ void k_normalise(double *v, const double *sumsq, double floor, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double nrm = sqrt(*sumsq);
    if (i < n && !(nrm <= floor)) v[i] = v[i] / nrm;
}

// x += sum_k y[k] V[k]
__global__ void k_update(const double *V, int64_t ldv, int nk, const double *y, double *x, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double acc = x[i];
    for (int k = 0; k < nk; ++k) acc += y[k] * V[(int64_t)k * ldv + i];
    x[i] = acc;
}

__global__ void k_scale(const double *in, double s, double *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = in[i] * s;
}

__global__ void k_sub(const double *a, const double *b, double *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_density(const double *x, const float *w, float *dens, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dens[i] = (float)(x[i] * (double)w[i]);
}

// y = a x + pot                      (FK)
// y = a x + c (field . n)            (dielectric)
__global__ void k_finish(int kind, const double *x, const float *a, const float *c, const float *pot,
                         const float *field, const float *nrm, double *y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double v = (double)a[i] * x[i];
    if (kind == FMM_OP_FK) {
        v += (double)pot[i];
    } else {
        double en = (double)field[3 * i] * nrm[3 * i] + (double)field[3 * i + 1] * nrm[3 * i + 1] +
                    (double)field[3 * i + 2] * nrm[3 * i + 2];
        v += (double)c[i] * en;
    }
    y[i] = v;
}

struct Gmres {
    Plan &P;
    const fmm_operator &op;
    hipStream_t s;
    int64_t n;
    int kmax;                        // most vectors a Gram-Schmidt pass works on (restart + 1)
    DBuf<float> dens, pot, field;
    DBuf<double> partial;            // [kmax][kDotBlocks] per-block dot products
    DBuf<double> hdev;               // [2 kmax + 1]: both Gram-Schmidt passes and the squared norm
    std::vector<double> hhost;

    Gmres(Plan &p, const fmm_operator &o, int restart, hipStream_t st)
        : P(p), op(o), s(st), n(p.t.n_src), kmax(restart + 1) {
        dens.alloc(n);
        if (op.kind == FMM_OP_FK) pot.alloc(n);
        else field.alloc(3 * n);
        partial.alloc((size_t)kDotBlocks * kmax);
        hdev.alloc(2 * (size_t)kmax + 1);
        hhost.resize(2 * (size_t)kmax + 1);
    }

    void matvec(const double *x, double *y) {
        hipLaunchKernelGGL(k_density, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, x, op.w, dens.p, n);
        FMM_HIP(hipGetLastError());
        // the same buffers every iteration: with graph replay on, one capture per solve
        const float *q = op.kind == FMM_OP_FK ? nullptr : dens.p;
        const float *mu = op.kind == FMM_OP_FK ? dens.p : nullptr;
        float *pt = op.kind == FMM_OP_FK ? pot.p : nullptr;
        float *fd = op.kind == FMM_OP_FK ? nullptr : field.p;
        if (P.graph.enabled && !P.timing)
            plan_apply_graph(P, q, mu, pt, fd, s);
        else
            plan_apply(P, q, mu, pt, fd, s);
        hipLaunchKernelGGL(k_finish, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, op.kind, x, op.a, op.c, pot.p,
                           field.p, P.trg_nrm_user.p, y, n);
        FMM_HIP(hipGetLastError());
    }

    // hd[k] = V[k] . w for k < nk, on the device (deterministic two-level sum)
    void dots(const double *V, int64_t ldv, int nk, const double *w, double *hd) {
        if (nk > kmax) throw Error(FMM_ERR_ARG, "gmres: more Krylov vectors than the restart length");
        hipLaunchKernelGGL(k_multi_dot, dim3(kDotBlocks, nk), dim3(kBlock), 0, s, V, ldv, nk, w, n, partial.p);
        FMM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_reduce_partials, dim3(nk), dim3(kBlock), 0, s, partial.p, kDotBlocks, hd);
        FMM_HIP(hipGetLastError());
    }
    double norm(const double *v) {
        dots(v, 0, 1, v, hdev.p);
        double h;
        d2h(&h, hdev.p, 1, s);
        return std::sqrt(h);
    }
    void axpy_many(const double *V, int64_t ldv, int nk, const double *hd, double *w) {
        hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, V, ldv, nk, hd, w, n);
        FMM_HIP(hipGetLastError());
    }

    // One Arnoldi step's orthogonalisation of w against V[0..nk): classical
    // Gram-Schmidt twice, then w normalised unless its norm is at most
    // `floor`. Everything stays on the device; one copy brings back both
    // passes' coefficients (summed into h[0..nk)) and the norm.
    double cgs2(const double *V, int64_t ldv, int nk, double *w, double floor, double *h) {
        double *h1 = hdev.p, *h2 = hdev.p + kmax, *nn = hdev.p + 2 * kmax;
        dots(V, ldv, nk, w, h1);
        axpy_many(V, ldv, nk, h1, w);
        dots(V, ldv, nk, w, h2);
        axpy_many(V, ldv, nk, h2, w);
        dots(w, 0, 1, w, nn);
        hipLaunchKernelGGL(k_normalise, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, w, nn, floor, n);
        FMM_HIP(hipGetLastError());
        d2h(hhost.data(), hdev.p, hhost.size(), s);
        for (int i = 0; i < nk; ++i) h[i] = hhost[i] + hhost[kmax + i];
        return std::sqrt(hhost[2 * kmax]);
    }
};

}  // namespace

void plan_gmres(Plan &P, const fmm_operator &op, const double *b, double *x, double rtol, int restart, int max_iter,
                int *iters_out, double *rel_out, int *status, hipStream_t s) {
    Gmres G(P, op, restart, s);
    const int64_t n = G.n;
    const int m = restart;
    DBuf<double> V((size_t)(m + 1) * n), w(n), r(n), dy(m);
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1);
    const double bnorm = G.norm(b);
    int iters = 0;
    *status = FMM_OK;
    if (bnorm == 0.0) {
        FMM_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
        *iters_out = 0;
        *rel_out = 0.0;
        FMM_HIP(hipStreamSynchronize(s));
        return;
    }
    double rel = 0.0;
    while (true) {
        G.matvec(x, w.p);
        hipLaunchKernelGGL(k_sub, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, b, w.p, r.p, n);
        FMM_HIP(hipGetLastError());
        const double beta = G.norm(r.p);
        rel = beta / bnorm;
        if (rel <= rtol) break;
        if (iters >= max_iter) {
            *status = FMM_ERR_NOT_CONVERGED;
            break;
        }
        hipLaunchKernelGGL(k_scale, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, r.p, 1.0 / beta, V.p, n);
        FMM_HIP(hipGetLastError());
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        const int mm = std::min(m, max_iter - iters);
        const double floor = 1e-14 * beta;
        for (int j = 0; j < mm; ++j) {
            double *vj1 = V.p + (int64_t)(j + 1) * n;
            G.matvec(V.p + (int64_t)j * n, vj1);
            const double hn = G.cgs2(V.p, n, j + 1, vj1, floor, h.data());
            const bool breakdown = hn <= floor;
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
            cs[j] = H[(size_t)j * m + j] / den;
            sn[j] = H[(size_t)(j + 1) * m + j] / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            k = j + 1;
            if (std::fabs(g[j + 1]) / bnorm <= rtol || breakdown) break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= H[(size_t)i * m + l] * y[l];
            y[i] = acc / H[(size_t)i * m + i];
        }
        h2d(dy.p, y.data(), k, s);
        hipLaunchKernelGGL(k_update, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, V.p, n, k, dy.p, x, n);
        FMM_HIP(hipGetLastError());
    }
    FMM_HIP(hipStreamSynchronize(s));
    *iters_out = iters;
    *rel_out = rel;
}

}  // namespace fmm
