// Surfaces, check-to-equivalent pseudo-inverses and translation operators.
//
// The paper's far field (Sec. III.A.1 Eq. p2m) is an interpolation at the
// sources, a translation with the plain 1/r kernel and an interpolation at the
// targets; here the interpolation is by equivalent densities on box surfaces
// (kernel-independent FMM with equivalent surfaces). Each map is built once
// per order p on the unit box in float64: the Laplace kernel is homogeneous
// of degree -1, so a box of half-width r uses the same matrices, and the
// equivalent density of a box is r times the unit-box pseudo-inverse applied
// to its check potential.
//
// The pseudo-inverse has entries of order 1/(eps sigma_max), which float32
// cannot apply without catastrophic cancellation. So the translations are
// pre-multiplied by it in float64 and act on check potentials, and the
// pseudo-inverse itself is only applied in float64 (right before the
// evaluation at the targets).
#include "operators.hpp"

#include <cmath>
#include <map>
#include <mutex>

#include "gemm.hpp"

namespace fmm {

std::vector<double> unit_surface(int p) {
    std::vector<double> Y;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k)
                if (i == 0 || i == p - 1 || j == 0 || j == p - 1 || k == 0 || k == p - 1) {
                    Y.push_back(-1.0 + 2.0 * i / (p - 1));
                    Y.push_back(-1.0 + 2.0 * j / (p - 1));
                    Y.push_back(-1.0 + 2.0 * k / (p - 1));
                }
    return Y;
}

// Threshold tuned for float32 application: 1e-8 keeps the pre-multiplied
// translations well enough conditioned that float32 products lose little,
// while the float64 approximation error stays far below the float32 floor.
double default_pinv_eps(int p) {
    (void)p;
    return 1e-8;
}

// One-sided (Hestenes) Jacobi SVD: rotate column pairs of W = K until they are
// orthogonal; then sigma_k = |w_k|, u_k = w_k / sigma_k, and V accumulates the
// rotations. Pairs are visited in round-robin order so that each round's
// rotations touch disjoint columns and run in parallel.
std::vector<double> pinv_jacobi(const std::vector<double> &K, int n, double eps) {
    std::vector<double> W((size_t)n * n), V((size_t)n * n, 0.0);  // column-major
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) W[(size_t)j * n + i] = K[(size_t)i * n + j];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    const int nn = n + (n & 1);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int r = 0; r < nn - 1; ++r) {
#pragma omp parallel for schedule(static) reduction(max : off)
            for (int k = 0; k < nn / 2; ++k) {
                int i, j;
                if (k == 0) {
                    i = r;
                    j = nn - 1;
                } else {
                    i = (r + k) % (nn - 1);
                    j = (r - k + nn - 1) % (nn - 1);
                }
                if (i > j) std::swap(i, j);
                if (j >= n) continue;
                double *wi = &W[(size_t)i * n], *wj = &W[(size_t)j * n];
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int q = 0; q < n; ++q) {
                    al += wi[q] * wi[q];
                    be += wj[q] * wj[q];
                    ga += wi[q] * wj[q];
                }
                if (al == 0.0 || be == 0.0) continue;
                double rel = std::fabs(ga) / std::sqrt(al * be);
                if (rel < 1e-15) continue;
                off = std::max(off, rel);
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int q = 0; q < n; ++q) {
                    double a = wi[q], b = wj[q];
                    wi[q] = c * a - s * b;
                    wj[q] = s * a + c * b;
                }
                double *vi = &V[(size_t)i * n], *vj = &V[(size_t)j * n];
                for (int q = 0; q < n; ++q) {
                    double a = vi[q], b = vj[q];
                    vi[q] = c * a - s * b;
                    vj[q] = s * a + c * b;
                }
            }
        }
        if (off < 1e-14) break;
    }
    std::vector<double> sig(n);
    double smax = 0.0;
    for (int k = 0; k < n; ++k) {
        double s2 = 0.0;
        for (int q = 0; q < n; ++q) s2 += W[(size_t)k * n + q] * W[(size_t)k * n + q];
        sig[k] = std::sqrt(s2);
        smax = std::max(smax, sig[k]);
    }
    // pinv = sum_k v_k u_k^T / sigma_k = sum_k v_k w_k^T / sigma_k^2
    std::vector<double> P((size_t)n * n, 0.0);  // row-major
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < n; ++k) {
            if (!(sig[k] > eps * smax)) continue;
            double f = V[(size_t)k * n + i] / (sig[k] * sig[k]);
            const double *wk = &W[(size_t)k * n];
            double *row = &P[(size_t)i * n];
            for (int j = 0; j < n; ++j) row[j] += f * wk[j];
        }
    }
    return P;
}

namespace {

std::shared_ptr<Operators> build_operators(int p, double eps, hipStream_t s) {
    auto op = std::make_shared<Operators>();
    op->p = p;
    op->eps = eps;
    op->Y = unit_surface(p);
    const int n = op->ns = (int)op->Y.size() / 3;
    const int np = op->n_pad = ((n + 31) / 32) * 32;
    op->mat_elems = (size_t)np * np;
    op->dY = upload(op->Y, s);

    // UC2E = pinv(G(2.95 Y, 1.05 Y)); DC2E = pinv(G(1.05 Y, 2.95 Y)) = UC2E^T
    std::vector<double> K((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double dx = kRadOut * op->Y[3 * i + c] - kRadIn * op->Y[3 * j + c];
                d2 += dx * dx;
            }
            K[(size_t)i * n + j] = 1.0 / (kFourPi * std::sqrt(d2));
        }
    std::vector<double> uc2e = pinv_jacobi(K, n, eps);
    std::vector<double> dc2e((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) dc2e[(size_t)i * n + j] = uc2e[(size_t)j * n + i];
    op->uc2e_host = uc2e;
    DBuf<double> d_uc2e = upload(uc2e, s), d_dc2e = upload(dc2e, s);

    op->uc2e_f64.alloc(op->mat_elems);
    op->dc2e_f64.alloc(op->mat_elems);
    to_frag_f64(d_uc2e.p, n, np, op->uc2e_f64.p, s);
    to_frag_f64(d_dc2e.p, n, np, op->dc2e_f64.p, s);

    // translation matrices: G built on the device, multiplied by the C2E map in float64
    auto build = [&](const std::vector<double> &prm, const DBuf<double> &c2e, DBuf<float> *f32,
                     DBuf<uint16_t> *bf, DBuf<double> *f64) {
        const int nb = (int)prm.size() / 9;
        if (f32) f32->alloc((size_t)nb * op->mat_elems);
        if (bf) bf->alloc((size_t)nb * 3 * op->mat_elems);
        if (f64) f64->alloc((size_t)nb * op->mat_elems);
        const int chunk = 32;
        DBuf<double> G((size_t)chunk * n * n), C((size_t)chunk * n * n);
        for (int b0 = 0; b0 < nb; b0 += chunk) {
            int cnt = std::min(chunk, nb - b0);
            std::vector<double> sub(prm.begin() + 9 * b0, prm.begin() + 9 * (b0 + cnt));
            DBuf<double> dprm = upload(sub, s);
            build_laplace_mats(op->dY.p, n, cnt, dprm.p, G.p, s);
            dgemm_batched(G.p, c2e.p, C.p, n, cnt, s);
            for (int b = 0; b < cnt; ++b) {
                const double *Cb = C.p + (size_t)b * n * n;
                if (f32) to_frag_f32(Cb, n, np, f32->p + (size_t)(b0 + b) * op->mat_elems, s);
                if (bf) to_frag_bf16x3(Cb, n, np, bf->p + (size_t)(b0 + b) * 3 * op->mat_elems, s);
                if (f64) to_frag_f64(Cb, n, np, f64->p + (size_t)(b0 + b) * op->mat_elems, s);
            }
            FMM_HIP(hipStreamSynchronize(s));
        }
    };
    auto sgn = [](int o, int c) { return ((o >> (2 - c)) & 1) ? 1.0 : -1.0; };
    std::vector<double> pm2m, pl2l, pm2l;
    for (int o = 0; o < 8; ++o) {
        // parent check (unit, origin) <- child equivalent (centre s_o/2, radius 0.525)
        pm2m.insert(pm2m.end(), {0.0, 0.0, 0.0, kRadOut, 0.5 * sgn(o, 0), 0.5 * sgn(o, 1), 0.5 * sgn(o, 2),
                                 0.5 * kRadIn, 0.5});
        // child check (centre s_o/2, radius 0.525) <- parent downward equivalent (unit)
        pl2l.insert(pl2l.end(), {0.5 * sgn(o, 0), 0.5 * sgn(o, 1), 0.5 * sgn(o, 2), 0.5 * kRadIn, 0.0, 0.0, 0.0,
                                 kRadOut, 1.0});
    }
    for (int i = -3; i <= 3; ++i)
        for (int j = -3; j <= 3; ++j)
            for (int k = -3; k <= 3; ++k)
                if (std::max(std::abs(i), std::max(std::abs(j), std::abs(k))) >= 2)
                    pm2l.insert(pm2l.end(), {0.0, 0.0, 0.0, kRadIn, 2.0 * i, 2.0 * j, 2.0 * k, kRadIn, 1.0});
    build(pm2m, d_uc2e, nullptr, nullptr, &op->m2m_f64);
    build(pl2l, d_dc2e, nullptr, nullptr, &op->l2l_f64);
    build(pm2l, d_uc2e, &op->m2l_f32, &op->m2l_bf, nullptr);
    FMM_HIP(hipStreamSynchronize(s));
    return op;
}

}  // namespace

std::shared_ptr<const Operators> get_operators(int p, double eps, hipStream_t s) {
    // Held until the process ends (never destroyed, so no device memory is
    // freed after the HIP runtime has shut down).
    static std::mutex mu;
    static auto *cache = new std::map<std::tuple<int, int, double>, std::shared_ptr<Operators>>();
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, p, eps);
    auto it = cache->find(key);
    if (it != cache->end()) return it->second;
    auto op = build_operators(p, eps, s);
    (*cache)[key] = op;
    return op;
}

}  // namespace fmm
