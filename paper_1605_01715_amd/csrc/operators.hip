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

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "gemm.hpp"
#include "m2l.hpp"

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
double default_pinv_eps(int basis, int p) {
    // Chebyshev basis: interpolation error falls about 7x per order (~3e-5 at
    // n = 5, ~1e-6 at n = 7 on clustered clouds); keep the M2L truncation an
    // order below it
    if (basis == kBasisChebyshev) return std::max(1e-7, std::pow(10.0, -(p + 1)));
    return 1e-8;
}

// One-sided (Hestenes) Jacobi SVD: rotate column pairs of W = K until they are
// orthogonal; then sigma_k = |w_k|, u_k = w_k / sigma_k, and V accumulates the
// rotations. Pairs are visited in round-robin order so that each round's
// rotations touch disjoint columns and run in parallel.
void svd_jacobi(const std::vector<double> &K, int n, std::vector<double> &U, std::vector<double> &s,
                std::vector<double> &Vout) {
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
                double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                for (int q = 0; q < n; ++q) {
                    double a = wi[q], b = wj[q];
                    wi[q] = c * a - sn * b;
                    wj[q] = sn * a + c * b;
                }
                double *vi = &V[(size_t)i * n], *vj = &V[(size_t)j * n];
                for (int q = 0; q < n; ++q) {
                    double a = vi[q], b = vj[q];
                    vi[q] = c * a - sn * b;
                    vj[q] = sn * a + c * b;
                }
            }
        }
        if (off < 1e-14) break;
    }
    std::vector<double> sig(n);
    for (int k = 0; k < n; ++k) {
        double s2 = 0.0;
        for (int q = 0; q < n; ++q) s2 += W[(size_t)k * n + q] * W[(size_t)k * n + q];
        sig[k] = std::sqrt(s2);
    }
    std::vector<int> ord(n);
    for (int k = 0; k < n; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sig[a] > sig[b]; });
    U.assign((size_t)n * n, 0.0);
    Vout.assign((size_t)n * n, 0.0);
    s.assign(n, 0.0);
    for (int c = 0; c < n; ++c) {
        const int k = ord[c];
        s[c] = sig[k];
        for (int q = 0; q < n; ++q) {
            U[(size_t)q * n + c] = sig[k] > 0.0 ? W[(size_t)k * n + q] / sig[k] : 0.0;
            Vout[(size_t)q * n + c] = V[(size_t)k * n + q];
        }
    }
}

std::vector<double> pinv_jacobi(const std::vector<double> &K, int n, double eps) {
    std::vector<double> U, s, V;
    svd_jacobi(K, n, U, s, V);
    std::vector<double> P((size_t)n * n, 0.0);
    const double smax = n ? s[0] : 0.0;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            if (!(s[k] > eps * smax)) continue;
            const double f = V[(size_t)i * n + k] / s[k];
            for (int j = 0; j < n; ++j) P[(size_t)i * n + j] += f * U[(size_t)j * n + k];
        }
    return P;
}

namespace {

// Translations C_b = left (r x n) * G_b * right (n x r), one per 9-double entry
// of prm (G_b as in build_laplace_mats, over the n points of dY), written as
// float64 fragments r_pad x r_pad (f64) and/or row-major float32 padded to
// r_pad x r_pad (rm). G is built on the device in chunks of 32.
void build_translations(const double *dY, int n, int r, int rp, const std::vector<double> &prm, const double *left,
                        const double *right, DBuf<double> *f64, DBuf<float> *rm, hipStream_t s) {
    const int nb = (int)prm.size() / 9;
    const size_t rr = (size_t)rp * rp;
    if (f64) f64->alloc((size_t)nb * rr);
    if (rm) rm->alloc((size_t)nb * rr);
    const int chunk = 32;
    DBuf<double> G((size_t)chunk * n * n), X((size_t)chunk * n * r), C((size_t)chunk * r * r);
    for (int b0 = 0; b0 < nb; b0 += chunk) {
        int cnt = std::min(chunk, nb - b0);
        std::vector<double> sub(prm.begin() + 9 * b0, prm.begin() + 9 * (b0 + cnt));
        DBuf<double> dprm = upload(sub, s);
        build_laplace_mats(dY, n, cnt, dprm.p, G.p, s);
        dgemm_batched(G.p, (size_t)n * n, right, 0, X.p, (size_t)n * r, n, r, n, cnt, s);
        dgemm_batched(left, 0, X.p, (size_t)n * r, C.p, (size_t)r * r, r, r, n, cnt, s);
        for (int b = 0; b < cnt; ++b) {
            const double *Cb = C.p + (size_t)b * r * r;
            if (f64) to_frag_f64(Cb, r, r, rp, rp, f64->p + (size_t)(b0 + b) * rr, s);
            if (rm) to_padded_f32(Cb, r, r, rp, rp, rm->p + (size_t)(b0 + b) * rr, s);
        }
        FMM_HIP(hipStreamSynchronize(s));
    }
}

// The 316 M2L directions d in {-3..3}^3 with max |d_c| >= 2, in (i, j, k)
// lexicographic order, as 9-double entries for build_laplace_mats: targets
// at ro * Y around the origin, sources at rs * Y around 2 d.
std::vector<double> m2l_params(double ro, double rs) {
    std::vector<double> prm;
    for (int i = -3; i <= 3; ++i)
        for (int j = -3; j <= 3; ++j)
            for (int k = -3; k <= 3; ++k)
                if (std::max(std::abs(i), std::max(std::abs(j), std::abs(k))) >= 2)
                    prm.insert(prm.end(), {0.0, 0.0, 0.0, ro, 2.0 * i, 2.0 * j, 2.0 * k, rs, 1.0});
    return prm;
}

// ---- on-disk cache of the float64 factorisations the operators start from
// (the SVD of the check-to-equivalent map of the surface form, the
// eigenvectors of the Chebyshev form's Gram matrix). They depend on the form
// and the order only (the threshold truncates them afterwards) and take most
// of the build time (a host Jacobi SVD of an n_s x n_s matrix). Directory:
// FMM_OP_CACHE, else ~/.cache/fmm_mi355x_ops; FMM_OP_CACHE=0 turns it off.
// A file holds a header (tag, format version, form, order, the surface radii,
// array lengths) and a checksum of the data; a file that does not match is
// ignored and rewritten. Files are written under a temporary name and renamed.
constexpr char kOpTag[8] = {'F', 'M', 'M', 'O', 'P', 'S', '0', '1'};
struct FactorHeader {
    char tag[8];
    int32_t form, order, narr, pad;
    double rad_in, rad_out;
    int64_t len[4];
    uint64_t sum;  // FNV-1a over the data bytes
};

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

std::string factor_path(int form, int order) {
    const char *dir = std::getenv("FMM_OP_CACHE");
    std::string d;
    if (dir) {
        if (!*dir || std::string(dir) == "0") return "";
        d = dir;
    } else {
        const char *home = std::getenv("HOME");
        if (!home) return "";
        d = std::string(home) + "/.cache/fmm_mi355x_ops";
    }
    return d + "/" + (form == kBasisChebyshev ? "cheb" : "surface") + "_" + std::to_string(order) + ".f64";
}

FactorHeader factor_header(int form, int order, const std::vector<std::vector<double> *> &arrs) {
    FactorHeader h{};
    std::memcpy(h.tag, kOpTag, 8);
    h.form = form;
    h.order = order;
    h.narr = (int)arrs.size();
    h.rad_in = kRadIn;
    h.rad_out = kRadOut;
    for (size_t a = 0; a < arrs.size(); ++a) h.len[a] = (int64_t)arrs[a]->size();
    return h;
}

// Fills arrs (sized by the caller) from the cache file; false if absent or not matching.
bool load_factors(int form, int order, const std::vector<std::vector<double> *> &arrs) {
    const std::string path = factor_path(form, order);
    if (path.empty()) return false;
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    const FactorHeader want = factor_header(form, order, arrs);
    FactorHeader got{};
    bool ok = std::fread(&got, sizeof got, 1, f) == 1 && std::memcmp(got.tag, want.tag, 8) == 0 &&
              got.form == want.form && got.order == want.order && got.narr == want.narr &&
              got.rad_in == want.rad_in && got.rad_out == want.rad_out;
    for (size_t a = 0; ok && a < arrs.size(); ++a) ok = got.len[a] == want.len[a];
    uint64_t sum = 1469598103934665603ull;
    for (size_t a = 0; ok && a < arrs.size(); ++a) {
        ok = std::fread(arrs[a]->data(), sizeof(double), arrs[a]->size(), f) == arrs[a]->size();
        if (ok) sum = fnv1a(arrs[a]->data(), arrs[a]->size() * sizeof(double), sum);
    }
    ok = ok && sum == got.sum && std::fgetc(f) == EOF;
    std::fclose(f);
    FMM_LOG("operators: factors %s %s\n", path.c_str(), ok ? "read" : "do not match; rebuilt");
    return ok;
}

void save_factors(int form, int order, const std::vector<std::vector<double> *> &arrs) {
    const std::string path = factor_path(form, order);
    if (path.empty()) return;
    // create the directory and its parents (existing ones are fine)
    const std::string dir = path.substr(0, path.rfind('/'));
    for (size_t k = 1; k <= dir.size(); ++k)
        if (k == dir.size() || dir[k] == '/') (void)mkdir(dir.substr(0, k).c_str(), 0755);
    FactorHeader h = factor_header(form, order, arrs);
    uint64_t sum = 1469598103934665603ull;
    for (auto *a : arrs) sum = fnv1a(a->data(), a->size() * sizeof(double), sum);
    h.sum = sum;
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;  // the cache is an optimisation: no file, no error
    bool ok = std::fwrite(&h, sizeof h, 1, f) == 1;
    for (auto *a : arrs) ok = ok && std::fwrite(a->data(), sizeof(double), a->size(), f) == a->size();
    ok = (std::fclose(f) == 0) && ok;
    if (ok && std::rename(tmp.c_str(), path.c_str()) == 0) {
        FMM_LOG("operators: factors written to %s\n", path.c_str());
    } else {
        std::remove(tmp.c_str());
    }
}

std::shared_ptr<Operators> build_operators(int p, double eps, hipStream_t s) {
    auto op = std::make_shared<Operators>();
    op->p = p;
    op->eps = eps;
    op->Y = unit_surface(p);
    const int n = op->ns = (int)op->Y.size() / 3;
    const int np = op->n_pad = ((n + 31) / 32) * 32;
    op->dY = upload(op->Y, s);

    // K = G(2.95 Y, 1.05 Y) = U S V^T, truncated at eps * sigma_max
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
    std::vector<double> Uf((size_t)n * n), sv(n), Vf((size_t)n * n);
    if (!load_factors(kBasisSurface, p, {&Uf, &sv, &Vf})) {
        svd_jacobi(K, n, Uf, sv, Vf);
        save_factors(kBasisSurface, p, {&Uf, &sv, &Vf});
    }
    int r = 0;
    while (r < n && sv[r] > eps * sv[0]) ++r;
    const int rp = ((r + 31) / 32) * 32;
    op->r = r;
    op->r_pad = rp;
    // host factors: Ur, Vr [n][r]; expansions U S^-1, V S^-1; projections U^T, V^T [r][n]
    std::vector<double> Ur((size_t)n * r), Vr((size_t)n * r), UrSi((size_t)n * r), VrSi((size_t)n * r);
    std::vector<double> PU((size_t)r * n), PV((size_t)r * n);
    for (int q = 0; q < n; ++q)
        for (int k = 0; k < r; ++k) {
            Ur[(size_t)q * r + k] = Uf[(size_t)q * n + k];
            Vr[(size_t)q * r + k] = Vf[(size_t)q * n + k];
            UrSi[(size_t)q * r + k] = Uf[(size_t)q * n + k] / sv[k];
            VrSi[(size_t)q * r + k] = Vf[(size_t)q * n + k] / sv[k];
            PU[(size_t)k * n + q] = Uf[(size_t)q * n + k];
            PV[(size_t)k * n + q] = Vf[(size_t)q * n + k];
        }
    op->U = Ur;
    op->V = Vr;
    DBuf<double> dUrSi = upload(UrSi, s), dVrSi = upload(VrSi, s), dPU = upload(PU, s), dPV = upload(PV, s);
    const size_t rr = (size_t)rp * rp;
    op->pu_f64.alloc((size_t)rp * np);
    op->pv_f64.alloc((size_t)rp * np);
    op->cu_f64.alloc((size_t)np * rp);
    op->cd_f64.alloc((size_t)np * rp);
    to_frag_f64(dPU.p, r, n, rp, np, op->pu_f64.p, s);
    to_frag_f64(dPV.p, r, n, rp, np, op->pv_f64.p, s);
    to_frag_f64(dVrSi.p, n, r, np, rp, op->cu_f64.p, s);
    to_frag_f64(dUrSi.p, n, r, np, rp, op->cd_f64.p, s);

    auto build = [&](const std::vector<double> &prm, const DBuf<double> &left, const DBuf<double> &right,
                     DBuf<double> *f64, DBuf<float> *rm) {
        build_translations(op->dY.p, n, r, rp, prm, left.p, right.p, f64, rm, s);
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
    pm2l = m2l_params(kRadIn, kRadIn);
    build(pm2m, dPU, dVrSi, &op->m2m_f64, nullptr);
    build(pl2l, dPV, dUrSi, &op->l2l_f64, nullptr);
    {
        DBuf<float> rm;  // row-major float32 translations, rearranged for the M2L kernel below
        build(pm2l, dPV, dVrSi, nullptr, &rm);
        op->m2l_f32.alloc(rr * kNumDirs);
        m2l_image_mats(rm.p, rp, kNumDirs, op->m2l_f32.p, s);
        op->m2l_bf.alloc(m2l_split_mats_elems(rp, kNumDirs, 3));
        m2l_split_mats(rm.p, rp, kNumDirs, 3, op->m2l_bf.p, s);
        op->m2l_bf2.alloc(m2l_split_mats_elems(rp, kNumDirs, 2));
        m2l_split_mats(rm.p, rp, kNumDirs, 2, op->m2l_bf2.p, s);
        FMM_HIP(hipStreamSynchronize(s));
    }
    return op;
}

// Lagrange polynomial of node i of the order-n Chebyshev nodes x, written in
// the Chebyshev basis: 1/n + (2/n) sum_{k=1}^{n-1} T_k(x_i) T_k(t).
double cheb_lagrange(const std::vector<double> &x, int i, double t) {
    const int n = (int)x.size();
    double s = 1.0 / n, a0 = 1.0, a1 = x[i], b0 = 1.0, b1 = t;
    for (int k = 1; k < n; ++k) {
        s += 2.0 / n * a1 * b1;
        const double a2 = 2.0 * x[i] * a1 - a0, b2 = 2.0 * t * b1 - b0;
        a0 = a1;
        a1 = a2;
        b0 = b1;
        b1 = b2;
    }
    return s;
}

// The paper's interpolation form (Sec. III.A.1 Eq. p2m) on Chebyshev nodes.
std::shared_ptr<Operators> build_chebyshev(int n, double eps, hipStream_t s) {
    auto op = std::make_shared<Operators>();
    op->basis = kBasisChebyshev;
    op->p = n;
    op->eps = eps;
    const std::vector<double> x = chebyshev_nodes(n);
    const int nn = op->ns = n * n * n;
    const int np = op->n_pad = ((nn + 31) / 32) * 32;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) op->Y.insert(op->Y.end(), {x[i], x[j], x[k]});
    op->dY = upload(op->Y, s);
    {
        std::vector<double> coef((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k)
                coef[(size_t)i * n + k] = k == 0 ? 1.0 / n : 2.0 / n * std::cos(k * (2 * i + 1) * kPi / (2 * n));
        op->cheb_coef = upload(coef, s);
    }

    // M2M / L2L: the map from child o's node weights to the parent's is
    // S[o_x] (x) S[o_y] (x) S[o_z] with S[side][i][i'] = S(x_i, -+1/2 + x_i' / 2)
    // (exact: the parent's polynomials have degree n - 1 per axis); L2L uses
    // the transposes.
    {
        std::vector<double> s1(2 * (size_t)n * n);
        for (int side = 0; side < 2; ++side)
            for (int i = 0; i < n; ++i)
                for (int i2 = 0; i2 < n; ++i2)
                    s1[((size_t)side * n + i) * n + i2] = cheb_lagrange(x, i, (side ? 0.5 : -0.5) + 0.5 * x[i2]);
        op->cheb_s1 = upload(s1, s);
    }

    // M2L: K_d = G(x, 2 d + x) between unit boxes. One basis Q for every
    // direction: the leading eigenvectors of sum_d K_d K_d^T (the left
    // singular vectors of [K_1 ... K_316]). The direction set is symmetric and
    // K_-d = K_d^T, so the same Q spans the right singular vectors of the
    // stacked [K_1; ...; K_316], and K_d ~ Q (Q^T K_d Q) Q^T.
    const std::vector<double> prm = m2l_params(1.0, 1.0), prmT = [&] {
        std::vector<double> t = prm;  // sources at the origin, targets at 2 d: G^T
        for (size_t b = 0; b < t.size(); b += 9)
            for (int c = 0; c < 3; ++c) std::swap(t[b + c], t[b + 4 + c]);
        return t;
    }();
    std::vector<double> Qf((size_t)nn * nn), lam(nn), Vf;
    if (!load_factors(kBasisChebyshev, n, {&Qf, &lam})) {
    std::vector<double> gram((size_t)nn * nn, 0.0);
    {
        const int chunk = 16, nb = (int)prm.size() / 9;
        const size_t n2 = (size_t)nn * nn;
        DBuf<double> G(chunk * n2), GT(chunk * n2), C(chunk * n2);
        std::vector<double> h(chunk * n2);
        for (int b0 = 0; b0 < nb; b0 += chunk) {
            const int cnt = std::min(chunk, nb - b0);
            std::vector<double> sub(prm.begin() + 9 * b0, prm.begin() + 9 * (b0 + cnt));
            std::vector<double> subT(prmT.begin() + 9 * b0, prmT.begin() + 9 * (b0 + cnt));
            DBuf<double> dp = upload(sub, s), dpT = upload(subT, s);
            build_laplace_mats(op->dY.p, nn, cnt, dp.p, G.p, s);
            build_laplace_mats(op->dY.p, nn, cnt, dpT.p, GT.p, s);
            dgemm_batched(G.p, n2, GT.p, n2, C.p, n2, nn, nn, nn, cnt, s);
            d2h(h.data(), C.p, cnt * n2, s);
            for (int b = 0; b < cnt; ++b)
                for (size_t e = 0; e < n2; ++e) gram[e] += h[b * n2 + e];
        }
    }
    svd_jacobi(gram, nn, Qf, lam, Vf);
    save_factors(kBasisChebyshev, n, {&Qf, &lam});
    }
    // sigma_k = sqrt(lambda_k); float64 resolves lambda to ~1e-16 lambda_max
    const double thr = std::max(eps * eps, 1e-15) * lam[0];
    int r = 0;
    while (r < nn && lam[r] > thr) ++r;
    r = std::max(r, 1);
    const int rp = ((r + 31) / 32) * 32;
    // M2L runs on r_pad values whatever r is, so the basis keeps r_pad
    // vectors when there are that many: the padded rows then carry the next
    // singular directions instead of zeros, at no cost in M2L. (No inverse is
    // taken here, unlike the surface form's pseudo-inverse, so more vectors
    // only bring the compressed operator closer to the dense one.)
    r = std::min(rp, nn);
    op->r = r;
    op->r_pad = rp;
    std::vector<double> Q((size_t)nn * r), QT((size_t)r * nn);
    for (int m = 0; m < nn; ++m)
        for (int k = 0; k < r; ++k) Q[(size_t)m * r + k] = QT[(size_t)k * nn + m] = Qf[(size_t)m * nn + k];
    op->U = Q;
    op->V = Q;
    DBuf<double> dQ = upload(Q, s), dQT = upload(QT, s);
    op->pv_f64.alloc((size_t)rp * np);  // node weights -> M2L basis
    op->cd_f64.alloc((size_t)np * rp);  // M2L basis -> node values
    to_frag_f64(dQT.p, r, nn, rp, np, op->pv_f64.p, s);
    to_frag_f64(dQ.p, nn, r, np, rp, op->cd_f64.p, s);
    op->pv_f32.alloc((size_t)rp * np);
    op->cd_f32.alloc((size_t)np * rp);
    to_frag_f32(dQT.p, r, nn, rp, np, op->pv_f32.p, s);
    to_frag_f32(dQ.p, nn, r, np, rp, op->cd_f32.p, s);
    {
        DBuf<float> rm;
        build_translations(op->dY.p, nn, r, rp, prm, dQT.p, dQ.p, nullptr, &rm, s);
        op->m2l_f32.alloc((size_t)rp * rp * kNumDirs);
        m2l_image_mats(rm.p, rp, kNumDirs, op->m2l_f32.p, s);
        op->m2l_bf.alloc(m2l_split_mats_elems(rp, kNumDirs, 3));
        m2l_split_mats(rm.p, rp, kNumDirs, 3, op->m2l_bf.p, s);
        op->m2l_bf2.alloc(m2l_split_mats_elems(rp, kNumDirs, 2));
        m2l_split_mats(rm.p, rp, kNumDirs, 2, op->m2l_bf2.p, s);
        FMM_HIP(hipStreamSynchronize(s));
    }
    return op;
}

}  // namespace

std::vector<double> chebyshev_nodes(int n) {
    std::vector<double> x(n);
    for (int i = 0; i < n; ++i) x[i] = std::cos((2 * i + 1) * kPi / (2 * n));
    return x;
}

std::shared_ptr<const Operators> get_operators(int basis, int p, double eps, hipStream_t s) {
    // Held until the process ends (never destroyed, so no device memory is
    // freed after the HIP runtime has shut down).
    static std::mutex mu;
    static auto *cache = new std::map<std::tuple<int, int, int, double>, std::shared_ptr<Operators>>();
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, basis, p, eps);
    auto it = cache->find(key);
    if (it != cache->end()) return it->second;
    auto op = basis == kBasisChebyshev ? build_chebyshev(p, eps, s) : build_operators(p, eps, s);
    (*cache)[key] = op;
    return op;
}

}  // namespace fmm
