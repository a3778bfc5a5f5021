// C ABI of the library (declared in include/fmm.h).
#include <chrono>
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "plan.hpp"
#include "probe.hpp"

// A handle is a small shell around the plan. fmm_destroy frees the plan and
// keeps the shell as a tombstone for the rest of the process, so a handle
// once issued is never reused for another plan and every later call on it can
// be answered with FMM_ERR_STATE without touching freed memory.
struct fmm_plan_s {
    std::unique_ptr<fmm::Plan> p;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

template <class F>
int guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return FMM_OK;
    } catch (const fmm::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(FMM_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(FMM_ERR_DEVICE, e.what());
    }
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Every handle the library has issued, live or destroyed (true = live).
std::mutex g_handles_mu;
std::unordered_map<const fmm_plan_s *, bool> g_handles;

void register_handle(fmm_plan_s *h) {
    std::lock_guard<std::mutex> lk(g_handles_mu);
    g_handles[h] = true;
}

// Look a handle up: NULL and pointers the library never issued are argument
// errors, destroyed handles are state errors.
fmm::Plan &live(fmm_plan plan) {
    if (!plan) throw fmm::Error(FMM_ERR_ARG, "plan is NULL");
    std::lock_guard<std::mutex> lk(g_handles_mu);
    auto it = g_handles.find(plan);
    if (it == g_handles.end()) throw fmm::Error(FMM_ERR_ARG, "not a plan handle issued by fmm_setup");
    if (!it->second) throw fmm::Error(FMM_ERR_STATE, "plan was destroyed");
    return *plan->p;
}

}  // namespace

extern "C" {

void fmm_default_options(fmm_options *opt) {
    if (!opt) return;
    *opt = fmm_options{};
    opt->order = 6;
    opt->leaf_size = 64;
    opt->uniform_depth = 0;
    opt->max_depth = 21;
    opt->precision = FMM_PREC_FP32;
    opt->src_kernels = FMM_SRC_SINGLE;
    opt->outputs = FMM_OUT_POT;
    opt->nrhs = 1;
    opt->cutoff = 1e-5f;
    opt->root[0] = opt->root[1] = opt->root[2] = opt->root[3] = 0.0;
    opt->pinv_eps = 0.0;
    opt->m2l_pieces = 0;
    opt->basis = FMM_BASIS_SURFACE;
}

const char *fmm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

void check_options(const fmm_options *opt) {
    using namespace fmm;
    FMM_REQUIRE(opt != nullptr, "fmm_setup: options are NULL");
    FMM_REQUIRE(opt->basis == FMM_BASIS_SURFACE || opt->basis == FMM_BASIS_CHEBYSHEV, "fmm_setup: unknown basis");
    if (opt->basis == FMM_BASIS_CHEBYSHEV)
        FMM_REQUIRE(opt->order >= 2 && opt->order <= 8, "fmm_setup: Chebyshev order must be in 2..8");
    else
        FMM_REQUIRE(opt->order >= 2 && opt->order <= 10, "fmm_setup: order must be in 2..10");
    FMM_REQUIRE(opt->leaf_size >= 0, "fmm_setup: leaf_size must be >= 0 (0: from the tuning cache)");
    FMM_REQUIRE(opt->max_depth >= 1 && opt->max_depth <= kMaxLevel, "fmm_setup: max_depth must be in 1..21");
    FMM_REQUIRE(opt->uniform_depth >= 0 && opt->uniform_depth <= kMaxLevel,
                "fmm_setup: uniform_depth must be in 0..21");
    FMM_REQUIRE(opt->nrhs >= 1 && opt->nrhs <= 4, "fmm_setup: nrhs must be in 1..4");
    FMM_REQUIRE(opt->precision == FMM_PREC_FP32 || opt->precision == FMM_PREC_SPLIT_BF16 ||
                    opt->precision == FMM_PREC_SPLIT_BF16X3 || opt->precision == FMM_PREC_SPLIT_BF16X4,
                "fmm_setup: unknown precision");
    FMM_REQUIRE((opt->src_kernels & ~3) == 0 && opt->src_kernels != 0,
                "fmm_setup: src_kernels must be a nonzero FMM_SRC_* mask");
    FMM_REQUIRE((opt->outputs & ~3) == 0 && opt->outputs != 0, "fmm_setup: outputs must be a nonzero FMM_OUT_* mask");
    FMM_REQUIRE(!((opt->outputs & FMM_OUT_FIELD) && (opt->src_kernels & FMM_SRC_DOUBLE)),
                "fmm_setup: the field output is defined for the single layer only");
    FMM_REQUIRE(std::isfinite(opt->cutoff) && opt->cutoff >= 0.f, "fmm_setup: cutoff must be finite and >= 0");
    FMM_REQUIRE(opt->root[3] <= 0.0 || (std::isfinite(opt->root[0]) && std::isfinite(opt->root[1]) &&
                                        std::isfinite(opt->root[2]) && std::isfinite(opt->root[3])),
                "fmm_setup: root cube is not finite");
    FMM_REQUIRE(opt->pinv_eps >= 0.0 && std::isfinite(opt->pinv_eps), "fmm_setup: pinv_eps must be finite and >= 0");
    FMM_REQUIRE(opt->m2l_pieces >= 0 && opt->m2l_pieces <= 8, "fmm_setup: m2l_pieces must be in 0..8");
}

// leaf_size = 0: the tuned cap for this configuration from the cache, else
// the default; the resolved options are returned (m2l_pieces from the cache
// only when the caller left it at 0)
fmm_options resolve_auto_leaf(const fmm_options *opt, int64_t points_per_instance, bool tsm, bool batch,
                              int &from_cache) {
    fmm_options o = *opt;
    from_cache = 0;
    if (o.leaf_size != 0) return o;
    int leaf = 0, pieces = 0;
    if (fmm::tune_cache_lookup(fmm::tune_cache_path(), fmm::tune_key(o, points_per_instance, tsm, batch), leaf,
                               pieces)) {
        o.leaf_size = leaf;
        if (o.m2l_pieces == 0) o.m2l_pieces = pieces;
        from_cache = 1;
    } else {
        o.leaf_size = fmm::kDefaultAutoLeaf;
    }
    return o;
}

fmm::TreeOptions tree_options(const fmm_options *opt) {
    fmm::TreeOptions to;
    to.leaf_size = opt->leaf_size;
    to.uniform_depth = opt->uniform_depth;
    to.max_depth = opt->max_depth;
    for (int c = 0; c < 4; ++c) to.root[c] = opt->root[c];
    return to;
}

void init_plan(fmm::Plan &P, const fmm_options *opt) {
    P.opt = *opt;
    P.nrhs = opt->nrhs;
    P.sl = opt->src_kernels & FMM_SRC_SINGLE;
    P.dl = opt->src_kernels & FMM_SRC_DOUBLE;
    P.want_pot = opt->outputs & FMM_OUT_POT;
    P.want_field = opt->outputs & FMM_OUT_FIELD;
    P.m2l_form = opt->precision == FMM_PREC_SPLIT_BF16     ? 6
                 : opt->precision == FMM_PREC_SPLIT_BF16X4 ? 4
                 : opt->precision == FMM_PREC_SPLIT_BF16X3 ? 3
                                                           : 0;
}

// Everything after the tree: operators, per-box buffers, work lists.
void finish_plan(fmm::Plan &P, const fmm_options *opt, const float *trg_nrm, hipStream_t s) {
    using namespace fmm;
    auto clock0 = std::chrono::steady_clock::now();
    auto phase_end = [&](int k) {
        FMM_HIP(hipStreamSynchronize(s));
        const auto now = std::chrono::steady_clock::now();
        P.setup_phase_ms[k] += std::chrono::duration<double, std::milli>(now - clock0).count();
        clock0 = now;
    };
    for (int k = 0; k < 3; ++k) P.setup_phase_ms[k] += P.t.phase_ms[k];
    double eps = opt->pinv_eps > 0 ? opt->pinv_eps : default_pinv_eps(opt->basis, opt->order);
    P.ops = get_operators(opt->basis, opt->order, eps, s);
    phase_end(3);
    P.cheb = opt->basis == FMM_BASIS_CHEBYSHEV;
    P.ns = P.ops->ns;
    P.n_pad = P.ops->n_pad;
    P.r = P.ops->r;
    P.r_pad = P.ops->r_pad;
    const size_t nvec = (size_t)P.t.nb * P.nrhs;
    P.ut.alloc(nvec * P.r_pad);
    P.dt.alloc(nvec * P.r_pad);
    P.chk.alloc(nvec * P.n_pad);
    if (P.m2l_form) P.ut_bf.alloc(m2l_split_vecs_elems(P.r_pad, (int64_t)nvec, m2l_form_parts(P.m2l_form)));
    P.phi_u.alloc(nvec * P.n_pad);
    P.phi_d.alloc(nvec * P.n_pad);
    if (P.cheb) {
        // expansion of the M2L result: 1 / half-width per vector
        std::vector<double> sc(nvec);
        for (size_t v = 0; v < nvec; ++v) sc[v] = 1.0 / P.t.h_half[v / P.nrhs];
        P.col_iscale = upload(sc, s);
    }
    // zero once: padding entries are never written, vectors of boxes
    // a stage skips stay zero
    for (DBuf<float> *b : {&P.ut, &P.chk, &P.phi_u, &P.phi_d})
        if (b->n) FMM_HIP(hipMemsetAsync(b->p, 0, b->bytes(), s));
    const size_t nsv = (size_t)P.nrhs * P.t.n_src;
    if (P.sl) P.q_sorted.alloc(nsv);
    if (P.dl) {
        P.mx.alloc(nsv);
        P.my.alloc(nsv);
        P.mz.alloc(nsv);
    }
    if (P.sl && P.dl) P.qm.alloc(2 * nsv);
    if (trg_nrm && !P.t.tsm && P.t.n_src) {
        P.trg_nrm_user.alloc(3 * (size_t)P.t.n_src);
        FMM_HIP(hipMemcpyAsync(P.trg_nrm_user.p, trg_nrm, 3 * P.t.n_src * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    phase_end(4);
    if (P.t.nb) plan_build_worklists(P, s);
    if (P.t.nb) plan_create_side(P);
    FMM_HIP(hipStreamSynchronize(s));
}

}  // namespace

extern "C" {

int fmm_setup(const float *src_xyz, const float *src_nrm, int64_t n_src, const float *trg_xyz, const float *trg_nrm,
              int64_t n_trg, const fmm_options *opt, void *hip_stream, fmm_plan *out) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(out != nullptr, "fmm_setup: out is NULL");
        *out = nullptr;
        check_options(opt);
        FMM_REQUIRE(n_src >= 0 && n_trg >= 0, "fmm_setup: negative point count");
        FMM_REQUIRE(n_src == 0 || src_xyz != nullptr, "fmm_setup: src_xyz is NULL");
        FMM_REQUIRE(!(opt->src_kernels & FMM_SRC_DOUBLE) || n_src == 0 || src_nrm != nullptr,
                    "fmm_setup: the double layer needs source normals");
        FMM_REQUIRE(n_src + n_trg < (int64_t(1) << 31), "fmm_setup: more than 2^31 - 1 points");

        auto t0 = std::chrono::steady_clock::now();
        hipStream_t s = as_stream(hip_stream);
        int from_cache = 0;
        const fmm_options ro = resolve_auto_leaf(opt, n_src + (trg_xyz ? n_trg : 0), trg_xyz != nullptr, false,
                                                 from_cache);
        opt = &ro;
        auto *h = new fmm_plan_s();
        h->p.reset(new Plan());
        try {
            Plan &P = *h->p;
            init_plan(P, opt);
            P.leaf_from_cache = from_cache;
            build_tree(P.t, src_xyz, src_nrm, n_src, trg_xyz, trg_nrm, n_trg, tree_options(opt), s);
            finish_plan(P, opt, trg_nrm, s);
            P.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        } catch (...) {
            delete h;
            throw;
        }
        register_handle(h);
        *out = h;
    });
}

int fmm_setup_batch(int n_inst, const int64_t *src_off, const int64_t *trg_off, const float *src_xyz,
                    const float *src_nrm, const float *trg_xyz, const float *trg_nrm, const fmm_options *opt,
                    void *hip_stream, fmm_plan *out) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(out != nullptr, "fmm_setup_batch: out is NULL");
        *out = nullptr;
        check_options(opt);
        FMM_REQUIRE(n_inst >= 1, "fmm_setup_batch: n_inst must be >= 1");
        FMM_REQUIRE(src_off != nullptr, "fmm_setup_batch: src_off is NULL");
        FMM_REQUIRE((trg_xyz == nullptr) == (trg_off == nullptr),
                    "fmm_setup_batch: trg_xyz and trg_off go together");
        const bool tsm = trg_xyz != nullptr;
        std::vector<int64_t> so(src_off, src_off + n_inst + 1), to(n_inst + 1, 0);
        if (tsm) to.assign(trg_off, trg_off + n_inst + 1);
        FMM_REQUIRE(so[0] == 0 && to[0] == 0, "fmm_setup_batch: offsets must start at 0");
        for (int i = 0; i < n_inst; ++i) {
            FMM_REQUIRE(so[i + 1] >= so[i], "fmm_setup_batch: src_off must be nondecreasing");
            FMM_REQUIRE(to[i + 1] >= to[i], "fmm_setup_batch: trg_off must be nondecreasing");
        }
        const int64_t n_src = so[n_inst], n_trg = to[n_inst];
        FMM_REQUIRE(n_src == 0 || src_xyz != nullptr, "fmm_setup_batch: src_xyz is NULL");
        FMM_REQUIRE(!(opt->src_kernels & FMM_SRC_DOUBLE) || n_src == 0 || src_nrm != nullptr,
                    "fmm_setup_batch: the double layer needs source normals");
        FMM_REQUIRE(n_src + n_trg < (int64_t(1) << 31), "fmm_setup_batch: more than 2^31 - 1 points");

        auto t0 = std::chrono::steady_clock::now();
        hipStream_t s = as_stream(hip_stream);
        int from_cache = 0;
        const fmm_options ro = resolve_auto_leaf(opt, (n_src + (tsm ? n_trg : 0)) / n_inst, tsm, true, from_cache);
        opt = &ro;
        auto *h = new fmm_plan_s();
        h->p.reset(new Plan());
        try {
            Plan &P = *h->p;
            init_plan(P, opt);
            P.leaf_from_cache = from_cache;
            build_forest(P.t, so, to, src_xyz, src_nrm, tsm ? trg_xyz : nullptr, trg_nrm, tree_options(opt), s);
            P.n_inst = n_inst;
            finish_plan(P, opt, trg_nrm, s);
            P.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        } catch (...) {
            delete h;
            throw;
        }
        register_handle(h);
        *out = h;
    });
}

int fmm_apply(fmm_plan plan, const float *q, const float *mu, float *pot, float *field, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(q == nullptr || P.sl, "fmm_apply: q given but the plan has no single layer");
        FMM_REQUIRE(mu == nullptr || P.dl, "fmm_apply: mu given but the plan has no double layer");
        FMM_REQUIRE(pot == nullptr || P.want_pot, "fmm_apply: potential not among the plan's outputs");
        FMM_REQUIRE(field == nullptr || P.want_field, "fmm_apply: field not among the plan's outputs");
        FMM_REQUIRE(field == nullptr || mu == nullptr, "fmm_apply: the field output needs the single layer only");
        hipStream_t s = as_stream(hip_stream);
        const int64_t nt = P.t.n_trg;
        if (P.t.nb == 0 || P.t.n_src == 0 || (q == nullptr && mu == nullptr)) {
            if (pot && nt) FMM_HIP(hipMemsetAsync(pot, 0, sizeof(float) * P.nrhs * nt, s));
            if (field && nt) FMM_HIP(hipMemsetAsync(field, 0, sizeof(float) * 3 * P.nrhs * nt, s));
            return;
        }
        if (P.graph.enabled && !P.timing)  // stage timing needs the ordinary apply
            plan_apply_graph(P, q, mu, pot, field, s);
        else
            plan_apply(P, q, mu, pot, field, s);
    });
}

int fmm_dielectric_rhs(fmm_plan plan, const float *sigma_f, const float *areas, const float *curvature,
                       const float *eps_i, float eps_m, const double *e0, double *b, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(sigma_f && areas && curvature && eps_i && b, "fmm_dielectric_rhs: NULL argument");
        FMM_REQUIRE(std::isfinite(eps_m) && eps_m > 0.f, "fmm_dielectric_rhs: eps_m must be > 0");
        dielectric_rhs(P, sigma_f, areas, curvature, eps_i, eps_m, e0, b, as_stream(hip_stream));
    });
}

int fmm_dielectric_rhs_noalloc(fmm_plan plan, const float *sigma_f, const float *areas, const float *curvature,
                               const float *eps_i, float eps_m, const double *e0, double *b, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(sigma_f && areas && curvature && eps_i && b, "fmm_dielectric_rhs_noalloc: NULL argument");
        FMM_REQUIRE(std::isfinite(eps_m) && eps_m > 0.f, "fmm_dielectric_rhs_noalloc: eps_m must be > 0");
        dielectric_rhs_noalloc(P, sigma_f, areas, curvature, eps_i, eps_m, e0, b, as_stream(hip_stream));
    });
}

int fmm_body_forces(fmm_plan plan, const float *sigma_f, const float *sigma_b, const float *areas,
                    const float *curvature, float eps_m, const double *e0, int n_body, const int64_t *body_off,
                    double *forces, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(sigma_f && areas && curvature && forces, "fmm_body_forces: NULL argument");
        FMM_REQUIRE(std::isfinite(eps_m) && eps_m > 0.f, "fmm_body_forces: eps_m must be > 0");
        body_forces(P, sigma_f, sigma_b, areas, curvature, eps_m, e0, n_body, body_off, forces,
                    as_stream(hip_stream));
    });
}

int fmm_set_graph(fmm_plan plan, int enable) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        P.graph.enabled = enable != 0;
        if (!P.graph.enabled) plan_release_graph(P);
    });
}

int gmres_solve(fmm_plan plan, const fmm_operator *op, const double *b, double *x, double rtol, int restart,
                int max_iter, int *iters, double *rel_res, void *hip_stream) {
    int status = FMM_OK;
    int rc = guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(op && b && x && iters && rel_res, "gmres_solve: NULL argument");
        FMM_REQUIRE(!P.t.tsm, "gmres_solve: the operator needs targets equal to sources");
        FMM_REQUIRE(P.nrhs == 1, "gmres_solve: the plan must have nrhs = 1");
        FMM_REQUIRE(P.t.n_src > 0, "gmres_solve: empty plan");
        FMM_REQUIRE(op->a && op->w, "gmres_solve: operator coefficients a and w are required");
        if (op->kind == FMM_OP_FK) {
            FMM_REQUIRE(P.dl && P.want_pot, "gmres_solve: FK needs a double-layer plan with potential output");
        } else if (op->kind == FMM_OP_DIELECTRIC) {
            FMM_REQUIRE(op->c, "gmres_solve: dielectric operator needs c");
            FMM_REQUIRE(P.sl && P.want_field, "gmres_solve: dielectric needs a single-layer plan with field output");
            FMM_REQUIRE(P.trg_nrm_user.n, "gmres_solve: dielectric needs target normals at setup");
        } else {
            throw Error(FMM_ERR_ARG, "gmres_solve: unknown operator kind");
        }
        FMM_REQUIRE(rtol > 0.0 && std::isfinite(rtol), "gmres_solve: rtol must be > 0");
        FMM_REQUIRE(restart >= 1 && restart <= 500, "gmres_solve: restart must be in 1..500");
        FMM_REQUIRE(max_iter >= 0, "gmres_solve: max_iter must be >= 0");
        plan_gmres(P, *op, b, x, rtol, restart, max_iter, iters, rel_res, &status, as_stream(hip_stream));
    });
    if (rc != FMM_OK) return rc;
    if (status == FMM_ERR_NOT_CONVERGED)
        g_last_error = "gmres_solve: not converged (relative residual " + std::to_string(*rel_res) + " after " +
                       std::to_string(*iters) + " iterations)";
    return status;
}

int fmm_destroy(fmm_plan plan) {
    if (!plan) return FMM_OK;
    return guarded([&] {
        std::unique_ptr<fmm::Plan> dead;
        {
            std::lock_guard<std::mutex> lk(g_handles_mu);
            auto it = g_handles.find(plan);
            if (it == g_handles.end()) throw fmm::Error(FMM_ERR_ARG, "not a plan handle issued by fmm_setup");
            if (!it->second) throw fmm::Error(FMM_ERR_STATE, "plan was already destroyed");
            it->second = false;  // the shell stays allocated as a tombstone
            dead = std::move(plan->p);
        }
        fmm::plan_release_graph(*dead);
        fmm::plan_release_events(*dead);
    });
}

int fmm_direct(const float *src_xyz, const float *src_nrm, int64_t n_src, const float *trg_xyz, int64_t n_trg,
               const float *q, const float *mu, float cutoff, float *pot, float *field, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(n_src >= 0 && n_trg >= 0, "fmm_direct: negative count");
        FMM_REQUIRE(n_src == 0 || src_xyz != nullptr, "fmm_direct: src_xyz is NULL");
        FMM_REQUIRE(n_trg == 0 || trg_xyz != nullptr, "fmm_direct: trg_xyz is NULL");
        FMM_REQUIRE(mu == nullptr || src_nrm != nullptr, "fmm_direct: mu needs normals");
        FMM_REQUIRE(field == nullptr || mu == nullptr, "fmm_direct: field is defined for the single layer only");
        FMM_REQUIRE(std::isfinite(cutoff) && cutoff >= 0.f, "fmm_direct: bad cutoff");
        direct_all_pairs(trg_xyz, n_trg, src_xyz, src_nrm, n_src, q, mu, cutoff, pot, field, as_stream(hip_stream));
    });
}

int fmm_plan_info(fmm_plan plan, fmm_info *info) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(info != nullptr, "fmm_plan_info: info is NULL");
        fmm_info r{};
        r.n_src = P.t.n_src;
        r.n_trg = P.t.n_trg;
        r.n_points = P.t.n;
        r.n_boxes = P.t.nb;
        int64_t nl = 0;
        for (auto v : P.t.h_leaf) nl += v;
        r.n_leaves = nl;
        r.n_levels = P.t.nlev;
        r.n_u = P.t.U.total;
        r.n_v = P.t.V.total;
        r.n_w = P.t.W.total;
        r.n_x = P.t.X.total;
        r.n_surface = P.ns;
        r.p2p_pairs = P.p2p_pairs;
        r.m2l_pairs = P.m2l_pairs;
        r.surf_evals = P.surf_evals;
        r.p2m_evals = P.p2m_evals;
        r.m2l_columns = P.m2l_steps * P.m2l_ncol;
        r.rank = P.r;
        r.m2l_pieces = P.m2l_pieces_per_tile;
        r.m2l_pair_tiles = P.m2l_pair_tiles;
        r.basis = P.cheb ? FMM_BASIS_CHEBYSHEV : FMM_BASIS_SURFACE;
        for (int c = 0; c < 3; ++c) r.root[c] = P.t.x0[c];
        r.root[3] = P.t.w;
        r.setup_ms = P.setup_ms;
        for (int k = 0; k < 8; ++k) r.setup_phase_ms[k] = P.setup_phase_ms[k];
        r.leaf_size = P.opt.leaf_size;
        r.leaf_from_cache = P.leaf_from_cache;
        r.p2l_evals = P.p2l_evals;
        *info = r;
    });
}

int fmm_export_tree(fmm_plan plan, const fmm_tree_export *o) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(o != nullptr, "fmm_export_tree: out is NULL");
        Tree &t = P.t;
        auto cp = [](auto *dst, const auto &src) {
            if (dst) std::copy(src.begin(), src.end(), dst);
        };
        cp(o->level, t.h_level);
        cp(o->anchor, t.h_anchor);
        cp(o->parent, t.h_parent);
        cp(o->begin, t.h_begin);
        cp(o->end, t.h_end);
        cp(o->tbeg, t.h_tbeg);
        cp(o->tend, t.h_tend);
        cp(o->sbeg, t.h_sbeg);
        cp(o->send, t.h_send);
        cp(o->u_off, t.U.h_off);
        cp(o->u_idx, t.U.h_idx);
        cp(o->v_off, t.V.h_off);
        cp(o->v_idx, t.V.h_idx);
        cp(o->w_off, t.W.h_off);
        cp(o->w_idx, t.W.h_idx);
        cp(o->x_off, t.X.h_off);
        cp(o->x_idx, t.X.h_idx);
        hipStream_t s = nullptr;
        if (o->src_perm && t.n_src) d2h(o->src_perm, t.src_perm.p, t.n_src, s);
        if (o->trg_perm && t.n_trg) d2h(o->trg_perm, t.tsm ? t.trg_perm.p : t.src_perm.p, t.n_trg, s);
        if (o->keys && t.n) d2h(o->keys, t.keys.p, t.n, s);
    });
}

int fmm_export_stage(fmm_plan plan, int which, float *host_out) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(host_out != nullptr, "fmm_export_stage: out is NULL");
        FMM_REQUIRE(which == 0 || which == 1, "fmm_export_stage: which must be 0 or 1");
        if (P.cheb) {
            // node weights W (upward) or node values L (downward), stored as they are
            const DBuf<float> &b = which == 0 ? P.phi_u : P.phi_d;
            std::vector<float> all(b.n);
            FMM_HIP(hipDeviceSynchronize());
            d2h(all.data(), b.p, b.n, nullptr);
            for (int64_t box = 0; box < P.t.nb; ++box)
                for (int m = 0; m < P.ns; ++m) host_out[box * P.ns + m] = all[((size_t)box * P.nrhs) * P.n_pad + m];
            return;
        }
        // reconstruct U_r ut (upward) or V_r dt (downward), [ns][r] host factors
        const DBuf<float> &b = which == 0 ? P.ut : P.dt;
        const std::vector<double> &B = which == 0 ? P.ops->U : P.ops->V;
        std::vector<float> all(b.n);
        FMM_HIP(hipDeviceSynchronize());
        d2h(all.data(), b.p, b.n, nullptr);
        for (int64_t box = 0; box < P.t.nb; ++box) {
            const float *x = &all[((size_t)box * P.nrhs) * P.r_pad];
            for (int m = 0; m < P.ns; ++m) {
                double v = 0.0;
                for (int k = 0; k < P.r; ++k) v += B[(size_t)m * P.r + k] * (double)x[k];
                host_out[box * P.ns + m] = (float)v;
            }
        }
    });
}

int fmm_autotune(int n_inst, const int64_t *src_off, const int64_t *trg_off, const float *src_xyz,
                 const float *src_nrm, int64_t n_src, const float *trg_xyz, const float *trg_nrm, int64_t n_trg,
                 const fmm_options *opt, const fmm_tune_space *space, const char *cache_path, fmm_tune_result *out,
                 void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(opt && space && out, "fmm_autotune: NULL argument");
        FMM_REQUIRE(n_inst >= 0, "fmm_autotune: n_inst must be >= 0");
        FMM_REQUIRE(n_inst == 0 || src_off != nullptr, "fmm_autotune: a batch needs src_off");
        FMM_REQUIRE(space->n_leaf >= 1 && space->n_leaf <= 8, "fmm_autotune: n_leaf must be in 1..8");
        FMM_REQUIRE(space->n_pieces >= 0 && space->n_pieces <= 4, "fmm_autotune: n_pieces must be in 0..4");
        FMM_REQUIRE(space->reps >= 1 && space->reps <= 100, "fmm_autotune: reps must be in 1..100");
        for (int i = 0; i < space->n_leaf; ++i)
            FMM_REQUIRE(space->leaf_sizes[i] >= 1, "fmm_autotune: leaf sizes must be >= 1");
        for (int i = 0; i < space->n_pieces; ++i)
            FMM_REQUIRE(space->pieces[i] >= 0 && space->pieces[i] <= 8, "fmm_autotune: pieces must be in 0..8");
        check_options(opt);
        const bool batch = n_inst > 0;
        const bool tsm = batch ? trg_off != nullptr : trg_xyz != nullptr;
        const int64_t ns_all = batch ? src_off[n_inst] : n_src;
        const int64_t nt_all = batch ? (tsm ? trg_off[n_inst] : ns_all) : (tsm ? n_trg : n_src);
        FMM_REQUIRE(ns_all >= 1, "fmm_autotune: no sources");
        const int64_t ppi = batch ? (ns_all + (tsm ? nt_all : 0)) / n_inst : ns_all + (tsm ? nt_all : 0);
        hipStream_t s = as_stream(hip_stream);
        const int nrhs = opt->nrhs;
        DBuf<float> q, mu, pot, fld;
        if (opt->src_kernels & FMM_SRC_SINGLE) {
            q.alloc((size_t)nrhs * ns_all);
            fill_random(q.p, (int64_t)q.n, 1u, s);
        }
        if (opt->src_kernels & FMM_SRC_DOUBLE) {
            mu.alloc((size_t)nrhs * ns_all);
            fill_random(mu.p, (int64_t)mu.n, 2u, s);
        }
        if (opt->outputs & FMM_OUT_POT) pot.alloc((size_t)nrhs * nt_all);
        else fld.alloc((size_t)3 * nrhs * nt_all);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        FMM_HIP(hipEventCreate(&e0));
        FMM_HIP(hipEventCreate(&e1));
        fmm_tune_result res{};
        double best = 1e300;
        try {
            const int np = space->n_pieces > 0 ? space->n_pieces : 1;
            for (int il = 0; il < space->n_leaf; ++il) {
                for (int ip = 0; ip < np; ++ip) {
                    fmm_options o = *opt;
                    o.leaf_size = space->leaf_sizes[il];
                    o.m2l_pieces = space->n_pieces > 0 ? space->pieces[ip] : opt->m2l_pieces;
                    fmm_plan plan = nullptr;
                    int rc = batch ? fmm_setup_batch(n_inst, src_off, trg_off, src_xyz, src_nrm, trg_xyz, trg_nrm, &o,
                                                     hip_stream, &plan)
                                   : fmm_setup(src_xyz, src_nrm, n_src, trg_xyz, trg_nrm, n_trg, &o, hip_stream,
                                               &plan);
                    if (rc != FMM_OK) throw Error(rc, std::string("fmm_autotune: ") + fmm_last_error());
                    fmm_info info{};
                    fmm_plan_info(plan, &info);
                    std::vector<float> times;
                    for (int k = 0; k <= space->reps && rc == FMM_OK; ++k) {  // one warm-up apply first
                        FMM_HIP(hipEventRecord(e0, s));
                        rc = fmm_apply(plan, q.p, mu.p, pot.p, fld.p, hip_stream);
                        FMM_HIP(hipEventRecord(e1, s));
                        FMM_HIP(hipEventSynchronize(e1));
                        float ms = 0.f;
                        FMM_HIP(hipEventElapsedTime(&ms, e0, e1));
                        if (k > 0) times.push_back(ms);
                    }
                    const std::string msg = rc == FMM_OK ? "" : fmm_last_error();
                    fmm_destroy(plan);
                    if (rc != FMM_OK) throw Error(rc, "fmm_autotune: " + msg);
                    std::sort(times.begin(), times.end());
                    const double med = times[times.size() / 2];
                    if (res.n_tried < 32) {
                        res.tried_leaf[res.n_tried] = o.leaf_size;
                        res.tried_pieces[res.n_tried] = (int)info.m2l_pieces;
                        res.tried_ms[res.n_tried] = med;
                        res.tried_setup_ms[res.n_tried] = info.setup_ms;
                        ++res.n_tried;
                    }
                    if (med < best) {
                        best = med;
                        res.leaf_size = o.leaf_size;
                        res.m2l_pieces = (int)info.m2l_pieces;
                        res.ms = med;
                    }
                }
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (cache_path) {
            const std::string path = cache_path[0] ? std::string(cache_path) : tune_cache_path();
            tune_cache_store(path, tune_key(*opt, ppi, tsm, batch), res.leaf_size, res.m2l_pieces, res.ms);
        }
        *out = res;
    });
}

int fmm_split_bf16(int which, int r_pad, int64_t count, const float *in, uint16_t *parts, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(which == 0 || which == 1, "fmm_split_bf16: which must be 0 or 1");
        FMM_REQUIRE(m2l_supported(r_pad), "fmm_split_bf16: r_pad must be a multiple of 32 in 32..512");
        FMM_REQUIRE(count >= 0 && count <= (int64_t(1) << 24), "fmm_split_bf16: count out of range");
        FMM_REQUIRE(count == 0 || (in && parts), "fmm_split_bf16: NULL argument");
        m2l_split_plain(which, r_pad, count, in, parts, as_stream(hip_stream));
    });
}

int fmm_pinv(const double *K, int n, double eps, double *out) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(K && out && n > 0 && n <= 4096, "fmm_pinv: bad arguments");
        FMM_REQUIRE(eps >= 0.0 && std::isfinite(eps), "fmm_pinv: bad eps");
        std::vector<double> k(K, K + (size_t)n * n);
        std::vector<double> p = pinv_jacobi(k, n, eps);
        std::copy(p.begin(), p.end(), out);
    });
}

int fmm_unit_surface(int p, double *out, int *ns) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(p >= 2 && p <= 10 && ns, "fmm_unit_surface: bad arguments");
        std::vector<double> y = unit_surface(p);
        *ns = (int)(y.size() / 3);
        if (out) std::copy(y.begin(), y.end(), out);
    });
}

int fmm_set_timing(fmm_plan plan, int enable) {
    return guarded([&] { live(plan).timing = enable != 0; });
}

int fmm_stage_times(fmm_plan plan, double *ms) {
    return guarded([&] {
        using namespace fmm;
        Plan &P = live(plan);
        FMM_REQUIRE(ms != nullptr, "fmm_stage_times: out is NULL");
        plan_report_times(P);
        for (int k = 0; k < ST_COUNT; ++k) ms[k] = P.have_times ? P.stage_ms[k] : -1.0;
    });
}

int fmm_issue_probe(int kind, int64_t nthreads, int iters, float *out, int64_t *instr_per_lane, void *hip_stream) {
    return guarded([&] {
        using namespace fmm;
        FMM_REQUIRE(kind >= 0 && kind <= 4, "fmm_issue_probe: kind must be 0..4");
        FMM_REQUIRE(nthreads > 0 && nthreads % 256 == 0 && nthreads <= (int64_t(1) << 24),
                    "fmm_issue_probe: nthreads must be a positive multiple of 256, at most 2^24");
        FMM_REQUIRE(iters >= 1 && iters <= (1 << 20), "fmm_issue_probe: iters must be in 1..2^20");
        FMM_REQUIRE(out != nullptr, "fmm_issue_probe: out is NULL");
        issue_probe(kind, nthreads, iters, out, as_stream(hip_stream));
        if (instr_per_lane) *instr_per_lane = (int64_t)iters * issue_probe_instr(kind);
    });
}

}  // extern "C"
