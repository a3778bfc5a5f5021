// Plan object shared by the API translation units.
#pragma once

#include <array>
#include <memory>

#include "gemm.hpp"
#include "m2l.hpp"
#include "nbody.hpp"
#include "operators.hpp"
#include "tree.hpp"

namespace fmm {

// Chebyshev M2M / L2L at one level (cheb_tensor): dst boxes, their sources
// (8 children per parent, or the parent of a child) and the child's octant.
struct ChebJob {
    DBuf<int32_t> dst, src;
    DBuf<int8_t> oct;
    int n = 0;
};

struct GemmJob {
    DBuf<int32_t> cols, src, mat;
    int ntile = 0, nterm = 0;
    bool use_mat = false;
};

enum Stage { ST_P2M = 0, ST_M2M, ST_P2L, ST_M2L, ST_L2L, ST_C2E, ST_EVAL, ST_COUNT };

struct Plan {
    fmm_options opt{};
    int nrhs = 1;
    int n_inst = 1;  // independent instances (fmm_setup_batch)
    bool sl = true, dl = false, want_pot = true, want_field = false;
    Tree t;
    std::shared_ptr<const Operators> ops;
    int ns = 0, n_pad = 0, r = 0, r_pad = 0;
    int m2l_form = 0;  // M2L arithmetic: 0 float32; 6, 4, 3 split-BF16 products (m2l.hpp)
    bool cheb = false;  // Chebyshev basis: node weights W in phi_u, node values L in phi_d

    DBuf<float> ut, dt;                     // [nb * nrhs][r_pad] compressed upward / downward state
    DBuf<uint16_t> ut_bf;                   // ut split into bfloat16 parts (split-BF16 M2L forms)
    DBuf<float> chk;                        // [nb * nrhs][n_pad] check potentials made from points
    DBuf<float> phi_u, phi_d;               // [nb * nrhs][n_pad] equivalent densities
    DBuf<float> q_sorted, mx, my, mz;       // [nrhs][n_src]
    DBuf<float> qm;                         // [nrhs][n_src][2]: q and mu side by side (both layers)
    DBuf<double> col_scale;                 // half-width per vector index
    DBuf<double> col_iscale;                // 1 / half-width per vector index (Chebyshev M2L expansion)
    DBuf<int8_t> expand_add;                // per vector index: 1 where P2L writes the node values (Chebyshev expansion adds there, writes elsewhere)
    DBuf<float> trg_nrm_user;               // [n_trg][3] target normals, caller's order

    DBuf<int32_t> p2m_items, p2m_roff, p2m_rng;
    int n_p2m = 0;
    DBuf<int32_t> p2l_items, p2l_roff, p2l_rng;
    int n_p2l = 0;
    GemmJob p2m_proj, p2l_proj;     // check potentials -> compressed state
    std::vector<GemmJob> m2m_jobs;  // bottom-up
    std::vector<GemmJob> l2l_jobs;  // top-down
    GemmJob c2e_down, c2e_up;
    GemmJob cheb_compress, cheb_expand;  // Chebyshev: W -> M2L basis (boxes with sources), back (with targets)
    std::vector<ChebJob> cheb_m2m, cheb_l2l;  // bottom-up / top-down, one per level
    // M2L: tiles with their active directions
    int m2l_ntile = 0, m2l_ncol = 0;
    int64_t m2l_steps = 0;  // (tile, direction) products the dedicated kernel runs
    DBuf<int64_t> m2l_toff;
    DBuf<int32_t> m2l_dir, m2l_src, m2l_cols;
    DBuf<float> m2l_zero;  // a zero source chunk (columns without a source)
    DBuf<int32_t> m2l_slot;  // per work item: partial-sum slot, or -1 (adds into dt)
    int m2l_nsplit = 0, m2l_pieces_per_tile = 1;  // tiles cut into pieces; pieces per cut tile
    DBuf<float> m2l_partial;                      // [slot][ncol][r_pad] partial sums of cut tiles
    DBuf<int32_t> m2l_red_cols, m2l_red_slot0, m2l_red_k;  // per cut tile: columns, first slot, pieces
    int m2l_ngather = 0, m2l_pair_tiles = 0;              // pair tiles: targets gathered, tiles
    DBuf<int32_t> m2l_gt, m2l_goff, m2l_gidx;             // per target vector: its partial rows (CSR)

    DBuf<int32_t> wleaf, wt0, soff, sbox, poff, prng;
    DBuf<int32_t> pmid;       // per box: its point ranges [poff, pmid) need the r < delta test
    int64_t p2p_tested = 0;   // target x source pairs in those ranges
    DBuf<int8_t> skind;
    int nwork = 0;

    int64_t p2p_pairs = 0;
    int64_t m2l_pairs = 0;
    int64_t surf_evals = 0;
    int64_t p2m_evals = 0;
    int64_t p2l_evals = 0;
    double setup_ms = 0;
    // host wall time of the setup phases (ms), in the order of fmm_info.setup_phase_ms
    double setup_phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int leaf_from_cache = 0;  // leaf_size = 0 resolved from the tuning cache (1) or the default (0)

    // captured apply (fmm_set_graph): replayed while the argument pointers match
    struct Graph {
        bool enabled = false;
        hipStream_t stream = nullptr;
        hipEvent_t in = nullptr, out = nullptr;
        hipGraphExec_t exec = nullptr;
        std::array<const void *, 4> key{};
    } graph;

    // Chebyshev form: P2L (needs only the points) and the leaf evaluation
    // (near field and M2P, needs only the node weights) run on a plan-owned
    // side stream, beside P2M/M2M and M2L/L2L on the caller's stream
    hipStream_t side = nullptr;
    hipEvent_t fork0 = nullptr, p2l_done = nullptr, fork = nullptr, join = nullptr;

    bool timing = false;
    // Stage events of timed applies, one set per slot. Applies take the slots
    // in turn and do not wait for their events; fmm_stage_times collects them
    // (an apply that finds its slot still uncollected collects it first).
    struct TimeSlot {
        hipEvent_t ev[ST_COUNT + 1] = {};
        hipEvent_t side[4] = {};       // P2L start / end, evaluation start / end on the side stream
        hipEvent_t l2l_end = nullptr;  // end of L2L before the join
        bool pending = false;
    };
    static constexpr int kTimeSlots = 16;
    TimeSlot tslot[kTimeSlots];
    int tnext = 0;                       // the slot the next timed apply takes
    double stage_sum[ST_COUNT] = {};     // over the applies collected since the last report
    int stage_n = 0;
    double stage_ms[ST_COUNT] = {-1, -1, -1, -1, -1, -1, -1};
    bool have_times = false;
};

void plan_build_worklists(Plan &P, hipStream_t s);
void plan_apply(Plan &P, const float *q, const float *mu, float *pot, float *field, hipStream_t s,
                bool capturing = false);
// The same apply as one captured HIP graph, replayed when called again with
// the same pointers (re-captured otherwise). Runs on a plan-owned stream
// ordered after and before the caller's stream s.
void plan_apply_graph(Plan &P, const float *q, const float *mu, float *pot, float *field, hipStream_t s);
// Stage times: the mean over the timed applies since the last report (every
// pending slot collected first); kept for later calls when there were none.
void plan_report_times(Plan &P);
void plan_release_graph(Plan &P);
// Streams and events the plan owns (side stream, fork/join, timing events).
void plan_create_side(Plan &P);
void plan_release_events(Plan &P);
// Dielectric problem (Sec. II.C): right-hand side with free charges (Eq. rhs)
// into device b, and per-body forces eps_m sigma E a (sigma = sigma + sigma2,
// sigma2 may be NULL) summed over the bodies' index ranges into host forces.
void dielectric_rhs(Plan &P, const float *sigma_f, const float *areas, const float *curv, const float *eps_i,
                    double eps_m, const double *e0, double *b, hipStream_t s);
// The same right-hand side with the charge and its field in a fixed scratch
// array (no device allocation, no synchronisation: stream-ordered); at most
// kNoAllocMaxPoints points.
constexpr int64_t kNoAllocMaxPoints = 2000000;
void dielectric_rhs_noalloc(Plan &P, const float *sigma_f, const float *areas, const float *curv,
                            const float *eps_i, double eps_m, const double *e0, double *b, hipStream_t s);
void body_forces(Plan &P, const float *sigma, const float *sigma2, const float *areas, const float *curv,
                 double eps_m, const double *e0, int n_body, const int64_t *body_off, double *forces, hipStream_t s);
// Leaf-size tuning cache (tune.hip): the key of a plan's configuration, the
// cache file (FMM_TUNE_CACHE, else ~/.cache/fmm_mi355x_tune.jsonl), lookup
// and store; random densities for trial runs.
std::string tune_key(const fmm_options &o, int64_t points_per_instance, bool tsm, bool batch);
std::string tune_cache_path();
bool tune_cache_lookup(const std::string &path, const std::string &key, int &leaf, int &pieces);
void tune_cache_store(const std::string &path, const std::string &key, int leaf, int pieces, double ms);
void fill_random(float *out, int64_t n, uint32_t seed, hipStream_t s);
constexpr int kDefaultAutoLeaf = 128;  // leaf_size = 0 with no cache entry

void plan_gmres(Plan &P, const fmm_operator &op, const double *b, double *x, double rtol, int restart, int max_iter,
                int *iters, double *rel_res, int *status, hipStream_t s);

}  // namespace fmm
