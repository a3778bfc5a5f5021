/*
 * fmm.h — C ABI of the MI355X kernel-independent FMM boundary-integral library.
 *
 * The library evaluates the quadrature sum of the general boundary-integral
 * problem (arXiv:1605.01715, Sec. II.A, Eq. sum_fmm)
 *
 *     f(r_i) = sum_j K(r_i, r_j) sigma_j
 *
 * in O(N) with a kernel-independent fast multipole method, for the Laplace
 * kernels of the paper's two model problems:
 *
 *   single layer  q_j / (4 pi |x_i - y_j|)
 *   double layer  mu_j (x_i - y_j) . n_j / (4 pi |x_i - y_j|^3)
 *                 (Sec. II.B Eq. fk_integral; the normal derivative is applied
 *                  at the particle-to-multipole step, Sec. III.A.1 Eq. p2m)
 *   field         -grad of the single layer, q_j (x_i - y_j) / (4 pi |x_i - y_j|^3)
 *                 (Sec. III.A.2 Eq. kernel_pol)
 *
 * Targets and sources may be distinct point sets (the target-source model of
 * Sec. III.A.1). A pair closer than the tolerance radius `cutoff` contributes
 * nothing (Sec. III.A.1, singularity exclusion). Quadrature weights are folded
 * into the densities by the caller (sigma_j = phi_1(r_j) w(r_j), Sec. III.A.1).
 *
 * GMRES solves the matrix-free systems of Sec. III (A x = b with only the
 * action of A defined), using one FMM evaluation per iteration.
 *
 * Conventions for every entry point:
 *   - Every pointer argument marked "device" is HIP device memory on the
 *     current device; every pointer marked "host" is ordinary host memory.
 *   - Device arrays are read or written in stream order on `hip_stream`
 *     (a hipStream_t; NULL is the default stream). The caller owns them and
 *     may free or reuse them once the stream has passed the call.
 *   - All functions return an fmm_status and never throw or abort across the
 *     ABI. On failure, fmm_last_error() returns a message describing it
 *     (thread-local, valid until the next call on the same thread).
 *   - Point arrays are float32, array-of-structures [n][3] (x, y, z).
 *
 * Environment variables read by the library:
 *   FMM_LOG            set (and not "0"): diagnostics on stderr
 *   FMM_TUNE_CACHE     the autotuner's cache file (fmm_autotune)
 *   FMM_OP_CACHE       directory of the cached float64 factorisations the
 *                      operators are built from (default ~/.cache/fmm_mi355x_ops;
 *                      "0" turns the cache off). A file that does not match its
 *                      header or checksum is ignored and rewritten.
 *   FMM_FAULT_INJECT   "alloc:<k>": the k-th device allocation counted from
 *                      when the variable took this value fails with
 *                      FMM_ERR_NOMEM, as if the device were out of memory
 *                      (for tests of the error paths; every buffer the failing
 *                      call had allocated is released)
 */
#ifndef FMM_MI355X_H
#define FMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s *fmm_plan; /* opaque; owned by the library */

typedef enum {
    FMM_OK = 0,
    FMM_ERR_ARG = 1,           /* invalid argument, detected before any device work */
    FMM_ERR_NOMEM = 2,         /* a device or host allocation failed */
    FMM_ERR_DEVICE = 3,        /* a HIP runtime call failed */
    FMM_ERR_NOT_CONVERGED = 4, /* gmres_solve reached max_iter; outputs hold the best iterate */
    FMM_ERR_STATE = 5          /* the plan was destroyed or is not usable */
} fmm_status;

/* Source kernels (bitmask). */
enum { FMM_SRC_SINGLE = 1, FMM_SRC_DOUBLE = 2 };
/* Outputs (bitmask). FIELD is defined for the single layer only. */
enum { FMM_OUT_POT = 1, FMM_OUT_FIELD = 2 };
/* Arithmetic of the box-to-box (M2L) translations. Every other step is float32
 * data (float64 for the SURFACE form's check-to-equivalent maps and the
 * CHEBYSHEV interpolation weights; the CHEBYSHEV changes of basis into and out
 * of the M2L basis are float32 on the matrix cores). The split forms run on
 * the bfloat16 matrix cores with float32 accumulation (the schemes of Henry,
 * Tang and Heinecke, ARITH 2019):
 *   SPLIT_BF16    both operands in three bfloat16 parts x = h + m + l, six
 *                 products hh hm mh mm hl lh (bf16x6): about float32 accuracy
 *   SPLIT_BF16X4  two parts x = h + m, four products (bf16x4): each operand
 *                 rounded to 16 significant bits, products of those exact
 *   SPLIT_BF16X3  two parts, three products hh hm mh (bf16x3)
 * The two-part forms copy two thirds of the bytes and issue two thirds (x4)
 * or half (x3) of the matrix-core work of bf16x6, at about 2^-16 relative
 * error per product instead of 2^-22. */
enum { FMM_PREC_FP32 = 0, FMM_PREC_SPLIT_BF16 = 1, FMM_PREC_SPLIT_BF16X3 = 2, FMM_PREC_SPLIT_BF16X4 = 3 };
/* Far-field representation of a box (Sec. III.A.1 Eq. p2m: the far field is
 * interpolated at the sources, translated with the plain 1/r kernel, and
 * interpolated at the targets).
 * SURFACE: equivalent densities on a box surface of p points per edge,
 *   fitted to the potential on a check surface (kernel-independent FMM in the
 *   equivalent-surface form).
 * CHEBYSHEV: the paper's own form. Weights at the n^3 tensor-product Chebyshev
 *   nodes of the box (n = order, 2..8): P2M interpolates the sources onto the
 *   nodes, with the double layer's normal derivative applied to the
 *   interpolating polynomial; M2L is the 1/r kernel between node sets, kept as
 *   r x r matrices in a basis shared by all 316 directions (truncated at
 *   pinv_eps, the SVD threshold); L2P interpolates back to the targets. */
enum { FMM_BASIS_SURFACE = 0, FMM_BASIS_CHEBYSHEV = 1 };

typedef struct {
    int order;          /* SURFACE: p, points per edge of the equivalent/check surfaces, 2..10;
                           CHEBYSHEV: n, interpolation nodes per axis, 2..8 */
    int leaf_size;      /* s: adaptive tree splits boxes holding more than s points (targets + sources);
                           0: the cap fmm_autotune stored for this configuration (see there), else 128 */
    int uniform_depth;  /* > 0: uniform tree, every box above this level is split (0 = adaptive) */
    int max_depth;      /* deepest level, <= 21 */
    int precision;      /* FMM_PREC_* */
    int src_kernels;    /* FMM_SRC_* bitmask: which densities fmm_apply takes */
    int outputs;        /* FMM_OUT_* bitmask */
    int nrhs;           /* number of density vectors per apply, 1..4 */
    float cutoff;       /* tolerance radius (Sec. III.A.1), e.g. 1e-5; r < cutoff excluded, r == 0 always */
    double root[4];     /* root cube x0, y0, z0, width; width <= 0: derived from the points */
    double pinv_eps;    /* relative SVD truncation (SURFACE: of the check-to-equivalent maps;
                           CHEBYSHEV: of the shared M2L basis, the count kept then rounded up
                           to a multiple of 32, the size M2L is padded to); <= 0: default */
    int m2l_pieces;     /* M2L work items per tile of target boxes, 1..8; 0: chosen at setup by
                           simulating the dispatch on the GPU's compute units (the default) */
    int basis;          /* FMM_BASIS_*: far-field representation (default SURFACE) */
} fmm_options;

/* Fill `opt` with defaults: order 6, leaf_size 64, adaptive, max_depth 21, FP32,
 * single layer, potential, nrhs 1, cutoff 1e-5, root derived, default pinv_eps,
 * surface basis. */
void fmm_default_options(fmm_options *opt);

/*
 * Build a plan: octree over targets and sources (Morton order, Sec. III.B),
 * interaction lists, translation operators and work lists.
 *   src_xyz  device [n_src][3]   source points (required when n_src > 0)
 *   src_nrm  device [n_src][3]   source normals; required iff FMM_SRC_DOUBLE
 *   trg_xyz  device [n_trg][3]   target points, or NULL: targets are the sources
 *   trg_nrm  device [n_trg][3]   target normals (used by FMM_OP_DIELECTRIC), or NULL
 *   opt      host               options (copied)
 *   out      host               receives the plan
 * Errors: FMM_ERR_ARG for NULL required pointers, n < 0, order outside 2..10,
 * leaf_size < 1, max_depth outside 1..21, nrhs outside 1..4, a field output
 * with the double layer, and non-finite coordinates or normals (detected by a
 * device reduction before the tree is built; no plan is created).
 * n_src == 0 is allowed: every apply then returns zeros.
 */
int fmm_setup(const float *src_xyz, const float *src_nrm, int64_t n_src,
              const float *trg_xyz, const float *trg_nrm, int64_t n_trg,
              const fmm_options *opt, void *hip_stream, fmm_plan *out);

/*
 * Build one plan over many independent instances (separate bodies that never
 * interact, e.g. a batch of ferromagnet surfaces each solved on its own,
 * Sec. II.B with one body per instance). Every instance gets its own octree
 * and lists; the plan runs each stage of fmm_apply as one launch over all of
 * them. Inputs are the instances' points concatenated in instance order:
 *   n_inst   host              number of instances, >= 1
 *   src_off  host [n_inst + 1] prefix offsets into the sources (src_off[0] = 0)
 *   trg_off  host [n_inst + 1] prefix offsets into the targets, or NULL
 *                              (then trg_xyz must be NULL: targets are the sources)
 *   src_xyz, src_nrm, trg_xyz, trg_nrm as in fmm_setup, concatenated
 * fmm_apply then takes densities [nrhs][total sources] and returns outputs
 * [nrhs][total targets] in the same concatenated order; gmres_solve solves the
 * block-diagonal system. Each instance's root cube is derived from its own
 * points unless opt->root gives one cube for all. Errors: as fmm_setup, plus
 * FMM_ERR_ARG for n_inst < 1, offsets that do not start at 0 or decrease, and
 * trg_off without trg_xyz (or the reverse).
 */
int fmm_setup_batch(int n_inst, const int64_t *src_off, const int64_t *trg_off, const float *src_xyz,
                    const float *src_nrm, const float *trg_xyz, const float *trg_nrm, const fmm_options *opt,
                    void *hip_stream, fmm_plan *out);

/*
 * One FMM evaluation (Sec. II.A Eq. sum_fmm with the kernels above).
 *   q      device [nrhs][n_src]      single-layer densities (weights folded in), or NULL
 *   mu     device [nrhs][n_src]      double-layer strengths, or NULL
 *   pot    device [nrhs][n_trg]      potentials, or NULL (overwritten)
 *   field  device [nrhs][n_trg][3]   fields, or NULL (overwritten)
 * At least one of q/mu that the plan's src_kernels names must be given, and
 * every output requested here must be in the plan's outputs.
 * A plan holds scratch: two applies of one plan must not overlap in time.
 */
int fmm_apply(fmm_plan plan, const float *q, const float *mu, float *pot, float *field,
              void *hip_stream);

/* Matrix-free operators for gmres_solve (targets = sources; n = n_src):
 *   FMM_OP_FK          y = a .* x + D[w .* x]            (Eq. fk_integral_discrete,
 *                                                          a = Omega/(4 pi) - 1, w = weights)
 *   FMM_OP_DIELECTRIC  y = a .* x + c .* (n_t . E[w .* x]) (Eqs. Ax, Eb, pol_discret,
 *                                                          a = ebar + self term, c = deps, w = areas)
 * D is the double-layer potential and E the single-layer field of the plan;
 * a, c, w are device float32 [n]. */
enum { FMM_OP_FK = 1, FMM_OP_DIELECTRIC = 2 };
typedef struct {
    int kind;
    const float *a;
    const float *c;
    const float *w;
} fmm_operator;

/*
 * Restarted GMRES(restart) on the operator above (Sec. III, matrix-free; the
 * paper's tolerance is 1e-5, Sec. IV.B). Orthogonalisation (classical
 * Gram-Schmidt twice) and residual norms are float64 on the device; one
 * fmm_apply and one device-to-host copy of the step's coefficients per
 * iteration. restart is 1..500; the Krylov basis takes (restart + 1) n
 * float64 of device memory, allocated per call.
 *   b        device double [n]    right-hand side
 *   x        device double [n]    in: initial guess, out: solution (best iterate)
 *   iters    host int             iterations done
 *   rel_res  host double          final true relative residual ||b - A x|| / ||b||
 * Returns FMM_ERR_NOT_CONVERGED (with iters, rel_res and x filled) when
 * max_iter is reached first.
 */
int gmres_solve(fmm_plan plan, const fmm_operator *op, const double *b, double *x,
                double rtol, int restart, int max_iter, int *iters, double *rel_res,
                void *hip_stream);

/*
 * Dielectric bodies around the solve (Sec. II.C, epsilon_0 = 1). The plan must
 * be single-layer with field output, targets = sources, nrhs = 1, and target
 * normals given at setup (the element normals). The field of a surface charge
 * s at element j is the plan's field of s.a plus the self-patch term
 * s_j sqrt(pi a_j) H_j / (4 pi) n_j (Eq. pol_discret, the reading of the
 * garbled term as the principal-value field of a uniformly charged cap).
 *
 * fmm_dielectric_rhs: b = (1 - ebar) sigma_f - deps n . (E_f + E0)
 *   (Eq. rhs with Eq. Ef and no volume charge; ebar = (eps_i + eps_m)/2,
 *   deps = eps_m - eps_i; a charge Q on a sphere of radius r is
 *   sigma_f = Q / (4 pi r^2)).
 *   sigma_f, areas, curvature (mean curvature H), eps_i: device float [n];
 *   eps_m: medium permittivity; e0: host double [3] uniform external field or
 *   NULL; b: device double [n], written. Synchronous on the stream.
 * fmm_body_forces: F_i = sum over the elements of body i of
 *   eps_m s_j a_j (E_j + E0), s = sigma_f + sigma_b, E the field of s
 *   (Sec. II.C, force density eps_m sigma E).
 *   sigma_b: device float [n] or NULL; body i is elements
 *   body_off[i] .. body_off[i+1] - 1 (host int64 [n_body + 1], from 0 to n,
 *   nondecreasing); forces: host double [n_body][3], written. Per-body sums
 *   run in a fixed order (deterministic).
 * Errors: FMM_ERR_ARG for NULL arguments, eps_m <= 0, a plan of the wrong kind
 * and bad body offsets.
 */
int fmm_dielectric_rhs(fmm_plan plan, const float *sigma_f, const float *areas, const float *curvature,
                       const float *eps_i, float eps_m, const double *e0, double *b, void *hip_stream);
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * right-hand side as fmm_dielectric_rhs, same arguments and results, with the
 * charge density and its field held in a fixed scratch array that the library
 * keeps on each GPU for the life of the process (32 MiB per GPU). It calls no
 * allocator and does not synchronise: b is written in stream order. At most
 * 2,000,000 points (FMM_ERR_ARG beyond). Every call on a GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (two streams, two
 * threads) race and must be serialised by the caller.
 */
int fmm_dielectric_rhs_noalloc(fmm_plan plan, const float *sigma_f, const float *areas, const float *curvature,
                               const float *eps_i, float eps_m, const double *e0, double *b, void *hip_stream);
int fmm_body_forces(fmm_plan plan, const float *sigma_f, const float *sigma_b, const float *areas,
                    const float *curvature, float eps_m, const double *e0, int n_body, const int64_t *body_off,
                    double *forces, void *hip_stream);

/* Release the plan and its device memory. NULL is a no-op. The handle stays
 * known to the library as destroyed (a few bytes are kept per handle until the
 * process ends, so no later plan reuses it): every later call that takes it,
 * fmm_destroy included, returns FMM_ERR_STATE without touching freed memory.
 * A pointer the library never issued gives FMM_ERR_ARG. Destroying a plan
 * while another thread is inside a call on it is not allowed. */
int fmm_destroy(fmm_plan plan);

/*
 * Leaf-size tuning by trial runs (the paper tunes its octree height per problem
 * by trial runs, Sec. III.A.1 and Sec. IV.A). For every leaf cap in
 * space->leaf_sizes (and every M2L piece count in space->pieces, or the
 * setup's own choice when n_pieces = 0) a plan is built with the caller's
 * other options, applied once to random densities to warm up and then
 * space->reps times, timed with HIP events on the stream; the median apply
 * time decides. Accuracy is not tuned (the form, order and threshold stay the
 * caller's). Points are given as for fmm_setup (n_inst = 0) or
 * fmm_setup_batch (n_inst >= 1 with its offsets; n_src, n_trg unused).
 *   cache_path  host string: file to record the choice in (JSON lines), "" for
 *               the default (FMM_TUNE_CACHE, else ~/.cache/fmm_mi355x_tune.jsonl),
 *               NULL to record nothing. fmm_setup and fmm_setup_batch with
 *               leaf_size = 0 look the choice up in the default file by the
 *               key of their configuration: device, basis, order, threshold,
 *               arithmetic, kernels, outputs, nrhs, separate targets, batch,
 *               and floor(log2(points per instance)).
 *   out         host: the choice, its median apply time, and every trial.
 * Builds and releases one plan per trial (device memory of one plan at a time
 * plus the random densities and outputs).
 */
typedef struct {
    int n_leaf;          /* 1..8 */
    int leaf_sizes[8];
    int n_pieces;        /* 0..4; 0: the setup's own choice */
    int pieces[4];
    int reps;            /* timed applies per trial, 1..100 */
} fmm_tune_space;
typedef struct {
    int leaf_size, m2l_pieces;  /* the choice (m2l_pieces as the plan used it) */
    double ms;                  /* its median apply time */
    int n_tried;
    int tried_leaf[32], tried_pieces[32];
    double tried_ms[32], tried_setup_ms[32];
} fmm_tune_result;
int fmm_autotune(int n_inst, const int64_t *src_off, const int64_t *trg_off, const float *src_xyz,
                 const float *src_nrm, int64_t n_src, const float *trg_xyz, const float *trg_nrm, int64_t n_trg,
                 const fmm_options *opt, const fmm_tune_space *space, const char *cache_path, fmm_tune_result *out,
                 void *hip_stream);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *fmm_last_error(void);

/*
 * Plain O(n_trg * n_src) evaluation of the same sum on the GPU (no tree):
 * the all-pairs reference and small-problem path. Arguments as fmm_apply
 * with nrhs = 1; nrm is required iff mu != NULL.
 */
int fmm_direct(const float *src_xyz, const float *src_nrm, int64_t n_src,
               const float *trg_xyz, int64_t n_trg, const float *q, const float *mu,
               float cutoff, float *pot, float *field, void *hip_stream);

/* Plan statistics (host struct filled from host-side copies). */
typedef struct {
    int64_t n_src, n_trg, n_points;      /* points inserted in the tree = n_points */
    int64_t n_boxes, n_leaves, n_levels;
    int64_t n_u, n_v, n_w, n_x;          /* list entries (U counts leaf pairs, self included) */
    int64_t n_surface;                   /* points of a box's far-field representation: n_s =
                                            6 (p-1)^2 + 2 surface points, or n^3 Chebyshev nodes */
    int64_t p2p_pairs;                   /* near-field point pairs evaluated per apply */
    int64_t m2l_pairs;                   /* M2L box pairs (V-list entries with sources) per rhs */
    int64_t surf_evals;                  /* target x surface-point kernel evaluations (L2P + M2P; for
                                            CHEBYSHEV M2P only, its L2P interpolates) per rhs */
    int64_t p2m_evals;                   /* P2M: (surface point or node) x source pairs per rhs */
    int64_t m2l_columns;                 /* matrix-vector products the M2L kernel computes, padding
                                            included (m2l_pairs / m2l_columns is its fill) */
    int64_t rank;                        /* r: singular values kept (SURFACE: of the check-from-
                                            equivalent map; CHEBYSHEV: of the shared M2L basis, a
                                            multiple of 32 or n^3); M2L acts on r values per box
                                            and rhs */
    int64_t m2l_pieces;                  /* M2L work items per tile of 128 target boxes (load
                                            balance across CUs; pieces add up in a fixed order) */
    int64_t m2l_pair_tiles;              /* M2L work items of one direction whose columns are
                                            (target, source) pairs (sparse V lists) */
    int64_t basis;                       /* FMM_BASIS_* of the plan */
    double root[4];                      /* root cube actually used */
    double setup_ms;                     /* wall time of fmm_setup */
    int64_t leaf_size;                   /* leaf cap the plan was built with */
    int64_t leaf_from_cache;             /* 1 when leaf_size = 0 was resolved from the tuning cache */
    int64_t p2l_evals;                   /* P2L: (check point or node) x X-list source evaluations per rhs */
    double setup_phase_ms[8];            /* host wall time of the setup phases, each ended by a stream
                                            synchronisation: [0] bounding box, Morton keys and radix
                                            sort; [1] octree levels, boxes and sorted point data;
                                            [2] U/V/W/X lists and their host copies; [3] operators
                                            (cached per device after the first plan of a form);
                                            [4] per-box buffers; [5] the M2L schedule (tiles,
                                            pieces, partial-sum slots); [6] the other work lists;
                                            [7] unused (0). A batch builds all its instance trees
                                            in the one pass of [0]-[2] */
} fmm_info;
int fmm_plan_info(fmm_plan plan, fmm_info *info);

/*
 * Copy the tree and lists to host memory for inspection. Any pointer may be
 * NULL to skip it. Sizes: box arrays [n_boxes]; list offsets [n_boxes+1];
 * list entries [n_u|n_v|n_w|n_x]; perms [n_src] / [n_trg]; keys [n_points].
 * Lists are sorted ascending within each box. Boxes are numbered level by
 * level, in Morton order within a level.
 */
typedef struct {
    int32_t *level, *anchor /* [n_boxes][3] */, *parent;
    int64_t *begin, *end;               /* range in the sorted combined point order */
    int64_t *tbeg, *tend, *sbeg, *send; /* target / source ranges */
    int32_t *u_off, *u_idx, *v_off, *v_idx, *w_off, *w_idx, *x_off, *x_idx;
    int64_t *src_perm, *trg_perm;       /* user index of the k-th sorted source / target */
    uint64_t *keys;                     /* sorted Morton keys of the combined points */
} fmm_tree_export;
int fmm_export_tree(fmm_plan plan, const fmm_tree_export *out);

/*
 * Inspection hook (no plan): split float32 values into the three bfloat16
 * parts x = h + m + l that the split-BF16 M2L form multiplies (h = bf16(x),
 * m = bf16(x - h), l = bf16(x - h - m), round to nearest even; the bf16x6
 * scheme of Henry, Tang and Heinecke, ARITH 2019), with the same device code
 * the library runs:
 *   which = 0  the split of the far-field state made at every apply: `in`
 *              holds count vectors of r_pad values;
 *   which = 1  the split of the translation matrices made when operators are
 *              built: `in` holds count r_pad x r_pad row-major matrices.
 *   in     device float [count * r_pad] or [count * r_pad * r_pad]
 *   parts  device uint16 [3][the same number], bit patterns of h, m, l, in
 *          the values' row-major order
 * r_pad is a multiple of 32 in 32..512, count in 0..2^24 (FMM_ERR_ARG
 * otherwise). Allocates a temporary; synchronous on the stream.
 */
int fmm_split_bf16(int which, int r_pad, int64_t count, const float *in, uint16_t *parts, void *hip_stream);

/* Host utility (no device work): truncated-SVD pseudo-inverse of the n x n
 * row-major float64 matrix K (host), singular values below eps * sigma_max
 * dropped, written to out (host, n x n row-major). This is the
 * check-to-equivalent map construction used by fmm_setup. */
int fmm_pinv(const double *K, int n, double eps, double *out);

/* Host utility: the unit surface Y(p) used for order p, [n_s][3] float64
 * written to out (host); returns n_s through *ns. out may be NULL to query. */
int fmm_unit_surface(int p, double *out, int *ns);

/* Turn per-stage device timing on or off for later applies of this plan
 * (hipEvents recorded on the streams the stages run on). A timed apply does
 * not wait for its events: they are read by fmm_stage_times. The plan keeps
 * the events of up to 16 timed applies; an apply that would reuse the events
 * of one not yet read waits for those and adds them to the next report. */
int fmm_set_timing(fmm_plan plan, int enable);

/* Turn graph replay on or off for later applies of this plan. When on, the
 * first fmm_apply records the whole apply (every kernel of every stage) into
 * a HIP graph and later calls with the same density and output pointers
 * replay it with one launch; other pointers re-record it. The graph runs on a
 * stream the plan owns, ordered after the work already queued on the
 * caller's stream and before the work queued after the call, so the call
 * behaves like the ordinary apply. While stage timing is on (fmm_set_timing)
 * applies run the ordinary way. Turning it off releases the graph. gmres_solve
 * replays one graph per solve for its matvecs. */
int fmm_set_graph(fmm_plan plan, int enable);

/*
 * Copy per-box check potentials of the last apply to host memory, rhs 0.
 * The far field is carried in compressed form (r values per box, see
 * fmm_info.rank): the upward state is U_r^T u and the downward state V_r^T d,
 * with K = U S V^T the check-from-equivalent map of the unit box. What is
 * written is the reconstruction
 * which = 0: U_r U_r^T u, the upward check potential projected onto the kept
 *            left singular vectors, [n_boxes][n_s];
 * which = 1: V_r V_r^T d, the same for the downward check potential after the
 *            parent's contribution, [n_boxes][n_s].
 * For a CHEBYSHEV plan the node values themselves are written: which = 0 the
 * multipole weights W, which = 1 the local expansion L at the nodes (after
 * M2L, P2L and L2L), [n_boxes][n^3].
 * Boxes that were not computed hold zeros.
 */
int fmm_export_stage(fmm_plan plan, int which, float *host_out);

/* Device time (ms) of each stage: the mean over the applies made with
 * timing on (fmm_set_timing) since the previous call, which this call waits
 * for; when there were none since, the previous means again; -1 when no apply
 * was ever timed. Order: P2M, M2M, P2L, M2L, L2L, C2E, EVAL.
 * Both forms run the leaf evaluation's near field on a second stream beside
 * M2L (its time is taken there). CHEBYSHEV plans also run P2L there, C2E is
 * their L2P, and their M2L stage times the translation kernel, the reduction
 * and the gather, while the split of its input (split-BF16) is in no stage.
 * SURFACE plans expand the upward densities in the M2M stage, and their EVAL
 * is the near field (second stream) plus the L2P pass after the join. */
int fmm_stage_times(fmm_plan plan, double *ms /* [7] */);

/* Measurement utility (no step of the method): an issue-rate probe, whose
 * lanes run independent chains so that only instruction issue limits it,
 * queued on hip_stream (asynchronous; the caller times it):
 *   kind = 0  float32 fused multiply-adds (v_fma_f32), 16 chains;
 *   kind = 1  float32 reciprocal square roots (v_rsq_f32), 16 chains;
 *   kind = 2  8 chains, each step 12 fused multiply-adds and one reciprocal
 *             square root (the ratio of the leaf evaluation's pair loop);
 *   kind = 3  32-bit integer add then exclusive or, 8 chains;
 *   kind = 4  bfloat16 matrix products (v_mfma_f32_32x32x16_bf16, 32768
 *             FLOP each) on operands held in registers, 4 accumulators; every
 *             lane's output is 512 iters.
 *   nthreads  lanes, a positive multiple of 256, at most 2^24 (workgroups
 *             of 256)
 *   iters     chain steps per lane, 1..2^20
 *   out       device float [nthreads], one value per lane (keeps the chains)
 *   instr_per_lane  if not NULL, receives the instructions of the chains:
 *             wave64 VALU instructions per lane, 16 iters (kinds 0, 1, 3) or
 *             104 iters (2); MFMA instructions per wave, 4 iters (4)
 * FMM_ERR_ARG for other arguments. */
int fmm_issue_probe(int kind, int64_t nthreads, int iters, float *out, int64_t *instr_per_lane, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FMM_MI355X_H */
