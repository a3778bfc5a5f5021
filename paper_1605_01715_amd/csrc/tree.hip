// Octree build and U/V/W/X interaction lists on the GPU.
//
// Points are mapped to 63-bit Morton keys and sorted (z-value ordering,
// Sec. III.B); the octree over targets and sources (Sec. III.A.1) is then
// built level by level from the sorted keys: a box is a maximal run of points
// sharing its key prefix, and only runs inside split boxes become children.
// The lists follow the standard kernel-independent FMM definitions (U: adjacent
// leaves, V: children of the parent's colleagues that are well separated,
// W/X: the adaptive-tree pairs between a leaf and finer boxes). Everything is
// integer arithmetic apart from the quantisation, which is two float64
// operations, so the tree is reproducible bit for bit.
#include "tree.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>

namespace fmm {

namespace {

constexpr int kBlock = 256;

__device__ __host__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
__device__ inline uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x100f00f00f00f00full;
    x = (x | (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x | (x >> 16)) & 0x1f00000000ffffull;
    x = (x | (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}
__device__ inline uint64_t morton(uint32_t ix, uint32_t iy, uint32_t iz) {
    return (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
}

__global__ void k_bbox_finite(const float *a, int64_t n, float *partial) {
    // partial[block][8]: min x,y,z, max x,y,z, nonfinite count (as float)
    __shared__ float sh[7][kBlock];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    float bad = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        for (int c = 0; c < 3; ++c) {
            float v = a[3 * i + c];
            if (!isfinite(v)) {
                bad += 1.f;
            } else {
                mn[c] = fminf(mn[c], v);
                mx[c] = fmaxf(mx[c], v);
            }
        }
    }
    for (int c = 0; c < 3; ++c) {
        sh[c][threadIdx.x] = mn[c];
        sh[3 + c][threadIdx.x] = mx[c];
    }
    sh[6][threadIdx.x] = bad;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            for (int c = 0; c < 3; ++c) {
                sh[c][threadIdx.x] = fminf(sh[c][threadIdx.x], sh[c][threadIdx.x + off]);
                sh[3 + c][threadIdx.x] = fmaxf(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + off]);
            }
            sh[6][threadIdx.x] += sh[6][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) partial[8 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// bbox over an array of n points; returns false if any coordinate is not finite
bool bbox(const float *a, int64_t n, hipStream_t s, double lo[3], double hi[3]) {
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    if (n == 0) return true;
    int nblk = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
    DBuf<float> part((size_t)8 * nblk);
    hipLaunchKernelGGL(k_bbox_finite, dim3(nblk), dim3(kBlock), 0, s, a, n, part.p);
    FMM_HIP(hipGetLastError());
    std::vector<float> h((size_t)8 * nblk);
    d2h(h.data(), part.p, h.size(), s);
    bool ok = true;
    for (int b = 0; b < nblk; ++b) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], (double)h[8 * b + c]);
            hi[c] = std::max(hi[c], (double)h[8 * b + 3 + c]);
        }
        if (h[8 * b + 6] != 0.f) ok = false;
    }
    return ok;
}

// Instance of global index j: the last i with off[i] <= j (instances with no
// points of this kind have off[i] == off[i + 1] and never match).
__device__ inline int32_t instance_of(const int64_t *off, int ni, int64_t j) {
    int lo = 0, hi = ni;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

// Morton key of combined point i (targets first when tsm) in the root cube of
// its instance: roots[5 k .. 5 k + 4] = x0, y0, z0, w, 2^21 / w of instance k.
// inst (with toff / soff) is NULL for a single tree.
__global__ void k_keys(const float *trg, const float *src, int64_t n_trg, int64_t n, bool tsm, const double *roots,
                       int ni, const int64_t *toff, const int64_t *soff, uint64_t *keys, int64_t *idx,
                       int32_t *inst) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const bool is_trg = tsm && i < n_trg;
    const float *p = is_trg ? trg + 3 * i : src + 3 * (tsm ? i - n_trg : i);
    int32_t k = 0;
    if (inst) {
        k = is_trg ? instance_of(toff, ni, i) : instance_of(soff, ni, tsm ? i - n_trg : i);
        inst[i] = k;
    }
    const double *r = roots + 5 * (int64_t)k;
    uint32_t q[3];
    for (int c = 0; c < 3; ++c) {
        double v = floor(((double)p[c] - r[c]) * r[4]);
        v = v < 0.0 ? 0.0 : v;
        v = v > 2097151.0 ? 2097151.0 : v;
        q[c] = (uint32_t)v;
    }
    keys[i] = morton(q[0], q[1], q[2]);
    idx[i] = i;
}

// forest: instance of the k-th sorted point as a sort key, and the identity
__global__ void k_inst_keys(const int64_t *order, const int32_t *inst, int64_t n, uint64_t *ik, int64_t *pos) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    ik[k] = (uint64_t)inst[order[k]];
    pos[k] = k;
}

__global__ void k_permute_sorted(const int64_t *pos, const uint64_t *keys, const int64_t *order, const uint64_t *ik,
                                 int64_t n, uint64_t *keys2, int64_t *order2, int32_t *sinst, int32_t *pbox,
                                 const int32_t *root_of) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t j = pos[k];
    keys2[k] = keys[j];
    order2[k] = order[j];
    sinst[k] = (int32_t)ik[k];
    pbox[k] = root_of[ik[k]];
}

// per-instance bounding boxes: one workgroup per instance,
// out[6 k .. 6 k + 5] = min x, y, z, max x, y, z over a[off[k] .. off[k + 1])
__global__ __launch_bounds__(kBlock) void k_inst_bbox(const float *a, const int64_t *off, double *out) {
    __shared__ float sh[6][kBlock];
    const int k = blockIdx.x;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = off[k] + threadIdx.x; i < off[k + 1]; i += kBlock)
        for (int c = 0; c < 3; ++c) {
            const float v = a[3 * i + c];
            mn[c] = fminf(mn[c], v);
            mx[c] = fmaxf(mx[c], v);
        }
    for (int c = 0; c < 3; ++c) {
        sh[c][threadIdx.x] = mn[c];
        sh[3 + c][threadIdx.x] = mx[c];
    }
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int c = 0; c < 3; ++c) {
                sh[c][threadIdx.x] = fminf(sh[c][threadIdx.x], sh[c][threadIdx.x + o]);
                sh[3 + c][threadIdx.x] = fmaxf(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[6 * k + threadIdx.x] = (double)sh[threadIdx.x][0];
}

// first level at which key[i] differs from key[i-1]; 22 if equal
// (0 where the instance changes, sinst = instance per sorted point or NULL)
__global__ void k_difflevel(const uint64_t *key, const int32_t *sinst, int64_t n, uint8_t *dl) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || (sinst && sinst[i] != sinst[i - 1])) { dl[i] = 0; return; }
    uint64_t x = key[i] ^ key[i - 1];
    if (x == 0) { dl[i] = 22; return; }
    int h = 63 - __clzll((long long)x);
    dl[i] = (uint8_t)(kMaxLevel - h / 3);
}

__global__ void k_split_flags(const int32_t *pbox, const uint8_t *dl, const int64_t *cbeg, const int64_t *cend,
                              int64_t n, int lvl, int uniform_depth, int leaf_size, int max_depth,
                              int32_t *flag) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t b = pbox[i];
    int32_t f = 0;
    if (b >= 0) {
        int64_t cnt = cend[b] - cbeg[b];
        bool split = uniform_depth > 0 ? (lvl < uniform_depth) : (cnt > leaf_size && lvl < max_depth);
        if (split && (i == cbeg[b] || dl[i] <= lvl + 1)) f = 1;
        if (!split) f = 0;
        // mark membership of split boxes in the high bit for the next pass
        if (split) f |= 2;
    }
    flag[i] = f;
}

__global__ void k_children(const int32_t *flag, const int32_t *cidx, const int32_t *pbox, int64_t n,
                           int64_t *nbeg, int32_t *nparent, int32_t *newpbox) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t f = flag[i];
    int32_t start = f & 1;
    if (start) {
        int32_t c = cidx[i];
        nbeg[c] = i;
        nparent[c] = pbox[i];
    }
    newpbox[i] = (f & 2) ? cidx[i] + start - 1 : -1;
}

__global__ void k_child_end(const int64_t *nbeg, const int32_t *nparent, const int64_t *cend, int64_t nc,
                            int64_t *nend) {
    int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    bool same = (c + 1 < nc) && nparent[c + 1] == nparent[c];
    nend[c] = same ? nbeg[c + 1] : cend[nparent[c]];
}

__global__ void k_strip_flag(int32_t *flag, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) flag[i] &= 1;
}

// assemble one level's boxes into the global arrays; a box's root cube is its
// instance's (sinst: instance per sorted point, NULL for a single tree; binst:
// instance per box, written when not NULL)
__global__ void k_assemble(const int64_t *lbeg, const int64_t *lend, const int32_t *lpar, int64_t nl, int lvl,
                           int64_t off, int64_t poff, const uint64_t *keys, const int32_t *sinst, const double *roots,
                           int32_t *level, int32_t *parent, int32_t *anchor, uint64_t *bkey, int64_t *begin,
                           int64_t *end, double *centre, double *half, int32_t *child, int32_t *binst) {
    int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= nl) return;
    int64_t g = off + c;
    level[g] = lvl;
    begin[g] = lbeg[c];
    end[g] = lend[c];
    const int32_t ii = sinst ? sinst[lbeg[c]] : 0;
    if (binst) binst[g] = ii;
    const double *r = roots + 5 * (int64_t)ii;
    uint64_t pre = lvl ? (keys[lbeg[c]] >> (3 * (kMaxLevel - lvl))) : 0ull;
    bkey[g] = pre;
    uint32_t a[3] = {compact3(pre >> 2), compact3(pre >> 1), compact3(pre)};
    double bw = r[3] / (double)(1ll << lvl);
    for (int k = 0; k < 3; ++k) {
        anchor[3 * g + k] = (int32_t)a[k];
        centre[3 * g + k] = r[k] + ((double)a[k] + 0.5) * bw;
    }
    half[g] = 0.5 * bw;
    int32_t p = lvl ? (int32_t)(poff + lpar[c]) : -1;
    parent[g] = p;
    if (p >= 0) {
        int o = (int)(((a[0] & 1u) << 2) | ((a[1] & 1u) << 1) | (a[2] & 1u));
        child[8 * (int64_t)p + o] = (int32_t)g;
    }
}

__global__ void k_leaf(const int32_t *child, int64_t nb, uint8_t *leaf) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    bool any = false;
    for (int o = 0; o < 8; ++o) any |= child[8 * b + o] >= 0;
    leaf[b] = any ? 0 : 1;
}

__global__ void k_type_flags(const int64_t *order, int64_t n, int64_t n_trg, int64_t *is_trg, int64_t *is_src) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    bool t = order[i] < n_trg;
    is_trg[i] = t ? 1 : 0;
    is_src[i] = t ? 0 : 1;
}

__global__ void k_ranges(const int64_t *begin, const int64_t *end, const int64_t *ct, const int64_t *cs,
                         int64_t nb, int64_t *tbeg, int64_t *tend, int64_t *sbeg, int64_t *send) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    tbeg[b] = ct[begin[b]];
    tend[b] = ct[end[b]];
    sbeg[b] = cs[begin[b]];
    send[b] = cs[end[b]];
}

// sorted SoA copies of the points (and perms); ct/cs may be NULL (no TSM)
__global__ void k_gather_points(const int64_t *order, int64_t n, int64_t n_trg, bool tsm, const int64_t *ct,
                                const int64_t *cs, const float *trg, const float *trg_nrm, const float *src,
                                const float *src_nrm, int64_t *trg_perm, int64_t *src_perm, float *tx, float *ty,
                                float *tz, float *tnx, float *tny, float *tnz, float *sx, float *sy, float *sz,
                                float *snx, float *sny, float *snz) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t o = order[i];
    if (!tsm) {
        src_perm[i] = o;
        sx[i] = src[3 * o];
        sy[i] = src[3 * o + 1];
        sz[i] = src[3 * o + 2];
        if (src_nrm) {
            snx[i] = src_nrm[3 * o];
            sny[i] = src_nrm[3 * o + 1];
            snz[i] = src_nrm[3 * o + 2];
        }
        return;
    }
    if (o < n_trg) {
        int64_t k = ct[i];
        trg_perm[k] = o;
        tx[k] = trg[3 * o];
        ty[k] = trg[3 * o + 1];
        tz[k] = trg[3 * o + 2];
        if (trg_nrm) {
            tnx[k] = trg_nrm[3 * o];
            tny[k] = trg_nrm[3 * o + 1];
            tnz[k] = trg_nrm[3 * o + 2];
        }
    } else {
        int64_t k = cs[i];
        int64_t j = o - n_trg;
        src_perm[k] = j;
        sx[k] = src[3 * j];
        sy[k] = src[3 * j + 1];
        sz[k] = src[3 * j + 2];
        if (src_nrm) {
            snx[k] = src_nrm[3 * j];
            sny[k] = src_nrm[3 * j + 1];
            snz[k] = src_nrm[3 * j + 2];
        }
    }
}

__global__ void k_copy_target_normals(const int64_t *perm, int64_t n, const float *nrm, float *nx, float *ny,
                                      float *nz) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t o = perm[i];
    nx[i] = nrm[3 * o];
    ny[i] = nrm[3 * o + 1];
    nz[i] = nrm[3 * o + 2];
}

// ------------------------------------------------------------------ lists
struct BoxView {
    const int32_t *level, *anchor, *child, *parent, *colleague;
    const uint8_t *leaf;
    const uint64_t *bkey;
    const int64_t *lvl_off;  // device copy [nlev + 1]
    int nlev;
    const int32_t *inst;     // forest: instance of each box (boxes of a level ordered by instance, then key)
};

// The box of instance `inst` at level lvl with anchor (ax, ay, az), or -1.
__device__ inline int32_t find_box(const BoxView &v, int lvl, int32_t ax, int32_t ay, int32_t az, int32_t inst) {
    if (lvl >= v.nlev) return -1;
    int32_t lim = 1 << lvl;
    if (ax < 0 || ay < 0 || az < 0 || ax >= lim || ay >= lim || az >= lim) return -1;
    uint64_t k = morton((uint32_t)ax, (uint32_t)ay, (uint32_t)az);
    int64_t lo = v.lvl_off[lvl], hi = v.lvl_off[lvl + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        const bool less = v.inst ? (v.inst[mid] < inst || (v.inst[mid] == inst && v.bkey[mid] < k)) : v.bkey[mid] < k;
        if (less) lo = mid + 1; else hi = mid;
    }
    return (lo < v.lvl_off[lvl + 1] && v.bkey[lo] == k && (!v.inst || v.inst[lo] == inst)) ? (int32_t)lo : -1;
}

__device__ inline bool adjacent(const BoxView &v, int32_t a, int32_t b) {
    int la = v.level[a], lb = v.level[b];
    int64_t sa = 1ll << (kMaxLevel - la), sb = 1ll << (kMaxLevel - lb);
    for (int k = 0; k < 3; ++k) {
        int64_t loa = (int64_t)v.anchor[3 * a + k] * sa;
        int64_t lob = (int64_t)v.anchor[3 * b + k] * sb;
        if (loa > lob + sb || lob > loa + sa) return false;
    }
    return true;
}

__global__ void k_colleagues(BoxView v, int64_t nb, int32_t *col) {
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nb * 27) return;
    int64_t b = t / 27;
    int k = (int)(t % 27);
    int dx = k / 9 - 1, dy = (k / 3) % 3 - 1, dz = k % 3 - 1;
    col[t] = find_box(v, v.level[b], v.anchor[3 * b] + dx, v.anchor[3 * b + 1] + dy, v.anchor[3 * b + 2] + dz,
                      v.inst ? v.inst[b] : 0);
}

__constant__ int8_t c_dirs[kNumDirs][3];

__global__ void k_vdense(BoxView v, int64_t nb, int32_t *vd) {
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nb * kNumDirs) return;
    int64_t b = t / kNumDirs;
    int k = (int)(t % kNumDirs);
    int lvl = v.level[b];
    int32_t r = -1;
    if (lvl >= 2) {
        int32_t a[3], na[3];
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
            a[c] = v.anchor[3 * b + c];
            na[c] = a[c] + c_dirs[k][c];
            int pd = (na[c] >> 1) - (a[c] >> 1);  // parents must be adjacent
            if (na[c] < 0 || pd < -1 || pd > 1) ok = false;
        }
        if (ok) r = find_box(v, lvl, na[0], na[1], na[2], v.inst ? v.inst[b] : 0);
    }
    vd[t] = r;
}

__global__ void k_vcount(const int32_t *vd, int64_t nb, int32_t *cnt) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    int c = 0;
    for (int k = 0; k < kNumDirs; ++k) c += vd[b * kNumDirs + k] >= 0;
    cnt[b] = c;
}

__global__ void k_vfill(const int32_t *vd, int64_t nb, const int32_t *off, int32_t *idx) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    int32_t p = off[b];
    for (int k = 0; k < kNumDirs; ++k) {
        int32_t a = vd[b * kNumDirs + k];
        if (a >= 0) idx[p++] = a;
    }
}

constexpr int kStack = 192;

// U and W lists of every leaf by a depth-first walk of the boxes adjacent to it.
template <bool Fill>
__global__ void k_uw(BoxView v, int64_t nb, int32_t *ucnt, int32_t *wcnt, const int32_t *uoff, int32_t *uidx,
                     const int32_t *woff, int32_t *widx, int32_t *overflow) {
    int64_t bb = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (bb >= nb || !v.leaf[bb]) {
        if (!Fill && bb < nb) { ucnt[bb] = 0; wcnt[bb] = 0; }
        return;
    }
    int32_t b = (int32_t)bb;
    int32_t nu = 0, nw = 0;
    int32_t ub = Fill ? uoff[b] : 0, wb = Fill ? woff[b] : 0;
    auto emit_u = [&](int32_t a) { if (Fill) uidx[ub + nu] = a; ++nu; };
    auto emit_w = [&](int32_t a) { if (Fill) widx[wb + nw] = a; ++nw; };
    int32_t stack[kStack];
    int sp = 0;
    emit_u(b);
    for (int k = 0; k < 27; ++k) {
        int32_t c = v.colleague[27 * (int64_t)b + k];
        if (c < 0 || c == b) continue;
        if (v.leaf[c]) emit_u(c);
        else if (sp < kStack) stack[sp++] = c;
        else overflow[0] = 1;
    }
    while (sp > 0) {
        int32_t c = stack[--sp];
        for (int o = 0; o < 8; ++o) {
            int32_t d = v.child[8 * (int64_t)c + o];
            if (d < 0) continue;
            if (adjacent(v, d, b)) {
                if (v.leaf[d]) emit_u(d);
                else if (sp < kStack) stack[sp++] = d;
                else overflow[0] = 1;
            } else {
                emit_w(d);
            }
        }
    }
    for (int32_t anc = v.parent[b]; anc >= 0; anc = v.parent[anc]) {
        for (int k = 0; k < 27; ++k) {
            int32_t c = v.colleague[27 * (int64_t)anc + k];
            if (c < 0 || c == anc) continue;
            if (v.leaf[c] && adjacent(v, c, b)) emit_u(c);
        }
    }
    if (!Fill) { ucnt[b] = nu; wcnt[b] = nw; }
}

__global__ void k_xcount(const int32_t *woff, const int32_t *widx, int64_t nb, int32_t *xcnt) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    for (int32_t k = woff[b]; k < woff[b + 1]; ++k) atomicAdd(&xcnt[widx[k]], 1);
}

__global__ void k_xfill(const int32_t *woff, const int32_t *widx, int64_t nb, const int32_t *xoff, int32_t *xcur,
                        int32_t *xidx) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    for (int32_t k = woff[b]; k < woff[b + 1]; ++k) {
        int32_t d = widx[k];
        int32_t p = atomicAdd(&xcur[d], 1);
        xidx[xoff[d] + p] = (int32_t)b;
    }
}

// sort each CSR segment ascending (insertion sort; segments are short)
__global__ void k_sort_segments(const int32_t *off, int32_t *idx, int64_t nb) {
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    int32_t lo = off[b], hi = off[b + 1];
    for (int32_t i = lo + 1; i < hi; ++i) {
        int32_t v = idx[i];
        int32_t j = i - 1;
        while (j >= lo && idx[j] > v) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
}

void csr_from_counts(Csr &l, DBuf<int32_t> &cnt, int64_t nb, hipStream_t s) {
    l.off.alloc(nb + 1);
    FMM_HIP(hipMemsetAsync(l.off.p + nb, 0, sizeof(int32_t), s));
    FMM_HIP(hipMemcpyAsync(l.off.p, cnt.p, nb * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    l.total = exclusive_scan_i32(l.off.p, l.off.p, nb + 1, s, true);
    l.idx.alloc(std::max<int64_t>(l.total, 1));
}

void csr_to_host(Csr &l, int64_t nb, hipStream_t s) {
    l.h_off.resize(nb + 1);
    d2h(l.h_off.data(), l.off.p, nb + 1, s);
    l.h_idx.resize(l.total);
    d2h(l.h_idx.data(), l.idx.p, l.total, s);
}

}  // namespace

bool all_finite(const float *a, int64_t n3, hipStream_t s) {
    double lo[3], hi[3];
    return bbox(a, n3 / 3, s, lo, hi);
}

// Root cube: float64 bounding box, width = max extent * (1 + 2^-20), centred.
// Each operation is rounded on its own (no contraction) so that the cube is a
// fixed function of the points.
static void derive_root(const double lo[3], const double hi[3], double x0[3], double &w) {
#pragma clang fp contract(off)
    double ext = 0.0;
    for (int c = 0; c < 3; ++c) ext = std::max(ext, hi[c] - lo[c]);
    w = ext > 0.0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
    for (int c = 0; c < 3; ++c) {
        double centre = (lo[c] + hi[c]) * 0.5;
        double hw = 0.5 * w;
        x0[c] = centre - hw;
    }
}

namespace {

// One pass over all points for a single tree (so == NULL) or a forest of
// independent instances (instance i: sources [so[i], so[i + 1]) and targets
// [to[i], to[i + 1]) of the caller's arrays). A forest's points are sorted by
// (instance, key), each instance quantised in its own root cube, and level 0
// holds one root per instance with points; the boxes of a level are then
// ordered by instance and, within one, exactly as in that instance's own
// tree, and no list links two instances.
void build_any(Tree &t, const float *src, const float *src_nrm, int64_t n_src, const float *trg,
               const float *trg_nrm, int64_t n_trg, const TreeOptions &opt, const std::vector<int64_t> *so,
               const std::vector<int64_t> *to, hipStream_t s) {
    auto clock0 = std::chrono::steady_clock::now();
    auto phase_end = [&](int k) {
        FMM_HIP(hipStreamSynchronize(s));
        const auto now = std::chrono::steady_clock::now();
        t.phase_ms[k] += std::chrono::duration<double, std::milli>(now - clock0).count();
        clock0 = now;
    };
    t.tsm = trg != nullptr;
    t.n_src = n_src;
    t.n_trg = t.tsm ? n_trg : n_src;
    t.n = t.tsm ? n_trg + n_src : n_src;
    const int64_t n = t.n;
    const bool forest = so != nullptr;
    const int ni = forest ? (int)so->size() - 1 : 1;

    // root cubes, one per instance: [5 k .. 5 k + 4] = x0, y0, z0, w, 2^21 / w
    std::vector<double> roots(5 * (size_t)ni);
    auto set_root = [&](int k, const double x0[3], double w) {
        for (int c = 0; c < 3; ++c) roots[5 * k + c] = x0[c];
        roots[5 * k + 3] = w;
        roots[5 * k + 4] = 2097152.0 / w;
    };
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double l1[3], h1[3];
        FMM_REQUIRE(bbox(src, n_src, s, l1, h1), "fmm_setup: non-finite source coordinates");
        for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], l1[c]); hi[c] = std::max(hi[c], h1[c]); }
        if (t.tsm) {
            FMM_REQUIRE(bbox(trg, n_trg, s, l1, h1), "fmm_setup: non-finite target coordinates");
            for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], l1[c]); hi[c] = std::max(hi[c], h1[c]); }
        }
        if (src_nrm) FMM_REQUIRE(all_finite(src_nrm, 3 * n_src, s), "fmm_setup: non-finite source normals");
        if (trg_nrm) FMM_REQUIRE(all_finite(trg_nrm, 3 * t.n_trg, s), "fmm_setup: non-finite target normals");
        const double unit[3] = {0.0, 0.0, 0.0};
        if (opt.root[3] > 0.0) {
            for (int k = 0; k < ni; ++k) set_root(k, opt.root, opt.root[3]);
        } else if (!forest) {
            double x0[3], w = 1.0;
            if (n == 0) {
                for (int c = 0; c < 3; ++c) x0[c] = 0.0;
            } else {
                derive_root(lo, hi, x0, w);
            }
            set_root(0, x0, w);
        } else {
            // per-instance boxes over the instance's sources and targets
            std::vector<double> bs(6 * (size_t)ni), bt(6 * (size_t)ni);
            auto inst_boxes = [&](const float *a, const std::vector<int64_t> &off, std::vector<double> &out) {
                DBuf<int64_t> doff = upload(off, s);
                DBuf<double> d(out.size());
                hipLaunchKernelGGL(k_inst_bbox, dim3(ni), dim3(kBlock), 0, s, a, doff.p, d.p);
                FMM_HIP(hipGetLastError());
                d2h(out.data(), d.p, out.size(), s);
            };
            inst_boxes(src, *so, bs);
            if (t.tsm) inst_boxes(trg, *to, bt);
            for (int k = 0; k < ni; ++k) {
                const int64_t nk = ((*so)[k + 1] - (*so)[k]) + (t.tsm ? (*to)[k + 1] - (*to)[k] : 0);
                if (nk == 0) {
                    set_root(k, unit, 1.0);
                    continue;
                }
                double l2[3], h2[3];
                for (int c = 0; c < 3; ++c) {
                    l2[c] = INFINITY;
                    h2[c] = -INFINITY;
                    if ((*so)[k + 1] > (*so)[k]) {
                        l2[c] = std::min(l2[c], bs[6 * k + c]);
                        h2[c] = std::max(h2[c], bs[6 * k + 3 + c]);
                    }
                    if (t.tsm && (*to)[k + 1] > (*to)[k]) {
                        l2[c] = std::min(l2[c], bt[6 * k + c]);
                        h2[c] = std::max(h2[c], bt[6 * k + 3 + c]);
                    }
                }
                double x0[3], w = 1.0;
                derive_root(l2, h2, x0, w);
                set_root(k, x0, w);
            }
        }
    }
    // the root reported is instance 0's
    for (int c = 0; c < 3; ++c) t.x0[c] = roots[c];
    t.w = roots[3];
    t.nlev = 0;
    t.nb = 0;
    t.lvl_off.assign(1, 0);
    if (n == 0) return;

    // keys and Morton sort (a forest: then stably by instance)
    DBuf<double> droots = upload(roots, s);
    t.keys.alloc(n);
    t.order.alloc(n);
    DBuf<int32_t> pinst, sinst;
    DBuf<int64_t> dso, dto;
    if (forest) {
        pinst.alloc(n);
        dso = upload(*so, s);
        dto = upload(*to, s);
    }
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, trg, src, n_trg, n, t.tsm, droots.p, ni,
                       dto.p, dso.p, t.keys.p, t.order.p, pinst.p);
    FMM_HIP(hipGetLastError());
    radix_sort_pairs(t.keys.p, t.order.p, n, 63, s);
    DBuf<int32_t> pbox(n);
    // level 0: one root per instance with points, over its run of sorted points
    std::vector<int64_t> b0, e0;
    if (forest) {
        std::vector<int32_t> root_of(ni, -1);
        int64_t at = 0;
        for (int k = 0; k < ni; ++k) {
            const int64_t nk = ((*so)[k + 1] - (*so)[k]) + (t.tsm ? (*to)[k + 1] - (*to)[k] : 0);
            if (nk == 0) continue;
            root_of[k] = (int32_t)b0.size();
            b0.push_back(at);
            e0.push_back(at + nk);
            at += nk;
        }
        int bits = 1;
        while ((1 << bits) < ni) ++bits;
        DBuf<uint64_t> ik(n), keys2(n);
        DBuf<int64_t> pos(n), order2(n);
        hipLaunchKernelGGL(k_inst_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, t.order.p, pinst.p, n, ik.p,
                           pos.p);
        FMM_HIP(hipGetLastError());
        radix_sort_pairs(ik.p, pos.p, n, bits, s);
        DBuf<int32_t> droot_of = upload(root_of, s);
        sinst.alloc(n);
        hipLaunchKernelGGL(k_permute_sorted, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, pos.p, t.keys.p, t.order.p,
                           ik.p, n, keys2.p, order2.p, sinst.p, pbox.p, droot_of.p);
        FMM_HIP(hipGetLastError());
        std::swap(t.keys, keys2);
        std::swap(t.order, order2);
        FMM_HIP(hipStreamSynchronize(s));  // the temporaries are freed on return from this block
    } else {
        b0 = {0};
        e0 = {n};
        FMM_HIP(hipMemsetAsync(pbox.p, 0, n * sizeof(int32_t), s));  // every point is in the root
    }
    phase_end(0);

    // level-by-level build
    DBuf<uint8_t> dl(n);
    hipLaunchKernelGGL(k_difflevel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, t.keys.p, sinst.p, n, dl.p);
    FMM_HIP(hipGetLastError());
    DBuf<int32_t> npbox(n), flag(n), cidx(n);
    std::vector<DBuf<int64_t>> lbeg, lend;
    std::vector<DBuf<int32_t>> lpar;
    {
        lbeg.push_back(upload(b0, s));
        lend.push_back(upload(e0, s));
        lpar.emplace_back(DBuf<int32_t>(b0.size()));
        FMM_HIP(hipMemsetAsync(lpar[0].p, 0xff, b0.size() * sizeof(int32_t), s));
    }
    std::vector<int64_t> counts = {(int64_t)b0.size()};
    for (int lvl = 0; lvl < kMaxLevel; ++lvl) {
        hipLaunchKernelGGL(k_split_flags, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, pbox.p, dl.p,
                           lbeg[lvl].p, lend[lvl].p, n, lvl, opt.uniform_depth, opt.leaf_size, opt.max_depth,
                           flag.p);
        FMM_HIP(hipGetLastError());
        // scan only the start bit: copy flags & 1 into cidx then scan
        FMM_HIP(hipMemcpyAsync(cidx.p, flag.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_strip_flag, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cidx.p, n);
        FMM_HIP(hipGetLastError());
        int64_t nc = exclusive_scan_i32(cidx.p, cidx.p, n, s, true);
        if (nc == 0) break;
        DBuf<int64_t> nbeg(nc), nend(nc);
        DBuf<int32_t> npar(nc);
        hipLaunchKernelGGL(k_children, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, flag.p, cidx.p, pbox.p, n,
                           nbeg.p, npar.p, npbox.p);
        FMM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_child_end, dim3(grid_for(nc, kBlock)), dim3(kBlock), 0, s, nbeg.p, npar.p,
                           lend[lvl].p, nc, nend.p);
        FMM_HIP(hipGetLastError());
        std::swap(pbox, npbox);
        lbeg.push_back(std::move(nbeg));
        lend.push_back(std::move(nend));
        lpar.push_back(std::move(npar));
        counts.push_back(nc);
    }
    t.nlev = (int)counts.size();
    t.lvl_off.assign(t.nlev + 1, 0);
    for (int l = 0; l < t.nlev; ++l) t.lvl_off[l + 1] = t.lvl_off[l] + counts[l];
    const int64_t nb = t.nb = t.lvl_off[t.nlev];

    t.level.alloc(nb);
    t.parent.alloc(nb);
    t.child.alloc(8 * nb);
    t.anchor.alloc(3 * nb);
    t.bkey.alloc(nb);
    t.begin.alloc(nb);
    t.end.alloc(nb);
    t.centre.alloc(3 * nb);
    t.half.alloc(nb);
    t.leaf.alloc(nb);
    if (forest) t.binst.alloc(nb);
    FMM_HIP(hipMemsetAsync(t.child.p, 0xff, 8 * nb * sizeof(int32_t), s));
    for (int l = 0; l < t.nlev; ++l) {
        int64_t nl = counts[l];
        hipLaunchKernelGGL(k_assemble, dim3(grid_for(nl, kBlock)), dim3(kBlock), 0, s, lbeg[l].p, lend[l].p,
                           lpar[l].p, nl, l, t.lvl_off[l], l ? t.lvl_off[l - 1] : 0, t.keys.p, sinst.p, droots.p,
                           t.level.p, t.parent.p, t.anchor.p, t.bkey.p, t.begin.p, t.end.p, t.centre.p, t.half.p,
                           t.child.p, t.binst.p);
        FMM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_leaf, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.child.p, nb, t.leaf.p);
    FMM_HIP(hipGetLastError());

    // target / source ranges and sorted point data
    t.tbeg.alloc(nb);
    t.tend.alloc(nb);
    t.sbeg.alloc(nb);
    t.send.alloc(nb);
    t.src_perm.alloc(n_src);
    t.sx.alloc(n_src);
    t.sy.alloc(n_src);
    t.sz.alloc(n_src);
    if (src_nrm) {
        t.snx.alloc(n_src);
        t.sny.alloc(n_src);
        t.snz.alloc(n_src);
    }
    if (t.tsm) {
        DBuf<int64_t> ct(n + 1), cs(n + 1);
        hipLaunchKernelGGL(k_type_flags, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, t.order.p, n, n_trg,
                           ct.p, cs.p);
        FMM_HIP(hipGetLastError());
        FMM_HIP(hipMemsetAsync(ct.p + n, 0, sizeof(int64_t), s));
        FMM_HIP(hipMemsetAsync(cs.p + n, 0, sizeof(int64_t), s));
        exclusive_scan_i64(ct.p, ct.p, n + 1, s, false);
        exclusive_scan_i64(cs.p, cs.p, n + 1, s, false);
        hipLaunchKernelGGL(k_ranges, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.begin.p, t.end.p, ct.p, cs.p,
                           nb, t.tbeg.p, t.tend.p, t.sbeg.p, t.send.p);
        FMM_HIP(hipGetLastError());
        t.trg_perm.alloc(n_trg);
        t.tx.alloc(n_trg);
        t.ty.alloc(n_trg);
        t.tz.alloc(n_trg);
        if (trg_nrm) {
            t.tnx.alloc(n_trg);
            t.tny.alloc(n_trg);
            t.tnz.alloc(n_trg);
        }
        hipLaunchKernelGGL(k_gather_points, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, t.order.p, n, n_trg,
                           true, ct.p, cs.p, trg, trg_nrm, src, src_nrm, t.trg_perm.p, t.src_perm.p, t.tx.p, t.ty.p,
                           t.tz.p, t.tnx.p, t.tny.p, t.tnz.p, t.sx.p, t.sy.p, t.sz.p, t.snx.p, t.sny.p, t.snz.p);
        FMM_HIP(hipGetLastError());
        FMM_HIP(hipStreamSynchronize(s));
    } else {
        FMM_HIP(hipMemcpyAsync(t.tbeg.p, t.begin.p, nb * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        FMM_HIP(hipMemcpyAsync(t.tend.p, t.end.p, nb * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        FMM_HIP(hipMemcpyAsync(t.sbeg.p, t.begin.p, nb * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        FMM_HIP(hipMemcpyAsync(t.send.p, t.end.p, nb * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_gather_points, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, t.order.p, n, n_trg,
                           false, (const int64_t *)nullptr, (const int64_t *)nullptr, trg, trg_nrm, src, src_nrm,
                           (int64_t *)nullptr, t.src_perm.p, (float *)nullptr, (float *)nullptr, (float *)nullptr,
                           (float *)nullptr, (float *)nullptr, (float *)nullptr, t.sx.p, t.sy.p, t.sz.p, t.snx.p,
                           t.sny.p, t.snz.p);
        FMM_HIP(hipGetLastError());
        if (trg_nrm) {
            t.tnx.alloc(n_src);
            t.tny.alloc(n_src);
            t.tnz.alloc(n_src);
            hipLaunchKernelGGL(k_copy_target_normals, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s,
                               t.src_perm.p, n, trg_nrm, t.tnx.p, t.tny.p, t.tnz.p);
            FMM_HIP(hipGetLastError());
        }
    }

    phase_end(1);

    // ---- lists
    DBuf<int64_t> d_lvl_off = upload(t.lvl_off, s);
    t.colleague.alloc(27 * nb);
    BoxView v{t.level.p, t.anchor.p,  t.child.p,  t.parent.p, t.colleague.p,
              t.leaf.p,  t.bkey.p,    d_lvl_off.p, t.nlev,    t.binst.p};
    hipLaunchKernelGGL(k_colleagues, dim3(grid_for(27 * nb, kBlock)), dim3(kBlock), 0, s, v, nb, t.colleague.p);
    FMM_HIP(hipGetLastError());
    {
        int8_t dirs[kNumDirs][3];
        int k = 0;
        for (int i = -3; i <= 3; ++i)
            for (int j = -3; j <= 3; ++j)
                for (int l = -3; l <= 3; ++l)
                    if (std::max(std::abs(i), std::max(std::abs(j), std::abs(l))) >= 2) {
                        dirs[k][0] = (int8_t)i;
                        dirs[k][1] = (int8_t)j;
                        dirs[k][2] = (int8_t)l;
                        ++k;
                    }
        FMM_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_dirs), dirs, sizeof(dirs), 0, hipMemcpyHostToDevice, s));
    }
    t.vdense.alloc((size_t)kNumDirs * nb);
    hipLaunchKernelGGL(k_vdense, dim3(grid_for(kNumDirs * nb, kBlock)), dim3(kBlock), 0, s, v, nb, t.vdense.p);
    FMM_HIP(hipGetLastError());
    {
        DBuf<int32_t> cnt(nb);
        hipLaunchKernelGGL(k_vcount, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.vdense.p, nb, cnt.p);
        FMM_HIP(hipGetLastError());
        csr_from_counts(t.V, cnt, nb, s);
        hipLaunchKernelGGL(k_vfill, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.vdense.p, nb, t.V.off.p,
                           t.V.idx.p);
        FMM_HIP(hipGetLastError());
    }
    {
        DBuf<int32_t> ucnt(nb), wcnt(nb), ovf(1);
        FMM_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_uw<false>, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, v, nb, ucnt.p, wcnt.p,
                           (const int32_t *)nullptr, (int32_t *)nullptr, (const int32_t *)nullptr,
                           (int32_t *)nullptr, ovf.p);
        FMM_HIP(hipGetLastError());
        csr_from_counts(t.U, ucnt, nb, s);
        csr_from_counts(t.W, wcnt, nb, s);
        hipLaunchKernelGGL(k_uw<true>, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, v, nb, ucnt.p, wcnt.p,
                           t.U.off.p, t.U.idx.p, t.W.off.p, t.W.idx.p, ovf.p);
        FMM_HIP(hipGetLastError());
        int32_t h_ovf = 0;
        d2h(&h_ovf, ovf.p, 1, s);
        if (h_ovf) throw Error(FMM_ERR_DEVICE, "fmm_setup: list traversal stack overflow");
        // X = inverse of W
        DBuf<int32_t> xcnt(nb), xcur(nb);
        FMM_HIP(hipMemsetAsync(xcnt.p, 0, nb * sizeof(int32_t), s));
        FMM_HIP(hipMemsetAsync(xcur.p, 0, nb * sizeof(int32_t), s));
        hipLaunchKernelGGL(k_xcount, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.W.off.p, t.W.idx.p, nb,
                           xcnt.p);
        FMM_HIP(hipGetLastError());
        csr_from_counts(t.X, xcnt, nb, s);
        hipLaunchKernelGGL(k_xfill, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, t.W.off.p, t.W.idx.p, nb,
                           t.X.off.p, xcur.p, t.X.idx.p);
        FMM_HIP(hipGetLastError());
    }
    for (Csr *l : {&t.U, &t.V, &t.W, &t.X}) {
        hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, l->off.p, l->idx.p, nb);
        FMM_HIP(hipGetLastError());
        csr_to_host(*l, nb, s);
    }

    // host copies of the box arrays
    auto cp32 = [&](std::vector<int32_t> &h, const DBuf<int32_t> &d) { h.resize(d.n); d2h(h.data(), d.p, d.n, s); };
    auto cp64 = [&](std::vector<int64_t> &h, const DBuf<int64_t> &d) { h.resize(d.n); d2h(h.data(), d.p, d.n, s); };
    cp32(t.h_level, t.level);
    cp32(t.h_parent, t.parent);
    cp32(t.h_child, t.child);
    cp32(t.h_anchor, t.anchor);
    cp64(t.h_begin, t.begin);
    cp64(t.h_end, t.end);
    cp64(t.h_tbeg, t.tbeg);
    cp64(t.h_tend, t.tend);
    cp64(t.h_sbeg, t.sbeg);
    cp64(t.h_send, t.send);
    t.h_leaf.resize(nb);
    d2h(t.h_leaf.data(), t.leaf.p, nb, s);
    t.h_centre.resize(3 * nb);
    d2h(t.h_centre.data(), t.centre.p, 3 * nb, s);
    t.h_half.resize(nb);
    d2h(t.h_half.data(), t.half.p, nb, s);
    phase_end(2);
}

}  // namespace

void build_tree(Tree &t, const float *src, const float *src_nrm, int64_t n_src, const float *trg,
                const float *trg_nrm, int64_t n_trg, const TreeOptions &opt, hipStream_t s) {
    build_any(t, src, src_nrm, n_src, trg, trg_nrm, n_trg, opt, nullptr, nullptr, s);
}

void build_forest(Tree &t, const std::vector<int64_t> &src_off, const std::vector<int64_t> &trg_off,
                  const float *src, const float *src_nrm, const float *trg, const float *trg_nrm,
                  const TreeOptions &opt, hipStream_t s) {
    FMM_REQUIRE(src_off.size() >= 2 && trg_off.size() == src_off.size(), "build_forest: bad offsets");
    const int64_t n_src = src_off.back(), n_trg = trg ? trg_off.back() : 0;
    build_any(t, src, src_nrm, n_src, trg, trg_nrm, n_trg, opt, &src_off, &trg_off, s);
}

}  // namespace fmm
