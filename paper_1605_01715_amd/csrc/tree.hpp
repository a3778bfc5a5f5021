// Octree and interaction lists on the device.
#pragma once

#include <vector>

#include "common.hpp"

namespace fmm {

struct TreeOptions {
    int leaf_size = 64;
    int uniform_depth = 0;
    int max_depth = kMaxLevel;
    double root[4] = {0, 0, 0, 0};
};

// CSR list: off[n_boxes + 1], idx[off[n_boxes]].
struct Csr {
    DBuf<int32_t> off, idx;
    std::vector<int32_t> h_off, h_idx;  // host copies
    int64_t total = 0;
};

struct Tree {
    int64_t n = 0, n_trg = 0, n_src = 0;
    bool tsm = false;
    double x0[3] = {0, 0, 0}, w = 1.0;
    int nlev = 0;
    int64_t nb = 0;
    std::vector<int64_t> lvl_off;  // [nlev + 1]

    // sorted combined points
    DBuf<uint64_t> keys;
    DBuf<int64_t> order;  // combined index of the k-th sorted point

    // boxes
    DBuf<int32_t> level, parent, child;  // child: [nb][8] by octant, -1 if absent
    DBuf<int32_t> anchor;                // [nb][3]
    DBuf<uint64_t> bkey;                 // Morton prefix of the box at its level
    DBuf<int64_t> begin, end, tbeg, tend, sbeg, send;
    DBuf<uint8_t> leaf;
    DBuf<int32_t> binst;  // forest: instance of each box (empty for a single tree)
    DBuf<double> centre;  // [nb][3]
    DBuf<double> half;    // [nb]

    // host copies of the box arrays
    std::vector<int32_t> h_level, h_parent, h_child, h_anchor;
    std::vector<int64_t> h_begin, h_end, h_tbeg, h_tend, h_sbeg, h_send;
    std::vector<uint8_t> h_leaf;
    std::vector<double> h_centre, h_half;

    // lists
    DBuf<int32_t> colleague;  // [nb][27]
    DBuf<int32_t> vdense;     // [nb][316], -1 where absent
    Csr U, V, W, X;

    // sorted point data (SoA)
    DBuf<int64_t> src_perm, trg_perm;
    DBuf<float> sx, sy, sz, snx, sny, snz;
    DBuf<float> tx, ty, tz, tnx, tny, tnz;

    // host wall time of the three phases of build_tree (ms): keys and sort,
    // octree levels and sorted point data, lists and host copies
    double phase_ms[3] = {0, 0, 0};
};

// Build the tree and lists. Pointers are device [n][3] float arrays; trg may be
// NULL (targets = sources). Throws fmm::Error.
void build_tree(Tree &t, const float *src, const float *src_nrm, int64_t n_src, const float *trg,
                const float *trg_nrm, int64_t n_trg, const TreeOptions &opt, hipStream_t s);

// Forest of independent instances in one pass: instance i owns the caller's
// sources [src_off[i], src_off[i + 1]) and targets [trg_off[i], trg_off[i + 1])
// (trg NULL: targets = sources, trg_off ignored), each with its own root cube.
// The result is one tree whose boxes are ordered by level, then by instance,
// each instance's boxes, points and lists exactly those of a tree built on it
// alone (box and point indices shifted); permutations refer to the caller's
// whole arrays, and no list links two instances. The root cube reported is
// instance 0's.
void build_forest(Tree &t, const std::vector<int64_t> &src_off, const std::vector<int64_t> &trg_off,
                  const float *src, const float *src_nrm, const float *trg, const float *trg_nrm,
                  const TreeOptions &opt, hipStream_t s);

// Device check that coordinates (and normals) are finite; returns false if not.
bool all_finite(const float *a, int64_t n3, hipStream_t s);

}  // namespace fmm
