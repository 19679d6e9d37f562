// Octree over the collocation points (Section 3.9): the bounding cube is
// split recursively to level lmax, empty boxes are skipped, points are
// ordered by Morton key (bit interleaving) so that every box owns a
// contiguous point range at every level.
#pragma once

#include <vector>

#include "common.h"

namespace bfm {

constexpr int kKeyBits = 15;  // bits per axis of the point keys (levels 0..15)
constexpr int kP2PChunk = 128;   // receivers per near-field work item (two per lane)
constexpr int kLeafChunk = 128;  // points per leaf work item of P2M and L2P
constexpr int kP2PPiece = 384;   // near-field sources per work item at most (a leaf's source
                                 // list longer than this is split into balanced pieces)
// symmetric near field (one channel of monopoles): receivers per chunk (up
// to four per lane), and the positions per work item at most in the chunk's
// diagonal block and in the two-sided rest of its list
constexpr int kSymChunk = 256;  // receivers per chunk at most (four per lane)
// work item shapes (bfm_options.p2p_shape): receivers per chunk, positions
// per piece of the chunk's own block (a multiple of 64: pieces start at
// receiver-group bounds) and per piece of the rest of its list
struct SymShape {
    int chunk, dpiece, piece;
};
constexpr int kSymShapeCount = 3;
constexpr SymShape kSymShapes[kSymShapeCount] = {{256, 128, 192}, {128, 128, 128}, {256, 128, 384}};

// Translation tasks grouped by operator: tasks op_off[o]..op_off[o+1] use
// operator o; task t moves expansion src[t] into expansion dst[t] (global
// box indices). tile_off counts workgroup tiles of a given column width per
// count (see fmm.hip), prepared per channel count on demand.
struct TaskList {
    int nops = 0;
    int64_t ntasks = 0;
    std::vector<int> op_off_h;  // host copy [nops + 1]
    DevBuf<int> op_off;         // [nops + 1]
    DevBuf<int> src, dst;       // [ntasks]
    // workgroup-tile prefix per (channel count, tile width 64, 128 or 16),
    // built lazily: slot = nch * 3 + (0, 1, 2 by width)
    DevBuf<int> tile_off[24];
    int ntiles[24] = {0};
    bool tiles_ready[24] = {false};
    // M2L lists only: the tasks of each target box, for a reduction of
    // per-task results: target box dst_box0 + k owns the tasks at grouped
    // positions pos_of[dst_off[k]] .. pos_of[dst_off[k + 1] - 1] (in the
    // order they were generated)
    DevBuf<int> pos_of;   // [ntasks] generation index -> grouped position
    DevBuf<int> dst_off;  // [dst_nbox + 1]
    int64_t dst_box0 = 0, dst_nbox = 0;
    static int slot(int nch, int width) { return nch * 3 + (width == 128 ? 1 : (width == 16 ? 2 : 0)); }
    int ntiles_for(int nch, int width) const { return ntiles[slot(nch, width)]; }
    const int *tile_for(int nch, int width) const { return tile_off[slot(nch, width)].get(); }
};

struct Tree {
    bool valid = false;
    int lmax = 0;
    double origin[3] = {0, 0, 0};
    double side = 1.0;
    int64_t n = 0;       // points
    int64_t nbox = 0;    // boxes over all levels
    int64_t nleaf = 0;   // boxes at level lmax
    int64_t npairs_near = 0;
    int max_leaf = 0;
    std::vector<int64_t> lvl_off;  // host [lmax + 2]: boxes of level l are lvl_off[l]..lvl_off[l+1]

    DevBuf<uint64_t> key_a, key_b;  // point keys (sorted result in key_a)
    DevBuf<int> idx_a, idx_b;       // point permutation (sorted -> original) in idx_a
    DevBuf<int> iperm;              // original -> sorted

    DevBuf<uint64_t> box_key;   // [nbox] key at the box's own level
    DevBuf<int> box_level;      // [nbox]
    DevBuf<int> box_pt0;        // [nbox + 1] first sorted point of each box (per level, + sentinel)
    DevBuf<int> box_parent;     // [nbox]  (-1 at level 0)
    DevBuf<double> box_centre;  // [nbox][3]
    DevBuf<int> nbr;            // [nbox][27] neighbours (incl. self at slot 13), -1 if empty
    DevBuf<int> leaf_pt;        // [nleaf + 1] point ranges of leaves
    DevBuf<int> pt_leaf;        // [n] leaf index of every sorted point
    // near-field sources of every leaf as merged contiguous point ranges:
    // near_rng[leaf][k] = (start, end) for k < near_cnt[leaf] (at most 27)
    DevBuf<int2> near_rng;      // [nleaf][27]
    DevBuf<int> near_cnt;       // [nleaf]
    // leaf work items: (leaf, first point) of chunks of at most kLeafChunk
    // points, in leaf order (P2M, L2P)
    DevBuf<int2> leaf_items;
    int64_t n_leaf_items = 0;
    // near-field work items: (leaf, first receiver, s0, s1): the receivers of
    // a leaf chunk against sources s0..s1-1 of the leaf's source list (its
    // near ranges in order), in leaf (Morton) order. near_split:
    // some leaf has more than one piece (the sums are then accumulated with
    // atomics into a cleared output)
    DevBuf<int4> near_items;
    int64_t n_near_items = 0;
    bool near_split = false;
    // symmetric near-field items (leaf, r0, s0, s1): receivers [r0, r0 +
    // kSymChunk) of the leaf against positions s0..s1-1 of its near ranges
    // clipped to start at r0 (the chunk itself first), in leaf order
    DevBuf<int4> sym_items;
    int64_t n_sym_items = 0;
    int sym_shape = 0, sym_chunk = kSymChunk;  // shape the items were built with

    // sorted point data (per tree): positions, weights, normals
    DevBuf<double> px, py, pz;  // [n]
    DevBuf<double> ps, pnx, pny, pnz;

    TaskList m2l;                   // all levels 2..lmax
    std::vector<TaskList *> m2m;    // per level l = 3..lmax: child (level l) -> parent

    // build scratch, kept between builds so that a rebuild allocates nothing
    // once the sizes have been seen
    struct Scratch {
        DevBuf<unsigned long long> cnt, np;
        DevBuf<int> mo, flag, pos, tmp, icnt, ioff, lcnt, loff, iidx, iidx2, count, offs, ts, td, to, cs, cd, co, hist;
        DevBuf<int> rs_hist, rs_scanned, rs_tmp;
        DevBuf<uint64_t> ikey, ikey2;
        DevBuf<double> bbox;
        void *host = nullptr;  // pinned block the build's waits read sizes into
    } scratch;

    ~Tree() {
        for (auto *t : m2m) delete t;
        if (scratch.host) (void)hipHostFree(scratch.host);
    }
};

// Build (or rebuild) the tree for the points xyz (device, [n][3] AoS).
// lmax_req > 0 fixes the depth; otherwise the deepest level whose mean leaf
// occupancy is >= leaf_target is used (at least 2).
void build_tree(Tree &t, const double *xyz, int64_t n, int lmax_req, int leaf_target, int sym_shape,
                hipStream_t st);

// Sorted-order copies of per-vertex geometry (s, n SoA in original order).
void sort_geometry(Tree &t, const double *s, const double *nrm, hipStream_t st);

// Build the wave-tile prefix of a task list for a channel count.
void prepare_tiles(TaskList &tl, int nch, int width, hipStream_t st);

// Stable LSD radix sort of (u64 key, int value) on the low `bits` bits of the
// key; results end in (keys, vals) (the *_tmp buffers are scratch of size n).
void radix_sort(uint64_t *keys, int *vals, uint64_t *keys_tmp, int *vals_tmp, int64_t n, int bits, Tree::Scratch &scr,
                hipStream_t st);

// Device-wide exclusive scan of int32 (in place allowed), left in flight on
// the stream (no wait).
void exclusive_scan_async(const int *in, int *out, int64_t n, hipStream_t st, DevBuf<int> &tmp);

}  // namespace bfm
