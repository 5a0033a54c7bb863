// Internal declarations shared by the host tree, the scheduler and the
// kernels of the afmg library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "afmg.h"

namespace afmg {

// Per-box topology as the kernels read it (64 bytes, one cache line).
struct BoxInfo {
    int32_t nbr[6];    // >= 0 same-level box, -1 physical, <= -2 coarse box -v-2
    int32_t bcoff[6];  // Dirichlet row of a physical side, else -1
    int32_t parent;    // parent box id, -1 for the root
    int32_t flags;     // bit 0 leaf; bits 1..3 position inside the parent (x,y,z)
    int32_t level;
    int32_t tree;      // tree of the box inside a forest (0 for a single tree)
};
static_assert(sizeof(BoxInfo) == 64, "BoxInfo must be 64 bytes");

constexpr int FLAG_LEAF = 1;
// bits 4..9: the same-level neighbour on side s is refined (a parent box)
constexpr int FLAG_NBR_REFINED = 1 << 4;
inline int oct_bit(int flags, int axis) { return (flags >> (1 + axis)) & 1; }

// Host tree, or forest of independent trees (built from leaves, immutable
// afterwards).  Boxes are ordered by level, then tree, then Morton index.
struct HostTree {
    int dim = 0, N = 0, lmin = 1, lmax = 1;
    int n_trees = 1;
    int64_t n_boxes = 0, n_leaves = 0;
    int64_t n_bfaces_leaf = 0;   // Dirichlet rows supplied by the caller
    int64_t n_bfaces_all = 0;    // plus rows derived for parent boxes
    std::vector<BoxInfo> info;
    std::vector<int32_t> ix, iy, iz;  // spatial index per box
    std::vector<int64_t> lvl_off;     // box range of level l: [lvl_off[l], lvl_off[l+1]), l = 0..lmax+1 (0 unused)
    std::vector<int32_t> leaf_box;    // box id of input leaf q
    std::vector<int32_t> child;       // [n_boxes][8] child ids (octant bits x|y<<1|z<<2), -1 if none
    bool uniform = true;              // every tree has all its leaves on one level
    int lmin_leaf = 1;                // coarsest level holding a leaf (any tree)
    std::vector<int32_t> tree_lmax;        // finest level of each tree
    std::vector<int64_t> tree_leaf_ptr;    // leaf boxes of tree t: tree_leaf_box[ptr[t] .. ptr[t+1])
    std::vector<int32_t> tree_leaf_box;
    std::vector<int32_t> bface_box, bface_side;  // per Dirichlet row (leaf rows first)
    // parent rows to derive, per level (fine to coarse order is by level)
    int64_t level_begin(int l) const { return lvl_off[l]; }
    int64_t level_count(int l) const { return lvl_off[l + 1] - lvl_off[l]; }
    int64_t n_below_lmax() const { return lvl_off[lmax]; }  // boxes at levels < lmax
};

// Builds a forest of n_trees trees; the leaves of tree t are entries
// tree_off[t] .. tree_off[t+1]-1 of level / idx.  Returns AFMG_OK or an
// error with msg filled.
int build_tree(int dim, int N, int n_trees, const int64_t *tree_off, const int32_t *level, const int32_t *idx,
               HostTree &t, std::string &msg);

// Leaves of the tree after refining the leaf boxes `ids` (paper §2.3): the
// unrefined leaves in their input order, then the 2^D children of each
// refined box (refined boxes in box order, children in octant order).
// balance 0: a coarser side neighbour of a refined box is an error; 1: such
// neighbours are refined too, recursively; 2: the same across sides, edges
// and corners.
int refine_leaves(const HostTree &t, const int32_t *ids, int64_t n, int balance, std::vector<int32_t> &level,
                  std::vector<int32_t> &idx, std::string &msg);

void set_error(const std::string &msg);

}  // namespace afmg
