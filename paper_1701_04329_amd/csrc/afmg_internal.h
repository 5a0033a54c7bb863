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
// bits 10..15: side s is a physical side of Neumann type (its boundary row
// holds the outward derivative q, ghost u1 + h q); other physical sides are
// Dirichlet (ghost 2 b - u1)
constexpr int FLAG_NEUMANN = 1 << 10;

// side types of the domain boundary, per orientation
constexpr int BC_DIRICHLET = 0, BC_NEUMANN = 1, BC_PERIODIC = 2;
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
    // domain of a single tree (paper §2.2, §3): the level-1 boxes sit on an
    // integer lattice of extent ext (a subset of it: L shapes and holes),
    // each side orientation has a type; general = more than one level-1 box
    // or a side that is not Dirichlet (such trees take the general coarse
    // path)
    int bc_type[6] = {0, 0, 0, 0, 0, 0};
    int ext[3] = {1, 1, 1};
    int n_roots = 1;                  // level-1 boxes (boxes 0 .. n_roots-1)
    bool general = false;
    bool singular = false;            // no Dirichlet side anywhere: L has the constants in its null space
    bool level1_leaf = false;         // some level-1 box is a leaf
    std::vector<char> root_at;        // [ext2][ext1][ext0]: a level-1 box sits at that lattice position
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
               HostTree &t, std::string &msg, const int32_t *bc_type = nullptr);

// Leaves of the tree after refining the leaf boxes `ids` (paper §2.3): the
// unrefined leaves in their input order, then the 2^D children of each
// refined box (refined boxes in box order, children in octant order).
// balance 0: a coarser side neighbour of a refined box is an error; 1: such
// neighbours are refined too, recursively; 2: the same across sides, edges
// and corners.
int refine_leaves(const HostTree &t, const int32_t *ids, int64_t n, int balance, std::vector<int32_t> &level,
                  std::vector<int32_t> &idx, std::string &msg);
// Mesh adaptation (paper §2.3) from one word per box (written by the flag
// kernel): ADAPT_REFINE when a cell is flagged for refinement, ADAPT_REMOVE
// when every cell is flagged for derefinement, and one bit per neighbour
// direction (dx, dy, dz in -1..1) that lies within the buffer distance of a
// refine-flagged cell.  The leaves after the adaptation: flagged leaves and
// their buffer neighbours (same-level leaves) refined, 2:1 balance across
// sides, edges and corners restored by refining coarser neighbours, and the
// children of a box removed when all are marked leaves, none is refined and
// the box as a leaf keeps 2:1 balance.  counts: boxes refined, boxes whose
// children were removed.
constexpr int ADAPT_REFINE = 1, ADAPT_REMOVE = 2;
constexpr int adapt_dir_bit(int dx, int dy, int dz) { return 1 << (2 + (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)); }
int adapt_leaves(const HostTree &t, const int32_t *words, std::vector<int32_t> &level, std::vector<int32_t> &idx,
                 int64_t counts[2], std::string &msg);
// the same-level box across every direction (dx, dy, dz) of every box of a
// single tree, index (dx+1) + 3 (dy+1) + 9 (dz+1) (periodic axes wrapped),
// -1 where there is none: [n_boxes][27]
void diagonal_neighbours(const HostTree &t, std::vector<int32_t> &out);
// Morton index of box m on its level (boxes of a level of one tree are in
// increasing Morton order; a parent's index is a child's shifted right by D)
uint64_t box_morton(const HostTree &t, int64_t m);
// the position (l, q) inside a single tree's domain (periodic axes wrapped),
// false outside it or in a lattice position without a level-1 box
bool domain_position(const HostTree &t, int l, int q[3]);

void set_error(const std::string &msg);

}  // namespace afmg
