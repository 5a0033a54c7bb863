// Host-side construction of a tree, or a forest of independent trees, from
// leaf lists (paper §2.1-§2.3): ancestors, completeness and 2:1 checks, Morton
// order per level (§2.3), neighbour / parent / child tables, and the
// numbering of boundary rows.  A single tree may have a coarse grid of several
// level-1 boxes on an integer lattice (§2.2) and Dirichlet, Neumann or
// periodic sides (§3); periodic axes wrap the neighbour search.
//
// Box numbering: by level over the whole forest, then by tree, then Morton
// index.  The boxes of one level of all trees form one contiguous range, the
// roots (level 1) are boxes 0 .. n_trees-1, and inside one tree the relative
// order of its boxes is the order the tree has on its own.
#include <algorithm>
#include <unordered_map>

#include "afmg_internal.h"

namespace afmg {

namespace {

struct Key {
    int tr, l, i, j, k;
    bool operator==(const Key &o) const { return tr == o.tr && l == o.l && i == o.i && j == o.j && k == o.k; }
};
struct KeyHash {
    size_t operator()(const Key &a) const {
        uint64_t x = (uint64_t)(uint32_t)a.l * 0x9E3779B97F4A7C15ULL;
        x ^= (uint64_t)(uint32_t)a.tr + 0xD6E8FEB86659FD93ULL + (x << 6) + (x >> 2);
        x ^= (uint64_t)(uint32_t)a.i + 0x632BE59BD9B4E019ULL + (x << 6) + (x >> 2);
        x ^= (uint64_t)(uint32_t)a.j + 0x8CB92BA72F3D8DD7ULL + (x << 6) + (x >> 2);
        x ^= (uint64_t)(uint32_t)a.k + 0xA24BAED4963EE407ULL + (x << 6) + (x >> 2);
        return (size_t)x;
    }
};

// Morton key of a 0-based spatial index (up to 21 bits per axis)
uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}
uint64_t spread2(uint64_t v) {
    v &= 0xffffffff;
    v = (v | v << 16) & 0x0000ffff0000ffffULL;
    v = (v | v << 8) & 0x00ff00ff00ff00ffULL;
    v = (v | v << 4) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | v << 2) & 0x3333333333333333ULL;
    v = (v | v << 1) & 0x5555555555555555ULL;
    return v;
}
uint64_t morton(int dim, int i, int j, int k) {
    if (dim == 2) return spread2((uint64_t)(i - 1)) | (spread2((uint64_t)(j - 1)) << 1);
    return spread3((uint64_t)(i - 1)) | (spread3((uint64_t)(j - 1)) << 1) |
           (spread3((uint64_t)(k - 1)) << 2);
}

}  // namespace

uint64_t box_morton(const HostTree &t, int64_t m) {
    return morton(t.dim, t.ix[(size_t)m], t.iy[(size_t)m], t.iz[(size_t)m]);
}

bool domain_position(const HostTree &t, int l, int q[3]) {
    int r[3] = {1, 1, 1};
    for (int d = 0; d < t.dim; d++) {
        const int n1 = t.ext[d] << (l - 1);
        if (q[d] < 1 || q[d] > n1) {
            if (t.bc_type[2 * d] != BC_PERIODIC) return false;
            q[d] = q[d] < 1 ? q[d] + n1 : q[d] - n1;
        }
        r[d] = ((q[d] - 1) >> (l - 1)) + 1;
    }
    return t.root_at[(size_t)((r[2] - 1) * t.ext[1] + (r[1] - 1)) * t.ext[0] + (r[0] - 1)] != 0;
}

int build_tree(int dim, int N, int n_trees, const int64_t *tree_off, const int32_t *level, const int32_t *idx,
               HostTree &t, std::string &msg, const int32_t *bc_type) {
    if (dim != 2 && dim != 3) { msg = "dim must be 2 or 3"; return AFMG_ERR_ARG; }
    if (N != 8 && N != 16) { msg = "box_n must be 8 or 16"; return AFMG_ERR_ARG; }
    if (n_trees <= 0 || !tree_off || !level || !idx) { msg = "empty or null leaf list"; return AFMG_ERR_ARG; }
    if (tree_off[0] != 0) { msg = "leaf offsets must start at 0"; return AFMG_ERR_ARG; }
    for (int tr = 0; tr < n_trees; tr++)
        if (tree_off[tr + 1] <= tree_off[tr]) { msg = "empty or null leaf list"; return AFMG_ERR_ARG; }
    const int64_t n_leaves = tree_off[n_trees];
    if (n_leaves > (int64_t)1 << 28) { msg = "too many leaves"; return AFMG_ERR_ARG; }
    const int max_level = dim == 3 ? 17 : 20;  // keeps box counts and indices in int32
    // the domain (one tree only): side types and the lattice of level-1
    // boxes; forests are trees of one level-1 box with Dirichlet sides
    for (int s = 0; s < 6; s++) t.bc_type[s] = BC_DIRICHLET;
    t.ext[0] = t.ext[1] = t.ext[2] = 1;
    if (bc_type) {
        if (n_trees != 1) { msg = "side types apply to single trees"; return AFMG_ERR_ARG; }
        for (int s = 0; s < 2 * dim; s++) {
            if (bc_type[s] < BC_DIRICHLET || bc_type[s] > BC_PERIODIC) { msg = "bad side type"; return AFMG_ERR_ARG; }
            t.bc_type[s] = bc_type[s];
        }
        for (int d = 0; d < dim; d++)
            if ((t.bc_type[2 * d] == BC_PERIODIC) != (t.bc_type[2 * d + 1] == BC_PERIODIC)) {
                msg = "periodic sides come in pairs";
                return AFMG_ERR_ARG;
            }
        for (int64_t q = 0; q < n_leaves; q++) {
            const int l = level[q];
            if (l < 1 || l > max_level) { msg = "leaf level out of range"; return AFMG_ERR_ARG; }
            for (int d = 0; d < dim; d++) {
                const int c = idx[3 * q + d];
                if (c < 1 || ((int64_t)(c - 1) >> (l - 1)) >= 64) { msg = "leaf spatial index out of range"; return AFMG_ERR_ARG; }
                t.ext[d] = std::max(t.ext[d], ((c - 1) >> (l - 1)) + 1);
            }
            if (dim == 2 && idx[3 * q + 2] != 1) { msg = "leaf spatial index out of range"; return AFMG_ERR_ARG; }
        }
        if ((int64_t)t.ext[0] * t.ext[1] * t.ext[2] > 4096) { msg = "coarse grid larger than 4096 boxes"; return AFMG_ERR_ARG; }
    }
    t.root_at.assign((size_t)t.ext[0] * t.ext[1] * t.ext[2], 0);
    struct Box { Key key; bool leaf; int64_t input; };
    std::vector<Box> boxes;
    std::unordered_map<Key, int64_t, KeyHash> map;
    boxes.reserve((size_t)(n_leaves * 8 / 7 + 16));
    map.reserve((size_t)(n_leaves * 8 / 7 + 16));
    for (int tr = 0; tr < n_trees; tr++) {
        for (int64_t q = tree_off[tr]; q < tree_off[tr + 1]; q++) {
            Key k{tr, level[q], idx[3 * q], idx[3 * q + 1], dim == 3 ? idx[3 * q + 2] : 1};
            if (k.l < 1 || k.l > max_level) { msg = "leaf level out of range"; return AFMG_ERR_ARG; }
            const int n1 = 1 << (k.l - 1);
            if (k.i < 1 || k.i > t.ext[0] * n1 || k.j < 1 || k.j > t.ext[1] * n1 || k.k < 1 ||
                k.k > (dim == 3 ? t.ext[2] * n1 : 1)) {
                msg = "leaf spatial index out of range";
                return AFMG_ERR_ARG;
            }
            // Morton keys hold 21 bits per axis in 3D
            if (dim == 3 && ((int64_t)std::max(t.ext[0], std::max(t.ext[1], t.ext[2])) << (k.l - 1)) > (1 << 21)) {
                msg = "leaf level too fine for the extent of the coarse grid";
                return AFMG_ERR_ARG;
            }
            auto ins = map.emplace(k, (int64_t)boxes.size());
            if (!ins.second) { msg = "duplicate leaf"; return AFMG_ERR_TREE; }
            boxes.push_back({k, true, q});
        }
    }
    for (int64_t q = 0; q < n_leaves; q++) {
        Key k = boxes[(size_t)q].key;
        while (k.l > 1) {
            Key p{k.tr, k.l - 1, (k.i + 1) / 2, (k.j + 1) / 2, dim == 3 ? (k.k + 1) / 2 : 1};
            auto it = map.find(p);
            if (it != map.end()) {
                if (boxes[(size_t)it->second].leaf) { msg = "a leaf overlaps finer leaves"; return AFMG_ERR_TREE; }
                break;
            }
            map.emplace(p, (int64_t)boxes.size());
            boxes.push_back({p, false, -1});
            k = p;
        }
    }
    // level-1 boxes on the lattice; periodic axes need every position
    int64_t n_roots = 0;
    for (const Box &b : boxes)
        if (b.key.l == 1) {
            // (forests: every tree's one level-1 box sits at (1, 1, 1))
            n_roots++;
            t.root_at[(size_t)((b.key.k - 1) * t.ext[1] + (b.key.j - 1)) * t.ext[0] + (b.key.i - 1)] = 1;
        }
    t.n_roots = n_trees == 1 ? (int)n_roots : 1;
    bool periodic = false;
    for (int d = 0; d < dim; d++) periodic |= t.bc_type[2 * d] == BC_PERIODIC;
    if (periodic && n_roots != (int64_t)t.ext[0] * t.ext[1] * t.ext[2]) {
        msg = "periodic sides need a rectangular coarse grid";
        return AFMG_ERR_ARG;
    }
    // every refined box has all 2^D children
    const int nch = 1 << dim;
    for (const Box &b : boxes) {
        if (b.leaf) continue;
        for (int c = 0; c < nch; c++) {
            Key ch{b.key.tr, b.key.l + 1, 2 * b.key.i - 1 + (c & 1), 2 * b.key.j - 1 + ((c >> 1) & 1),
                   dim == 3 ? 2 * b.key.k - 1 + ((c >> 2) & 1) : 1};
            if (!map.count(ch)) { msg = "leaves do not tile the domain"; return AFMG_ERR_TREE; }
        }
    }
    // order: level, tree, Morton index
    std::vector<int64_t> order(boxes.size());
    for (size_t m = 0; m < order.size(); m++) order[m] = (int64_t)m;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const Key &x = boxes[(size_t)a].key, &y = boxes[(size_t)b].key;
        if (x.l != y.l) return x.l < y.l;
        if (x.tr != y.tr) return x.tr < y.tr;
        return morton(dim, x.i, x.j, x.k) < morton(dim, y.i, y.j, y.k);
    });
    const int64_t nb = (int64_t)boxes.size();
    if (nb >= ((int64_t)1 << 30)) { msg = "too many boxes"; return AFMG_ERR_ARG; }
    std::vector<int64_t> newid(boxes.size());
    for (int64_t m = 0; m < nb; m++) newid[(size_t)order[(size_t)m]] = m;
    t.dim = dim;
    t.N = N;
    t.n_trees = n_trees;
    t.n_boxes = nb;
    t.n_leaves = n_leaves;
    int lg = 0;
    while ((1 << (lg + 1)) < N) lg++;  // N = 2^(lg+1)
    t.lmin = 1 - lg;
    t.lmax = 1;
    t.tree_lmax.assign((size_t)n_trees, 1);
    t.info.assign((size_t)nb, BoxInfo{});
    t.ix.resize((size_t)nb);
    t.iy.resize((size_t)nb);
    t.iz.resize((size_t)nb);
    for (int64_t m = 0; m < nb; m++) {
        const Box &b = boxes[(size_t)order[(size_t)m]];
        t.ix[(size_t)m] = b.key.i;
        t.iy[(size_t)m] = b.key.j;
        t.iz[(size_t)m] = b.key.k;
        BoxInfo &bi = t.info[(size_t)m];
        bi.level = b.key.l;
        bi.tree = b.key.tr;
        bi.flags = (b.leaf ? FLAG_LEAF : 0) | (((b.key.i - 1) & 1) << 1) | (((b.key.j - 1) & 1) << 2) |
                   (dim == 3 ? (((b.key.k - 1) & 1) << 3) : 0);
        if (b.key.l > t.lmax) t.lmax = b.key.l;
        if (b.key.l > t.tree_lmax[(size_t)b.key.tr]) t.tree_lmax[(size_t)b.key.tr] = b.key.l;
        for (int s = 0; s < 6; s++) { bi.nbr[s] = -1; bi.bcoff[s] = -1; }
        bi.parent = -1;
    }
    t.lvl_off.assign((size_t)t.lmax + 2, 0);
    for (int64_t m = 0; m < nb; m++) t.lvl_off[(size_t)t.info[(size_t)m].level + 1]++;
    // prefix sums: lvl_off[l] = first box of level l (level 1 starts at 0)
    t.lvl_off[0] = 0;
    for (int l = 1; l <= t.lmax + 1; l++) t.lvl_off[(size_t)l] += t.lvl_off[(size_t)l - 1];
    t.leaf_box.resize((size_t)n_leaves);
    for (int64_t m = 0; m < nb; m++) {
        const Box &b = boxes[(size_t)order[(size_t)m]];
        if (b.leaf) t.leaf_box[(size_t)b.input] = (int32_t)m;
    }
    // parents, neighbours, 2:1 balance
    for (int64_t m = 0; m < nb; m++) {
        BoxInfo &bi = t.info[(size_t)m];
        const Key key{bi.tree, bi.level, t.ix[(size_t)m], t.iy[(size_t)m], t.iz[(size_t)m]};
        if (key.l > 1) {
            Key p{key.tr, key.l - 1, (key.i + 1) / 2, (key.j + 1) / 2, dim == 3 ? (key.k + 1) / 2 : 1};
            bi.parent = (int32_t)newid[(size_t)map.at(p)];
        }
        for (int s = 0; s < 2 * dim; s++) {
            int d = s / 2, dir = (s & 1) ? 1 : -1;
            int q[3] = {key.i, key.j, key.k};
            q[d] += dir;
            // outside the lattice on a non-periodic axis, or a lattice
            // position without a level-1 box: a physical side
            if (!domain_position(t, key.l, q)) {
                bi.nbr[s] = -1;
                if (t.bc_type[s] == BC_NEUMANN) bi.flags |= FLAG_NEUMANN << s;
                continue;
            }
            auto it = map.find(Key{key.tr, key.l, q[0], q[1], q[2]});
            if (it != map.end()) { bi.nbr[s] = (int32_t)newid[(size_t)it->second]; continue; }
            int pq[3] = {(key.i + 1) / 2, (key.j + 1) / 2, dim == 3 ? (key.k + 1) / 2 : 1};
            pq[d] += dir;
            const bool inside = domain_position(t, key.l - 1, pq);
            auto itp = inside ? map.find(Key{key.tr, key.l - 1, pq[0], pq[1], pq[2]}) : map.end();
            if (itp == map.end()) { msg = "grid is not 2:1 balanced across a box side"; return AFMG_ERR_TREE; }
            bi.nbr[s] = -2 - (int32_t)newid[(size_t)itp->second];
        }
    }
    // children, refined same-level neighbours, uniformity
    t.child.assign((size_t)nb * 8, -1);
    for (int64_t m = 0; m < nb; m++) {
        const BoxInfo &bi = t.info[(size_t)m];
        if (bi.parent >= 0) {
            const int oc = ((bi.flags >> 1) & 1) | (((bi.flags >> 2) & 1) << 1) | (((bi.flags >> 3) & 1) << 2);
            t.child[(size_t)bi.parent * 8 + oc] = (int32_t)m;
        }
    }
    t.uniform = true;
    t.lmin_leaf = t.lmax;
    t.singular = true;
    for (int s = 0; s < 2 * dim; s++) t.singular &= t.bc_type[s] != BC_DIRICHLET;
    t.general = t.n_roots > 1;
    for (int s = 0; s < 2 * dim; s++) t.general |= t.bc_type[s] != BC_DIRICHLET;
    t.level1_leaf = false;
    for (int64_t m = 0; m < nb; m++) {
        BoxInfo &bi = t.info[(size_t)m];
        if ((bi.flags & FLAG_LEAF) && bi.level != t.tree_lmax[(size_t)bi.tree]) t.uniform = false;
        if ((bi.flags & FLAG_LEAF) && bi.level < t.lmin_leaf) t.lmin_leaf = bi.level;
        if ((bi.flags & FLAG_LEAF) && bi.level == 1) t.level1_leaf = true;
        for (int s = 0; s < 2 * dim; s++) {
            const int v = bi.nbr[s];
            if (v >= 0 && !(t.info[(size_t)v].flags & FLAG_LEAF)) bi.flags |= FLAG_NBR_REFINED << s;
        }
    }
    // leaf boxes of each tree, in box order (per-tree residual norms)
    t.tree_leaf_ptr.assign((size_t)n_trees + 1, 0);
    for (int64_t m = 0; m < nb; m++)
        if (t.info[(size_t)m].flags & FLAG_LEAF) t.tree_leaf_ptr[(size_t)t.info[(size_t)m].tree + 1]++;
    for (int tr = 0; tr < n_trees; tr++) t.tree_leaf_ptr[(size_t)tr + 1] += t.tree_leaf_ptr[(size_t)tr];
    t.tree_leaf_box.assign((size_t)n_leaves, 0);
    {
        std::vector<int64_t> next(t.tree_leaf_ptr.begin(), t.tree_leaf_ptr.end() - 1);
        for (int64_t m = 0; m < nb; m++)
            if (t.info[(size_t)m].flags & FLAG_LEAF)
                t.tree_leaf_box[(size_t)next[(size_t)t.info[(size_t)m].tree]++] = (int32_t)m;
    }
    // boundary rows (Dirichlet values or Neumann derivatives): leaf sides
    // first (box order, side order), then parents
    t.bface_box.clear();
    t.bface_side.clear();
    for (int pass = 0; pass < 2; pass++) {
        for (int64_t m = 0; m < nb; m++) {
            BoxInfo &bi = t.info[(size_t)m];
            bool leaf = bi.flags & FLAG_LEAF;
            if ((pass == 0) != leaf) continue;
            for (int s = 0; s < 2 * dim; s++) {
                if (bi.nbr[s] != -1) continue;
                bi.bcoff[s] = (int32_t)t.bface_box.size();
                t.bface_box.push_back((int32_t)m);
                t.bface_side.push_back(s);
            }
        }
        if (pass == 0) t.n_bfaces_leaf = (int64_t)t.bface_box.size();
    }
    t.n_bfaces_all = (int64_t)t.bface_box.size();
    return AFMG_OK;
}

namespace {

// Leaf and box lookup of a single tree by (level, i, j, k).
struct Lookup {
    const HostTree &t;
    std::unordered_map<Key, int64_t, KeyHash> leaf, box;
    explicit Lookup(const HostTree &tt) : t(tt) {
        leaf.reserve((size_t)t.n_leaves * 2);
        box.reserve((size_t)t.n_boxes * 2);
        for (int64_t m = 0; m < t.n_boxes; m++) {
            const Key k = key_of(m);
            box.emplace(k, m);
            if (t.info[(size_t)m].flags & FLAG_LEAF) leaf.emplace(k, m);
        }
    }
    Key key_of(int64_t m) const {
        return Key{0, t.info[(size_t)m].level, t.ix[(size_t)m], t.iy[(size_t)m], t.iz[(size_t)m]};
    }
    // box at (l, i, j, k) after wrapping periodic axes, or -1 (outside the
    // domain, or no box there)
    int64_t box_at(int l, int i, int j, int k) const {
        int q[3] = {i, j, t.dim == 3 ? k : 1};
        if (!domain_position(t, l, q)) return -1;
        auto it = box.find(Key{0, l, q[0], q[1], q[2]});
        return it == box.end() ? -1 : it->second;
    }
    // the leaf covering position (l, i, j, k), or -1 outside the domain
    int64_t covering(int l, int i, int j, int k) const {
        int q[3] = {i, j, t.dim == 3 ? k : 1};
        if (!domain_position(t, l, q)) return -1;
        i = q[0];
        j = q[1];
        k = q[2];
        while (l >= 1) {
            auto it = leaf.find(Key{0, l, i, j, k});
            if (it != leaf.end()) return it->second;
            l--;
            i = (i + 1) / 2;
            j = (j + 1) / 2;
            k = t.dim == 3 ? (k + 1) / 2 : 1;
        }
        return -1;
    }
};

// Coarser leaves that touch a leaf to be refined are refined too, until no
// refinement breaks 2:1 balance (balance 1: across sides; 2: also edges and
// corners).  refine[m] marks the leaf boxes to refine; `work` holds the ones
// whose neighbours are still to be checked.
int close_refinement(const Lookup &lk, std::vector<char> &refine, std::vector<int64_t> &work, int balance,
                     std::string &msg) {
    const HostTree &t = lk.t;
    const int dim = t.dim;
    while (!work.empty()) {
        const int64_t m = work.back();
        work.pop_back();
        const Key kk = lk.key_of(m);
        for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int nz = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nz == 0 || (balance < 2 && nz != 1)) continue;
                    const int64_t v = lk.covering(kk.l, kk.i + dx, kk.j + dy, kk.k + dz);
                    if (v < 0 || t.info[(size_t)v].level >= kk.l || refine[(size_t)v]) continue;
                    if (balance == 0) {
                        msg = "refinement breaks 2:1 balance with a coarser neighbour";
                        return AFMG_ERR_TREE;
                    }
                    refine[(size_t)v] = 1;
                    work.push_back(v);
                }
    }
    return AFMG_OK;
}

// the leaves of t with the boxes marked in `refine` replaced by their
// children and the children of the boxes marked in `coarsen` by their parent
void emit_leaves(const Lookup &lk, const std::vector<char> &refine, const std::vector<char> &coarsen,
                 std::vector<int32_t> &level, std::vector<int32_t> &idx) {
    const HostTree &t = lk.t;
    const int dim = t.dim;
    level.clear();
    idx.clear();
    for (int64_t q = 0; q < t.n_leaves; q++) {
        const int64_t m = t.leaf_box[(size_t)q];
        const int32_t p = t.info[(size_t)m].parent;
        if (refine[(size_t)m] || (p >= 0 && coarsen[(size_t)p])) continue;
        const Key kk = lk.key_of(m);
        level.push_back(kk.l);
        idx.insert(idx.end(), {kk.i, kk.j, kk.k});
    }
    for (int64_t m = 0; m < t.n_boxes; m++) {
        const Key kk = lk.key_of(m);
        if (coarsen[(size_t)m]) {
            level.push_back(kk.l);
            idx.insert(idx.end(), {kk.i, kk.j, kk.k});
        }
        if (!refine[(size_t)m]) continue;
        for (int c = 0; c < (1 << dim); c++) {
            level.push_back(kk.l + 1);
            idx.insert(idx.end(), {2 * kk.i - 1 + (c & 1), 2 * kk.j - 1 + ((c >> 1) & 1),
                                   dim == 3 ? 2 * kk.k - 1 + ((c >> 2) & 1) : 1});
        }
    }
}

}  // namespace

void diagonal_neighbours(const HostTree &t, std::vector<int32_t> &out) {
    const Lookup lk(t);
    out.assign((size_t)t.n_boxes * 27, -1);
    for (int64_t m = 0; m < t.n_boxes; m++) {
        const Key kk = lk.key_of(m);
        for (int o = 0; o < 27; o++) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            if (t.dim == 2 && dz != 0) continue;
            if (dx == 0 && dy == 0 && dz == 0) continue;
            out[(size_t)m * 27 + o] = (int32_t)lk.box_at(kk.l, kk.i + dx, kk.j + dy, kk.k + dz);
        }
    }
}

int refine_leaves(const HostTree &t, const int32_t *ids, int64_t n, int balance, std::vector<int32_t> &level,
                  std::vector<int32_t> &idx, std::string &msg) {
    if (n < 0 || (n > 0 && !ids)) { msg = "bad leaf id list"; return AFMG_ERR_ARG; }
    if (balance < 0 || balance > 2) { msg = "balance must be 0, 1 or 2"; return AFMG_ERR_ARG; }
    if (t.n_trees != 1) { msg = "refinement applies to single trees"; return AFMG_ERR_ARG; }
    const int max_level = t.dim == 3 ? 17 : 20;
    const Lookup lk(t);
    std::vector<char> refine((size_t)t.n_boxes, 0);
    std::vector<int64_t> work;
    for (int64_t q = 0; q < n; q++) {
        const int64_t m = ids[q];
        if (m < 0 || m >= t.n_boxes || !(t.info[(size_t)m].flags & FLAG_LEAF)) {
            msg = "refinement id is not a leaf box";
            return AFMG_ERR_ARG;
        }
        if (t.info[(size_t)m].level >= max_level) { msg = "refinement beyond the maximum level"; return AFMG_ERR_ARG; }
        if (!refine[(size_t)m]) {
            refine[(size_t)m] = 1;
            work.push_back(m);
        }
    }
    const int rc = close_refinement(lk, refine, work, balance, msg);
    if (rc != AFMG_OK) return rc;
    emit_leaves(lk, refine, std::vector<char>((size_t)t.n_boxes, 0), level, idx);
    return AFMG_OK;
}

int adapt_leaves(const HostTree &t, const int32_t *words, std::vector<int32_t> &level, std::vector<int32_t> &idx,
                 int64_t counts[2], std::string &msg) {
    if (t.n_trees != 1) { msg = "adaptation applies to single trees"; return AFMG_ERR_ARG; }
    const int dim = t.dim;
    const int max_level = dim == 3 ? 17 : 20;
    const Lookup lk(t);
    std::vector<char> refine((size_t)t.n_boxes, 0);
    std::vector<int64_t> work;
    auto mark = [&](int64_t m) {
        if (m >= 0 && !refine[(size_t)m] && (t.info[(size_t)m].flags & FLAG_LEAF) &&
            t.info[(size_t)m].level < max_level) {
            refine[(size_t)m] = 1;
            work.push_back(m);
        }
    };
    // a flagged cell refines its box, and the same-level leaves within the
    // buffer distance of it (direction bits of the box's word)
    for (int64_t q = 0; q < t.n_leaves; q++) {
        const int64_t m = t.leaf_box[(size_t)q];
        const int32_t w = words[m];
        if (!(w & ADAPT_REFINE)) continue;
        mark(m);
        const Key kk = lk.key_of(m);
        for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    if (!(w & adapt_dir_bit(dx, dy, dz))) continue;
                    const int64_t v = lk.box_at(kk.l, kk.i + dx, kk.j + dy, kk.k + dz);
                    mark(v);
                }
    }
    int rc = close_refinement(lk, refine, work, 2, msg);
    if (rc != AFMG_OK) return rc;
    // removal: parents whose children are all leaves marked for removal and
    // none to be refined, and whose neighbours' children that touch them stay
    // leaves (the parent as a leaf keeps 2:1 balance)
    std::vector<char> coarsen((size_t)t.n_boxes, 0);
    const int nch = 1 << dim;
    for (int64_t p = 0; p < t.n_boxes; p++) {
        if (t.info[(size_t)p].flags & FLAG_LEAF) continue;
        bool all = true;
        for (int c = 0; c < nch && all; c++) {
            const int32_t ch = t.child[(size_t)p * 8 + c];
            all = ch >= 0 && (t.info[(size_t)ch].flags & FLAG_LEAF) && (words[ch] & ADAPT_REMOVE) && !refine[(size_t)ch];
        }
        if (!all) continue;
        const Key kp = lk.key_of(p);
        bool ok = true;
        for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0) && ok; dz++)
            for (int dy = -1; dy <= 1 && ok; dy++)
                for (int dx = -1; dx <= 1 && ok; dx++) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    const int64_t v = lk.box_at(kp.l, kp.i + dx, kp.j + dy, kp.k + dz);
                    if (v < 0 || (t.info[(size_t)v].flags & FLAG_LEAF)) continue;
                    const int o[3] = {dx, dy, dz};
                    for (int c = 0; c < nch && ok; c++) {
                        bool touch = true;
                        for (int d = 0; d < dim; d++) {
                            const int bit = (c >> d) & 1;
                            if ((o[d] == -1 && bit != 1) || (o[d] == 1 && bit != 0)) touch = false;
                        }
                        if (!touch) continue;
                        const int32_t ch = t.child[(size_t)v * 8 + c];
                        if (ch < 0 || !(t.info[(size_t)ch].flags & FLAG_LEAF) || refine[(size_t)ch]) ok = false;
                    }
                }
        if (ok) coarsen[(size_t)p] = 1;
    }
    counts[0] = counts[1] = 0;
    for (int64_t m = 0; m < t.n_boxes; m++) {
        counts[0] += refine[(size_t)m];
        counts[1] += coarsen[(size_t)m];
    }
    emit_leaves(lk, refine, coarsen, level, idx);
    return AFMG_OK;
}

}  // namespace afmg
