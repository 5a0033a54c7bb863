// Launch interface between the cycle scheduler and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "afmg_internal.h"

namespace afmg {

// Arguments of a kernel over one level (a contiguous box-id range).
// Cell arrays are colour-split inside each box (see afmg_kernels.hip).
template <typename T>
struct LevelArgs {
    const BoxInfo *info;
    T *u;               // [n_boxes][N^D]
    T *rho;             // [n_boxes][N^D]: caller's rho on leaves, FAS /
                        // restricted right-hand side on parents
    T *uold;            // copy v'_H (boxes of levels < lmax)
    const T *bc;        // Dirichlet rows (leaf rows, then derived rows)
    int64_t b0;         // first box of the range
    int nb;             // number of boxes
    int homog;          // 1: zero Dirichlet values
    T h2, ih2;          // h^2 and 1/h^2 of the level
    const int *active;  // forest: per-tree flag, boxes of trees at 0 are left
                        // untouched; null: every box is processed
    int no_remap;       // 1: workgroups take boxes in launch order (no XCD remap)
    int xmask;          // complete level of one tree (every box present, box
                        // index = Morton key): the x bits of the key, else 0
    // half sweeps of a mixed-precision correction on a complete level that
    // holds every leaf of the one tree (xmask != 0), else null / 0:
    double *add_to;     // last half sweep: instead of storing the new values,
                        // add_to += u on every cell, u of the updated colour = 0
    int own_zero;       // first half sweep after one with add_to: the old
                        // values of the updated colour are taken as zero
    T h;                // cell size of the level (Neumann ghosts u1 + h q)
    // forests: the level's compacted list of boxes of trees still iterating
    // (box ids, *nact of them); the forest variants of the level kernels
    // take their boxes from it
    const int32_t *act;
    const int *nact;
    // operator of the tree (OPK_* bits, 0: the Laplacian), its cell
    // coefficients eps (colour-split like u; leaves and their restriction on
    // parents) and the x index of every box (cylindrical radius)
    const T *eps;
    const int32_t *bx;
    int opk;
    // OPK_PROLONG_LIN: [n_boxes][27] same-level box across direction
    // (dx, dy, dz), index (dx+1) + 3 (dy+1) + 9 (dz+1), -1 if none
    const int32_t *dnbr;
};

// Operators (paper §3.4, §3.5): a cell's equation is
//   (1/h^2) sum over its 2D sides of w_s (u_s - u_c) = rho_c
// with u_s the value across side s (neighbour cell or ghost) and w_s = 1 for
// the Laplacian; OPK_EPS: w_s = 2 eps_c eps_s / (eps_c + eps_s), eps_s the
// coefficient across the side; OPK_CYL: the cylindrical (r, z) form, x = r,
// the radial sides also carry r_face / r_c, and restriction is the mean over
// the parent cell's volume (children weighted by radius); OPK_PROLONG_EPS:
// eps-weighted prolongation; OPK_GHOST_BIL: bilinear-extrapolation
// refinement-boundary ghosts; OPK_PROLONG_LIN: bi/trilinear prolongation
// with edge and corner ghosts (diagonal neighbours in LevelArgs::dnbr).
constexpr int OPK_EPS = 1, OPK_CYL = 2, OPK_PROLONG_EPS = 4, OPK_GHOST_BIL = 8, OPK_PROLONG_LIN = 16;

// Per-tree stop rule of a forest, kept on the device (paper: no error
// control is built into the method, §3.2; the stop rule is the library's)
struct TreeStop {
    int cycles;   // V-cycles (or refinement steps) run
    int status;   // afmg_status of the tree
    int grow;     // consecutive cycles whose max-norm grew
    int conv;     // 1 once max |r| <= tol max |r0|
    double prev;  // max |r| of the previous cycle
    double r0;    // max |r| of the initial guess
    double rmax, rl2;  // norms after the last cycle
};

enum class Op { GSRB, RESID_RESTRICT, COARSE_RHS, PROLONG, RESTRICT_RHO };

// Modes of the coarse kernel.  Levels <= 1: V_FROM_2 (level 1 right after
// the restriction from level 2), V_TOP1 (V-cycle from level 1), FMG.
// Levels <= 2 (the 2^D boxes of level 2 as one grid; only where
// coarse_kernel_level2() holds): V2_FROM_3 (level 2 right after the
// restriction from level 3: FAS right-hand side, then the V-cycle from level
// 2), V2_TOP (V-cycle from level 2).  A tree without the levels a mode
// assumes takes the mode that fits it.
enum { COARSE_V_FROM_2 = 0, COARSE_V_TOP1 = 1, COARSE_FMG = 2, COARSE_V2_FROM_3 = 3, COARSE_V2_TOP = 4 };

// Arguments of the coarse kernel: one workgroup per tree, whose root is box
// `tree` (the roots come first in the box order).
template <typename T>
struct CoarseArgs {
    const BoxInfo *info;
    T *u;
    T *rho;
    T *uold;            // may be null when the tree has one level
    const double *bc;
    int mode;
    int homog;
    int n_down, n_up, n_base;
    const int *active;    // per-tree flag as in LevelArgs (null: all trees)
    const int32_t *child; // [n_boxes][8] child ids (modes V2_*)
    T h2_2, ih2_2;        // h^2 and 1/h^2 of level 2 (modes V2_*)
};

// Arguments of the coarse kernel of a general domain (several level-1 boxes,
// Neumann or periodic sides): one workgroup for the tree's levels <= 1; the
// level-1 boxes are boxes 0 .. n_roots-1.
template <typename T>
struct CoarseGenArgs {
    const BoxInfo *info;
    T *u;
    T *rho;
    T *uold;            // null when the tree has one level
    const double *bc;
    double *ws;         // scratch of coarse_gen_doubles(n_roots, opk) doubles
    int n_roots;
    int mode;           // COARSE_V_FROM_2, COARSE_V_TOP1 or COARSE_FMG
    int homog;
    int n_down, n_up, n_base;
    // operator (as in LevelArgs): eps of the tree's boxes (the level-1
    // boxes' values are read), x index of the boxes
    const double *eps;
    const int32_t *bx;
    int opk;
    const int32_t *dnbr;  // OPK_PROLONG_LIN: as in LevelArgs (the roots' rows)
    int in_lds;           // set by launch_coarse_gen: the grids live in LDS, not in ws
};

// Workgroup size of the kernels of a tree with an operator: 128 threads, or
// one box where a box has more rows (N^(D-1) threads per box)
constexpr int op_wg(int dim, int n) { return (dim == 3 ? n * n : n) > 128 ? (dim == 3 ? n * n : n) : 128; }

// wg: workgroup size of the launch (64, 128 or 256 threads; W / N^(D-1)
// boxes per workgroup); every size gives bitwise the same results
template <int D, int N, typename T>
void launch_level(Op op, const LevelArgs<T> &a, int colour, int wg, hipStream_t st);
template <int D, int N, typename T>
void launch_final(const LevelArgs<T> &a, double *partial, int64_t part0, double hD, float *rout, int wg,
                  hipStream_t st);
template <int D, int N>
void launch_ir_update(const BoxInfo *info, double *u, float *e, int64_t nb, const int *active,
                      hipStream_t st);
template <int D, int N>
int final_wgs(int64_t nb, int wg);
void launch_reduce(const double *partial, int64_t n, double *out, hipStream_t st);
// forests: per-tree (max, L2) of the per-box partials of each tree's leaf boxes
void launch_reduce_trees(const double *partial, const int64_t *ptr, const int32_t *boxes, const int *active,
                         double *out, int n_trees, hipStream_t st);
// out[t] = base[t] (1 if base is null) and tree_lmax[t] >= l
void launch_level_mask(const int *base, const int32_t *tree_lmax, int l, int *out, int n_trees, hipStream_t st);
// forests: per level l = 1 .. lmax, the boxes of the trees whose mask entry
// is set, into act[lvl_off[l] ..] (count nact[l]); ltoff [(lmax+2)][n+1]: first
// box of tree t on level l
void launch_compact(const int *mask, const int64_t *ltoff, const int64_t *lvl_off, int n_trees, int lmax,
                    int32_t *act, int *nact, hipStream_t st);
// forests: the stop rule after one cycle for every tree whose mask entry is
// set (norm: (max, L2) per tree; hist [n][2][AFMG_HIST]); a tree that stops
// leaves the mask
void launch_tree_stop(const double *norm, int *mask, TreeStop *state, double *hist, int n_trees, double tol,
                      int fixed, int nmax, hipStream_t st);
// the one-tree coarse kernel holds levels <= 1 in LDS, and level 2 as well
// where that fits a workgroup's LDS (all but 3D boxes of 16^3 cells); where
// it does not, level 2 runs box by box and the kernel starts at level 1
bool coarse_kernel_level2(int dim, int box_n);
template <int D, int N, typename T>
void launch_coarse(const CoarseArgs<T> &a, int n_trees, hipStream_t st);
template <int D, int N, typename T>
void launch_coarse_gen(const CoarseGenArgs<T> &a, hipStream_t st);
template <int D, int N>
size_t coarse_gen_doubles(int n_roots, int opk);
template <int D, int N, typename T>
void launch_permute(const BoxInfo *info, T *f, int64_t b0, int64_t nb, int to_split, int leaves_only,
                    hipStream_t st);
// caller's boxes (natural order; box map[b], or b if map is null) -> working
// boxes (colour-split); leaves_only skips parents
template <int D, int N, typename T>
void launch_load_rho(const BoxInfo *info, const int32_t *map, const T *src, T *dst, int64_t nb, int leaves_only,
                     hipStream_t st);
// working box b -> caller's box map[b]
template <int D, int N, typename T>
void launch_store_boxes(const int32_t *map, const T *src, T *dst, int64_t nb, hipStream_t st);
// dst row r (F values) <- src row map[r]
void launch_gather_rows(const int32_t *map, const double *src, double *dst, int64_t n_rows, int F, hipStream_t st);
template <int D, int N>
void launch_bc_derive(const BoxInfo *info, int64_t b0, int64_t nb, double *bc, hipStream_t st);
// adjoint support (FP64)
constexpr int DOT_WGS = 1024;  // fixed grid of k_dot: deterministic sums
template <int D, int N>
void launch_apply_lt(const BoxInfo *info, const int *child, const double *y, double *out, int64_t nb,
                     hipStream_t st);
template <int D, int N>
void launch_apply_l(const BoxInfo *info, const double *x, double *out, int64_t nb, hipStream_t st);
template <int D, int N>
void launch_restrict_field(const BoxInfo *info, double *f, int64_t b0, int64_t nb, hipStream_t st);
// the same with the operator's restriction (opk: OPK_CYL weights by volume)
template <int D, int N>
void launch_restrict_field_op(const BoxInfo *info, double *f, int64_t b0, int64_t nb, int opk, const int32_t *bx,
                              double h, hipStream_t st);
// *flag |= 1 if a cell of a leaf box among the nb boxes from b0 is not
// positive and finite
template <int D, int N>
void launch_check_positive(const BoxInfo *info, const double *f, int64_t nb, int *flag, hipStream_t st);
// mesh adaptation: one word per box from the int8 cell flags (see adapt_leaves)
template <int D, int N>
void launch_box_flags(const BoxInfo *info, const int8_t *flags, int64_t nb, int n_buf, int32_t *words,
                      hipStream_t st);
// field transfer between trees (colour-split arrays): whole boxes copied
// (copy_dst[q] <- copy_src[q]) and new boxes prolonged from their parent in
// the from-tree (pro_dst[q] <- P(pro_src[q]), ghosts from bc unless homog)
template <int D, int N>
void launch_transfer(const BoxInfo *to_info, const BoxInfo *from_info, const int32_t *copy_dst,
                     const int32_t *copy_src, int64_t n_copy, const int32_t *pro_dst, const int32_t *pro_src,
                     int64_t n_pro, const double *from, const double *bc, int homog, double *to, hipStream_t st);
template <int D, int N>
void launch_push_down(const BoxInfo *info, double *f, int64_t b0, int64_t nb, hipStream_t st);
template <int D, int N>
void launch_scale_leaves(const BoxInfo *info, double *dst, const double *src, int pw, int64_t nb, hipStream_t st);
template <int D, int N>
void launch_store_leaves(const BoxInfo *info, const double *src, double *dst, int64_t nb, hipStream_t st);
template <int D, int N>
void launch_bc_grad(const BoxInfo *info, const double *lam, double *bc_bar, int64_t nb, hipStream_t st);
// out[0] = max |a|, out[1] = sum a b (partial: DOT_WGS pairs)
void launch_dot(const double *a, const double *b, int64_t n, double *partial, double *out, hipStream_t st);
void launch_lc3(double *out, double a, const double *x, double b, const double *y, double c, const double *z,
                int64_t n, hipStream_t st);
template <typename T>
void launch_copy(const T *src, T *dst, int64_t n, hipStream_t st);
template <typename T>
void launch_fill(T *dst, int64_t n, T v, hipStream_t st);

}  // namespace afmg
