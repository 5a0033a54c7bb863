/*
 * afmg — FAS geometric multigrid for Poisson's equation on quadtree (2D) and
 * octree (3D) box grids, on one AMD MI355X (gfx950).
 *
 * The method is the one of Teunissen & Ebert, "Afivo: a framework for
 * quadtree/octree AMR with shared-memory parallelization and geometric
 * multigrid methods" (Comput. Phys. Commun.), sections 2 and 3:
 *   - grid of boxes of N^D cells, one root box covering [0,1]^D at level 1,
 *     children of box (i,j[,k]) at (2i-1..2i, ...) one level finer (§2.1);
 *   - Gauss-Seidel red-black smoothing (§3.1), FAS V-cycle and FMG cycle with
 *     averaging restriction and 2-1-1 prolongation (§2.5, §3.2, eqs.
 *     residual, coarse-rhs, coarse-corr);
 *   - side ghost cells: copy from a same-level neighbour, Dirichlet values
 *     through g = 2 b - u1, and the default conservative scheme at refinement
 *     boundaries (§2.4, §3.3);
 *   - extra coarse grids of N/2, ..., 2 cells below the root (§3.2);
 *   - general domains (afmg_tree_create_domain): a coarse grid of several
 *     level-1 boxes (§2.2) and Dirichlet, Neumann or periodic sides (§3).
 * The operator is the 5-point (2D) / 7-point (3D) Laplacian: the library
 * solves lap_h(u) = rho with the given boundary values.
 *
 * Conventions
 *   - All entry points return an afmg_status; nothing is thrown or exits.
 *     afmg_last_error() returns a thread-local message for the last failure.
 *   - Box ids: after afmg_tree_create the library numbers boxes level by
 *     level (level 1 first) and in Morton order within a level.
 *     afmg_tree_leaf_boxes maps the caller's leaf order to box ids.
 *   - Cell fields are device arrays of doubles laid out [n_boxes][N^D] in
 *     box-id order, x fastest within a box, no ghost cells.
 *   - Boundary values are a device array [n_bfaces][N^(D-1)]: one row per
 *     physical-boundary side of a LEAF box, rows ordered as
 *     afmg_tree_bfaces lists them; within a row the tangential axes are
 *     taken in increasing order, the first fastest; values sit at the face
 *     centres: the solution on Dirichlet sides, its outward normal
 *     derivative on Neumann sides (afmg_tree_create_domain).  Values for
 *     coarser boxes are derived by averaging.
 *   - Every device operation is enqueued on the caller's HIP stream.
 *   - A tree may be used by one stream at a time.
 */
#ifndef AFMG_H
#define AFMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afmg_tree afmg_tree;
typedef struct afmg_batch afmg_batch;

typedef enum {
    AFMG_OK = 0,
    AFMG_NOT_CONVERGED = 1,  /* max_cycles reached before tol; stats filled */
    AFMG_ERR_ARG = -1,       /* bad argument (null, misaligned, size, range) */
    AFMG_ERR_TREE = -2,      /* leaves overlap, leave gaps, or break 2:1 balance */
    AFMG_ERR_HIP = -3,       /* a HIP call or kernel failed */
    AFMG_ERR_OOM = -4,       /* host or device allocation failed */
    AFMG_ERR_NONFINITE = -5, /* a residual norm became NaN or Inf */
    AFMG_ERR_DIVERGED = -6   /* residual grew for 3 consecutive cycles */
} afmg_status;

typedef enum { AFMG_CYCLE_V = 0, AFMG_CYCLE_FMG_V = 1 } afmg_cycle;
typedef enum { AFMG_FP64 = 0, AFMG_MIXED = 1 } afmg_precision;

#define AFMG_HIST 128

typedef struct {
    int cycle;        /* AFMG_CYCLE_V: V-cycles from the initial guess;
                         AFMG_CYCLE_FMG_V: one FMG cycle from zero, then V-cycles */
    int n_down;       /* smoothing steps before restriction (paper default 2) */
    int n_up;         /* smoothing steps after correction (default 2) */
    int n_base;       /* relaxation steps on the coarsest grid (default 4) */
    double tol;       /* stop when max|r| <= tol * max|r0| (default 1e-10);
                         r0 is the composite residual of u = 0 */
    int max_cycles;   /* cap on V-cycles (default 100) */
    int fixed_cycles; /* > 0: run exactly this many V-cycles, no stop test */
    int use_guess;    /* 1: u holds the initial guess on leaf boxes (V only) */
    int precision;    /* AFMG_FP64 (default) or AFMG_MIXED */
    int profile;      /* 1: time the finest-level kernels with HIP events
                         (stats.prof_*); one event pair per launch, or per
                         group of consecutive half sweeps */
    int graph;        /* 1: record the repeated cycle (V-cycle, refinement
                         update, residual) once as a HIP graph and replay it;
                         ignored while profiling.  Results are identical. */
    int check_every;  /* read the residual norms (one stream synchronisation)
                         and apply the stop test every check_every cycles
                         (default 1; 0 is taken as 1).  The composite
                         residual of the FP64 path is then only computed at
                         those cycles; a solve may run up to check_every - 1
                         cycles past convergence; stats history entries of
                         the unchecked cycles are NaN.  Batches apply every
                         tree's stop test on the device after every cycle,
                         so results and histories do not depend on
                         check_every, which only sets the cycles between
                         host synchronisations (one recorded graph replay
                         each with opts.graph). */
    int prof_level;   /* level whose launches opts.profile times (2 .. lmax;
                         0: the finest level, the default) */
} afmg_opts;

/* kernel classes timed when opts.profile is set (on level opts.prof_level,
   by default the finest; levels <= 2 run inside the coarse kernel and are
   not timed) */
enum {
    AFMG_PROF_GSRB = 0,      /* one red or black half sweep (in the mixed
                                path of a tree whose leaves all lie on its
                                complete finest level, not the last one of
                                each correction, which also adds the
                                correction to u and is not timed) */
    AFMG_PROF_RESID = 1,     /* residual + restriction */
    AFMG_PROF_PROLONG = 2,   /* prolongation + correction */
    AFMG_PROF_FINAL = 3,     /* restriction of u + composite leaf residual */
    AFMG_PROF_KINDS = 4
};

typedef struct {
    int status;       /* final afmg_status of the solve */
    int cycles;       /* V-cycles run (the FMG cycle is not counted) */
    double r0_max, r0_l2;  /* residual norms of the initial guess (u = 0
                              unless opts.use_guess) */
    double r_max, r_l2;    /* residual norms on return */
    double hist_max[AFMG_HIST]; /* max|r| after each V-cycle */
    double hist_l2[AFMG_HIST];  /* sqrt(sum r^2 h^D) after each V-cycle */
    double t_ms;      /* device time from first kernel to last norm */
    double prof_ms[AFMG_PROF_KINDS]; /* summed kernel time per class */
    int prof_n[AFMG_PROF_KINDS];     /* launches per class */
    double bytes_model;  /* algorithmic HBM bytes of the solve (afmg_solve_bytes_model
                            with the cycles run); FP64 solves of one tree with
                            the Laplacian, else 0 */
} afmg_stats;

typedef struct {
    int dim, box_n;
    int64_t n_boxes, n_leaves, n_bfaces;
    int lmin, lmax;   /* lmin < 1: coarse grids below the root */
    int64_t cells_per_box;
    int64_t n_unknowns;  /* leaf cells */
    int n_roots;      /* level-1 boxes (boxes 0 .. n_roots-1) */
    int ext[3];       /* extent of their lattice per axis (1 for unused axes) */
    int bc_type[6];   /* afmg_bc_type per side orientation */
    int singular;     /* 1: no Dirichlet side; solutions are defined up to a
                         constant and rho must be compatible */
    int op;           /* afmg_operator set by afmg_tree_set_operator */
    int prolong;      /* afmg_prolong set by afmg_tree_set_operator */
    int ghost;        /* afmg_ghost set by afmg_tree_set_ghost_scheme */
} afmg_tree_desc;

/* Side types of the domain boundary (paper §3), per orientation -x, +x, -y,
   +y, -z, +z.  Dirichlet rows hold the value b at the face centre (ghost
   2 b - u1); Neumann rows the outward normal derivative q (ghost u1 + h q);
   periodic sides have no rows (the neighbour across is the box at the other
   end of the axis). */
typedef enum { AFMG_BC_DIRICHLET = 0, AFMG_BC_NEUMANN = 1, AFMG_BC_PERIODIC = 2 } afmg_bc_type;

typedef struct {
    int level;
    int idx[3];       /* 1-based spatial index (idx[2] = 1 in 2D) */
    int parent;       /* box id, -1 for the root */
    int leaf;
    int nbr[6];       /* per side (-x,+x,-y,+y,-z,+z): >= 0 same-level box,
                         -1 physical boundary, <= -2 refinement boundary with
                         the coarser leaf box -nbr-2 */
    int children[8];  /* box ids of the 2^D children, octant bits x | y<<1 |
                         z<<2; -1 for a leaf (entries >= 2^D unused) */
    double x_lo[3];   /* lower corner of the box (x_lo[2] = 0 in 2D) */
    double h;         /* cell size of the box's level, 1 / (N 2^(level-1)) */
} afmg_box_desc;

/* Fill opts with the paper's defaults (V(2,2), N_base = 4, tol 1e-10,
   100 cycles, FP64). */
void afmg_default_opts(afmg_opts *opts);

/*
 * Build a tree from its leaves (paper §2.1-§2.3).  level[i] >= 1 and the
 * 1-based spatial index idx[3*i .. 3*i+2] (third entry ignored in 2D) name
 * leaf i.  The leaves must tile [0,1]^D exactly and neighbouring leaves
 * (across a side) may differ by at most one level.  Host-only: no device
 * work happens here.  dim in {2,3}; box_n, the cells per box side (§2.1:
 * an even parameter of the grid), is 8 or 16.  Below level 1 the solve adds
 * coarse grids of N/2, ..., 2 cells per side (§3.2: two levels for N = 8,
 * three for N = 16).  On success *out owns the tree (free with
 * afmg_tree_destroy).  Errors: AFMG_ERR_ARG, AFMG_ERR_TREE, AFMG_ERR_OOM.
 */
int afmg_tree_create(int dim, int box_n, int64_t n_leaves, const int32_t *level,
                     const int32_t *idx, afmg_tree **out);

/*
 * A tree on a general domain (paper §2.2, §3).  The coarse grid is the set
 * of level-1 boxes that hold the leaves: unit boxes at 1-based lattice
 * positions 1 .. ext[d] per axis (ext[d] <= 64, at most 4096 positions),
 * which may leave positions out (L shapes, holes); the leaves tile their
 * union.  Below every level-1 box the solve adds coarse grids of N/2, ...,
 * 2 cells, linked like the level-1 boxes, so a non-square coarse grid has
 * several 2^D-cell boxes at the bottom and may need a larger opts.n_base
 * (§3.2).  bc_type[2 * dim] gives the type of each side orientation
 * (afmg_bc_type; NULL: all Dirichlet); faces of holes take the type of
 * their orientation; periodic sides come in pairs and need every lattice
 * position filled.  Neighbour searches wrap on periodic axes, 2:1 balance
 * included.  Without a Dirichlet side the problem is singular: rho must be
 * compatible (its volume integral equals the boundary integral of the
 * Neumann derivatives), the solution is defined up to a constant, and
 * afmg_adjoint refuses the tree.  Trees made here are not accepted by
 * afmg_batch_create unless they have one level-1 box and Dirichlet sides.
 * Host-only.  Errors: AFMG_ERR_ARG (bad types, unpaired periodic sides,
 * periodic sides on a non-rectangular coarse grid, indices out of range),
 * AFMG_ERR_TREE, AFMG_ERR_OOM.
 */
int afmg_tree_create_domain(int dim, int box_n, const int32_t *bc_type, int64_t n_leaves,
                            const int32_t *level, const int32_t *idx, afmg_tree **out);

void afmg_tree_destroy(afmg_tree *tree);

/*
 * Refinement (paper §2.3): a new tree whose leaves are those of `tree` with
 * the leaf boxes box_ids[0..n) replaced by their 2^D children.  balance:
 *   0  a refined box whose side neighbour is a coarser leaf (not refined in
 *      the same call) is an error (AFMG_ERR_TREE: 2:1 balance would break);
 *   1  such coarser side neighbours are refined too, recursively (the
 *      paper's rule);
 *   2  the same for neighbours across sides, edges and corners.
 * Leaf order of the new tree: the unrefined leaves in their input order, then
 * the children of each refined box (refined boxes in box-id order, children in
 * octant order x | y<<1 | z<<2).  `tree` is unchanged; *out is owned by the
 * caller.  Host-only.  Errors: AFMG_ERR_ARG (ids that are not leaf boxes,
 * refinement past the maximum level), AFMG_ERR_TREE, AFMG_ERR_OOM.
 */
int afmg_tree_refine(const afmg_tree *tree, const int32_t *box_ids, int64_t n, int balance, afmg_tree **out);

/* Upload the tree's device tables (box records, children) to the current
   device now rather than at its first solve.  Trees are immutable, so this
   is the only preparation a tree needs.  Errors: AFMG_ERR_ARG (another
   device than the first use), AFMG_ERR_OOM, AFMG_ERR_HIP. */
int afmg_tree_finalize(afmg_tree *tree, void *stream);

/*
 * Elliptic operator of the tree's later solves and steps (paper §3.4, §3.5;
 * the default is the Laplacian).  Each cell's equation is
 *   (1/h^2) sum over its 2D sides s of w_s (u_s - u_c) = rho_c
 * with u_s the value across the side (neighbour cell or ghost, as for the
 * Laplacian) and the face weight w_s:
 *   AFMG_OPERATOR_EPS   div(eps grad u) with eps per cell: w_s is the
 *                       harmonic mean 2 eps_c eps_s / (eps_c + eps_s) of the
 *                       cell's eps and the eps across the side (the
 *                       neighbour cell; the cell's own on a physical side;
 *                       the coarse cell holding the ghost centre on a
 *                       refinement side).  The paper's setting is a jump on
 *                       a coarse-grid cell face (§3.4); any positive eps is
 *                       accepted.
 *   AFMG_OPERATOR_CYL   cylindrical (r, z) coordinates, 2D only, x = r >= 0
 *                       (the domain starts on the axis): the radial sides
 *                       carry r_face / r_c as well, the face on the axis has
 *                       weight 0; restriction is the mean over the parent
 *                       cell's volume (children weighted by radius).
 *   AFMG_OPERATOR_CYL_EPS both (the paper's §4.1 case 2).
 * prolong: AFMG_PROLONG_DEFAULT (the 2-1-1 interpolation of §2.5),
 * AFMG_PROLONG_EPS (needs eps): per axis the fine cell moves from its coarse
 * cell P towards P + s e_d by eps_d / (2 (eps_P + eps_d)) of the difference,
 * the piecewise-linear profile with continuous value and flux eps du/dn
 * (the local reconstruction of §3.4; with equal eps the default weights),
 * or AFMG_PROLONG_LINEAR: bilinear (3D: trilinear) interpolation from the
 * 2^D nearest coarse cells (§2.5), whose edge and corner ghosts are copied
 * from the same-level box across that edge or corner or else extrapolated
 * linearly, b + c - a (§2.4; a 3D corner: its three edge ghosts minus its
 * three side ghosts plus the inner cell).  Any operator, the Laplacian
 * included, takes any prolongation but AFMG_PROLONG_EPS (eps needed).
 *   eps     device, [n_boxes][N^D] FP64 in the layout of rho (x fastest;
 *           only leaf boxes are read), positive and finite; NULL unless the
 *           operator has eps.  Copied: the caller may free it on return.
 * Parents receive the (volume) means of their children's eps.  The tree
 * keeps the coefficients in device memory of its own (allocated here,
 * released with the tree).  The solve then takes the general coarse path
 * (afmg_workspace_bytes grows: query it after this call) and FP64 only.
 * Synchronises the stream.  Errors: AFMG_ERR_ARG (a batch, a bad operator
 * or prolongation, the cylindrical form in 3D, eps missing, misaligned, not
 * positive or not finite), AFMG_ERR_OOM, AFMG_ERR_HIP.  With an operator
 * set, afmg_apply, afmg_adjoint, the autotuner, launch shapes other than the
 * default and afmg_batch_create reject the tree (AFMG_ERR_ARG);
 * afmg_tree_refine returns a tree with the Laplacian.  Setting
 * AFMG_OPERATOR_LAPLACIAN with AFMG_PROLONG_DEFAULT restores the default.
 */
/*
 * Mesh adaptation (paper §2.3): a new tree from per-cell flags on the leaves.
 *   flags   device int8 [n_boxes][N^D] in the layout of rho (x fastest; only
 *           leaf boxes are read): > 0 refine, < 0 derefine, 0 keep
 *   n_buf   buffer distance in cells (0 .. box_n; the paper's default is 2)
 *   counts  host int64[2] or NULL: boxes refined, boxes whose children were
 *           removed
 * Rules: a leaf with a refine-flagged cell is refined, and so is every
 * same-level leaf neighbour (across sides, edges or corners) that such a
 * cell lies within n_buf cells of; coarser leaves that touch a refined box
 * are refined as well until 2:1 balance holds across sides, edges and
 * corners; the 2^D children of a box are removed when all are leaves whose
 * cells are all flagged for derefinement, none of them is refined, and the
 * box as a leaf keeps 2:1 balance.  The grid changes by at most one level;
 * boxes at the deepest level (17 in 3D, 20 in 2D) are not refined.  The new
 * tree has the same domain and side types and the Laplacian (its boxes are
 * ordered by level and Morton index as every tree's); free it with
 * afmg_tree_destroy.  The flags are reduced on the device (one word per
 * box), the rules run on the host.  Allocates (a device word per box, the
 * new tree) and synchronises the stream.  Errors: AFMG_ERR_ARG (null, a
 * batch, n_buf out of range), AFMG_ERR_OOM, AFMG_ERR_HIP.
 */
int afmg_tree_adapt(afmg_tree *tree, void *stream, const int8_t *flags, int n_buf, afmg_tree **out,
                    int64_t *counts);

/*
 * Transfer of a cell field from tree `from` to tree `to` (paper §2.3: the
 * prolongation and restriction of §2.5 applied when the mesh changes).  The
 * trees share the domain, and every leaf of `to` is a box of `from` or a
 * child of a leaf of `from` (afmg_tree_adapt's result, or
 * afmg_tree_refine's, satisfies this).
 *   u_from   device [n_boxes(from)][N^D], layout of rho; leaf boxes read
 *   bc_from  device Dirichlet / Neumann rows of `from` (as for afmg_solve),
 *            or NULL for zero values: they enter the ghosts of prolongation
 *   u_to     device [n_boxes(to)][N^D] out: on every leaf of `to`, the value
 *            of the same box in `from` (a leaf there, or a box whose children
 *            were removed: the mean of its children), or for a new box the
 *            default prolongation from its parent in `from` with the side
 *            ghosts of the solve; parents receive the means of their children
 *   workspace  device, >= afmg_transfer_workspace_bytes(from, to), 256-byte
 *            aligned
 * Synchronises the stream.  Errors: AFMG_ERR_ARG (null, misaligned, trees of
 * different domains, a leaf of `to` two or more levels below the leaves of
 * `from`), AFMG_ERR_HIP.
 */
int afmg_transfer_workspace_bytes(const afmg_tree *from, const afmg_tree *to, size_t *bytes);
int afmg_tree_transfer(afmg_tree *from, afmg_tree *to, void *stream, const double *u_from, const double *bc_from,
                       double *u_to, void *workspace, size_t workspace_bytes);

typedef enum {
    AFMG_OPERATOR_LAPLACIAN = 0,
    AFMG_OPERATOR_EPS = 1,
    AFMG_OPERATOR_CYL = 2,
    AFMG_OPERATOR_CYL_EPS = 3
} afmg_operator;
typedef enum { AFMG_PROLONG_DEFAULT = 0, AFMG_PROLONG_EPS = 1, AFMG_PROLONG_LINEAR = 2 } afmg_prolong;
int afmg_tree_set_operator(afmg_tree *tree, void *stream, int op, const double *eps, int prolong);

/*
 * Refinement-boundary ghost scheme of the tree's later solves and steps
 * (paper §3.3): AFMG_GHOST_DEFAULT, from the two closest fine values
 * (2D 1/2 u_H + u1 - 1/4 (u1p + u2), 3D 1/2 u_H + 5/4 u1 - 1/4 (u2 + u1p +
 * u1q)), or AFMG_GHOST_BILINEAR, bilinear extrapolation (2D 1/2 u_H +
 * 9/8 u1 - 3/8 (u1p + u2) + 1/8 u2p), whose 3D form extends the
 * construction by the second tangential axis: 1/2 u_H + 27/16 u1
 * - 9/16 (u2 + u1p + u1q) + 3/16 (u2p + u2q + u1pq) - 1/16 u2pq.  Here u1 is
 * the face cell, u2 the next inward, and p, q, pq mark the partner inside
 * the same coarse cell along the first, the second and both tangential
 * axes.  Both keep the coarse flux across a refinement boundary equal to
 * the mean of the fine fluxes.  A tree with a scheme other than the
 * default takes the operator kernels (as afmg_tree_set_operator: general
 * coarse path, FP64, default launch shapes; the adjoint, afmg_apply, the
 * autotuner and batches reject it).  afmg_tree_transfer keeps the default
 * scheme.  Errors: AFMG_ERR_ARG (null, a batch, a bad scheme), AFMG_ERR_HIP.
 */
typedef enum { AFMG_GHOST_DEFAULT = 0, AFMG_GHOST_BILINEAR = 1 } afmg_ghost;
int afmg_tree_set_ghost_scheme(afmg_tree *tree, void *stream, int scheme);

/* Box lists per level (paper §2.1): all boxes, parents (refined boxes) or
   leaves of `level` (1 .. lmax), in box-id order, which is Morton order
   within a level.  *n receives the count; ids (host array of at least that
   many entries, or NULL to query the count first) receives the ids. */
typedef enum { AFMG_LIST_ALL = 0, AFMG_LIST_PARENT = 1, AFMG_LIST_LEAF = 2 } afmg_list_kind;
int afmg_tree_level_list(const afmg_tree *tree, int level, int kind, int32_t *ids, int64_t *n);

/* Sizes of the tree (paper §2.1: boxes of N^D cells on levels 1 .. lmax,
   §3.2: coarse grids below level 1 down to lmin): dim, N, box, leaf and
   Dirichlet-row counts, level range, unknowns (leaf cells).  Host-only.
   Errors: AFMG_ERR_ARG (null). */
int afmg_tree_info(const afmg_tree *tree, afmg_tree_desc *out);

/* box id of each input leaf: out[n_leaves] (host array) */
int afmg_tree_leaf_boxes(const afmg_tree *tree, int32_t *out);

/* (box id, side) of each Dirichlet row: out[2*n_bfaces] (host array) */
int afmg_tree_bfaces(const afmg_tree *tree, int32_t *out);

/* The record of one box (paper §2.1: refinement level, spatial index,
   parent, children and side neighbours, with the neighbour codes of
   afmg_box_desc; origin and cell size from the level).  box in
   [0, n_boxes).  Host-only.  Errors: AFMG_ERR_ARG (null, box out of
   range). */
int afmg_tree_box(const afmg_tree *tree, int64_t box, afmg_box_desc *out);

/* Device workspace bytes afmg_solve needs for these options. */
int afmg_workspace_bytes(const afmg_tree *tree, const afmg_opts *opts, size_t *bytes);

/* Algorithmic HBM bytes of an FP64 solve of this tree with the Laplacian
   (paper §3.2's cycle): every array a kernel of the solve reads or writes,
   counted once per launch over the scheduler's launch sequence, with
   v_cycles V-cycles after the FMG cycle (opts->cycle FMG) or from the
   initial guess.  Per cell of a level (s = 8 B, D the dimension): half sweep
   1.5 s; residual + restriction 2 s + 2 s / 2^D; FAS right-hand side + copy
   4 s (parents' level); prolongation + correction 2 s + 2 s / 2^D; the
   end-of-cycle pass 2 s + s / 2^D on leaves, s + s / 2^D on parents; the
   coarse kernel 4 s per cell of the coarsest level it loads (2, or 1 where
   level 2 runs box by box); layout conversions 2 s and fills s; the ghosts
   read from neighbouring boxes are not counted.  stats.bytes_model reports it
   for the solve's cycle count.  Host-only.  Errors: AFMG_ERR_ARG (null, a
   tree with an operator or a batch's forest, v_cycles < 0). */
int afmg_solve_bytes_model(const afmg_tree *tree, const afmg_opts *opts, int v_cycles, double *bytes);

/*
 * Solve lap_h(u) = rho (paper §3, eq. mg-discr-equation) on the tree.
 *   stream     hipStream_t to enqueue on (NULL = default stream)
 *   rho        device [n_boxes][N^D]; only leaf boxes are read
 *   bc         device [n_bfaces][N^(D-1)] Dirichlet values, or NULL for zero
 *   u          device [n_boxes][N^D]; in: initial guess on leaf boxes if
 *              opts->use_guess, out: solution on leaf boxes and its
 *              restriction on parent boxes
 *   workspace  device, >= afmg_workspace_bytes, 256-byte aligned; the
 *              caller owns it; contents are scratch
 * Arrays must be 8-byte aligned and must not overlap.  The call
 * synchronises the stream once per V-cycle to read the residual norm.
 * Returns AFMG_OK, AFMG_NOT_CONVERGED (stats filled), or an error.
 */
int afmg_solve(afmg_tree *tree, void *stream, const double *rho, const double *bc, double *u,
               void *workspace, size_t workspace_bytes, const afmg_opts *opts,
               afmg_stats *stats);

/*
 * afmg_solve without a caller workspace, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same kernels and result as afmg_solve, bitwise.
 * The workspace is instead an array inside the library of AFMG_SCRATCH_BYTES
 * (128 MiB), one copy on every GPU the library runs on, held until the
 * process ends; trees whose workspace (afmg_workspace_bytes for these
 * options) is larger are rejected.  The call allocates nothing, so the tree
 * must already be prepared on the current device (afmg_tree_finalize, or an
 * earlier solve), and opts->graph and opts->profile must be 0 (recording a
 * graph and profiling events allocate).  All calls on one GPU share that
 * GPU's array: calls that overlap on one GPU (on other streams or from other
 * host threads) race and must be serialised by the caller.  The array keeps
 * the contents of the last call; a solve writes every part it reads.
 * Arguments and return values otherwise as afmg_solve.  Errors: AFMG_ERR_ARG
 * (null or misaligned arrays, a batch, an unprepared tree, graph or profile
 * set, workspace above AFMG_SCRATCH_BYTES), AFMG_ERR_HIP.
 */
#define AFMG_SCRATCH_BYTES ((size_t)128 << 20)
int afmg_solve_noalloc(afmg_tree *tree, void *stream, const double *rho, const double *bc, double *u,
                       const afmg_opts *opts, afmg_stats *stats);

/* Operators of afmg_apply (homogeneous Dirichlet values). */
typedef enum { AFMG_OP_L = 0, AFMG_OP_LT = 1 } afmg_op;

/* Device workspace bytes afmg_apply and afmg_adjoint need. */
int afmg_adjoint_workspace_bytes(const afmg_tree *tree, const afmg_opts *opts, size_t *bytes);

/*
 * y = L x or y = L^T x on the leaf cells, where L is the composite operator of
 * the solve with zero Dirichlet values: the 5/7-point Laplacian with the side
 * ghosts of §2.4 and §3.3 written out, the value of a refined same-level
 * neighbour being the mean of its children (§2.5).  On adaptive grids the
 * refinement-boundary ghost makes L non-symmetric.  x, y: device
 * [n_boxes][N^D] in the layout of afmg_solve; only leaf boxes of x are read,
 * parent boxes of y are set to zero.  Errors: AFMG_ERR_ARG, AFMG_ERR_HIP.
 */
int afmg_apply(afmg_tree *tree, void *stream, int op, const double *x, double *y, void *workspace,
               size_t workspace_bytes);

/*
 * Adjoint of the solve.  With u* = L^-1 (rho - B b) the converged solution
 * ((B b)_c = sum over the Dirichlet sides of c of 2 b / h^2), a loss l(u*) and
 * u_bar = dl/du* on the leaf cells:
 *   rho_bar = dl/drho = lambda,  lambda = L^-T u_bar;
 *   bc_bar  = dl/db   = -2 lambda_c / h^2 for each Dirichlet row entry, c the
 *             leaf cell next to that face (zero for non-leaf values, which the
 *             converged solution does not depend on).
 * On grids whose leaves all lie on one level L is symmetric and lambda is one
 * more multigrid solve (V-cycles, zero Dirichlet values).  Otherwise lambda
 * comes from BiCGSTAB on L^T, right-preconditioned by one V-cycle of L scaled
 * by the cell volumes.  opts: tol (relative max-norm of u_bar - L^T lambda),
 * max_cycles (iterations), n_down/n_up/n_base of the V-cycle; stats.cycles
 * counts V-cycles or BiCGSTAB iterations, stats.r_max is the final true
 * residual max |u_bar - L^T lambda|.  Where BiCGSTAB's recursive residual
 * meets tol but the true one does not, the iteration restarts from the true
 * residual (at most twice); if it still misses tol the call returns
 * AFMG_NOT_CONVERGED.
 *   u_bar    device [n_boxes][N^D]; entries on parent boxes (where u* is the
 *            restriction of the leaves) reach the leaves through the
 *            transposed restriction
 *   rho_bar  device [n_boxes][N^D] out (parents zero)
 *   bc_bar   device [n_bfaces][N^(D-1)] out, or NULL
 *   workspace >= afmg_adjoint_workspace_bytes
 * Returns AFMG_OK, AFMG_NOT_CONVERGED, or an error.
 */
int afmg_adjoint(afmg_tree *tree, void *stream, const double *u_bar, double *rho_bar, double *bc_bar,
                 void *workspace, size_t workspace_bytes, const afmg_opts *opts, afmg_stats *stats);

/*
 * Batches: many independent trees of one dimension solved together.
 *
 * The paper parallelises the loops over the boxes of one level (§2.6).  A
 * batch extends each such loop over the boxes of that level of every tree:
 * the boxes of all trees form one list ordered by level, then tree, then
 * Morton index, and every kernel of the cycle (§3.2) runs once per level for
 * all trees.  Each tree still follows exactly the iteration afmg_solve runs on
 * it alone (same kernels and arithmetic, its own stop test): trees that have
 * stopped are masked out of later cycles, and an FMG step at level l involves
 * only trees that reach level l.  The solution of each tree is therefore
 * identical to its afmg_solve result.  Each tree's stop test runs on the
 * device after every cycle; a tree that stops leaves the per-level lists of
 * boxes the kernels take their work from, so later launches do no work for
 * it.
 */
typedef struct {
    int dim, box_n, n_trees;
    int lmax;            /* finest level over all trees */
    int64_t n_boxes;     /* sum of the trees' n_boxes (the caller's layout) */
    int64_t n_bfaces;    /* sum of the trees' n_bfaces */
    int64_t n_unknowns;  /* sum of the trees' leaf cells */
} afmg_batch_desc;

/*
 * Group n_trees >= 1 trees of the same dim and box_n.  Their topology is
 * copied: the trees may be destroyed afterwards.  Trees take part when they
 * have one level-1 box, Dirichlet sides and the Laplacian.  Host-only.
 * Errors: AFMG_ERR_ARG (null, empty, mixed dimensions or box sizes, a tree
 * that cannot take part), AFMG_ERR_OOM.
 */
int afmg_batch_create(afmg_tree *const *trees, int n_trees, afmg_batch **out);

void afmg_batch_destroy(afmg_batch *batch);

int afmg_batch_info(const afmg_batch *batch, afmg_batch_desc *out);

/* Device workspace bytes afmg_batch_solve needs for these options. */
int afmg_batch_workspace_bytes(const afmg_batch *batch, const afmg_opts *opts, size_t *bytes);

/*
 * afmg_solve on every tree of the batch.  rho, u: device arrays holding the
 * trees' [n_boxes][N^D] arrays one after the other, in the order the trees
 * were given (each in its own box-id order, as afmg_solve takes it); bc:
 * likewise the trees' Dirichlet rows one after the other, or NULL for zero.
 * stats: host array of n_trees records, one per tree (t_ms is the time of the
 * whole batch).  Returns AFMG_OK when every tree converged, the first error of
 * a tree (in tree order) if any tree failed, else AFMG_NOT_CONVERGED.
 */
int afmg_batch_solve(afmg_batch *batch, void *stream, const double *rho, const double *bc, double *u,
                     void *workspace, size_t workspace_bytes, const afmg_opts *opts,
                     afmg_stats *stats);

/*
 * Launch shapes and the autotuner.
 *
 * The per-level kernels of the cycle run in workgroups of 64, 128 or 256
 * threads, one thread per x-row of a box (N^(D-1) threads per box, so 1, 2
 * or 4 boxes of 8^3 cells per workgroup in 3D and 8, 16 or 32 of 8^2 in 2D;
 * a box of 16^3 cells needs the 256-thread workgroup), and either hand each
 * of the eight XCDs a contiguous run of boxes (siblings and neighbours share
 * that XCD's L2) or take boxes in launch order.  The shape is chosen per
 * kernel class, level and precision; every shape computes bitwise the same
 * values.  The default is 256 threads with XCD runs.
 */
typedef enum {
    AFMG_K_GSRB = 0,       /* red-black half sweep (§3.1) */
    AFMG_K_RESID = 1,      /* residual + restriction (eq. residual, §2.5) */
    AFMG_K_COARSE_RHS = 2, /* FAS right-hand side and the copy v' (eq. coarse-rhs) */
    AFMG_K_PROLONG = 3,    /* prolongation + correction (eq. coarse-corr) */
    AFMG_K_FINAL = 4,      /* restriction of u + composite leaf residual (FP64 only) */
    AFMG_K_KINDS = 5
} afmg_kernel_kind;

/* Device workspace bytes afmg_tree_autotune needs (scratch, 256-aligned). */
int afmg_autotune_workspace_bytes(const afmg_tree *tree, size_t *bytes);

/*
 * Time every shape of every kernel class on every level of the tree, for
 * FP64 and FP32 arrays, on zero-filled scratch arrays in workspace, and keep
 * the fastest for later solves (the default unless another is at least 10%
 * faster).  Synchronises the stream.  Errors: AFMG_ERR_ARG, AFMG_ERR_HIP.
 */
int afmg_tree_autotune(afmg_tree *tree, void *stream, void *workspace, size_t workspace_bytes);

/* Shape of kernel class `kind` on level `level` (1 .. lmax) for precision 0
   (FP64 arrays) or 1 (FP32 arrays of the mixed refinement). */
int afmg_tree_shape(const afmg_tree *tree, int precision, int kind, int level, int *wg, int *no_remap);

/* Set a shape; -1 for precision, kind or level selects all of them.
   wg in {64, 128, 256} holding whole boxes (wg >= box_n^(dim-1)),
   no_remap in {0, 1}.  Errors: AFMG_ERR_ARG. */
int afmg_tree_set_shape(afmg_tree *tree, int precision, int kind, int level, int wg, int no_remap);

/* The same for a batch (its levels are those of the whole batch). */
int afmg_batch_autotune_workspace_bytes(const afmg_batch *batch, size_t *bytes);
int afmg_batch_autotune(afmg_batch *batch, void *stream, void *workspace, size_t workspace_bytes);
int afmg_batch_shape(const afmg_batch *batch, int precision, int kind, int level, int *wg, int *no_remap);
int afmg_batch_set_shape(afmg_batch *batch, int precision, int kind, int level, int wg, int no_remap);

/*
 * One step of the cycle on caller arrays, for checking the kernels one at a
 * time against a reference implementation (a solve does not need it).
 *   AFMG_STEP_HALF_SWEEP      one red (colour 0) or black (1) half sweep of
 *                             every box of `level` >= 1, side ghosts formed
 *                             from the current u (§3.1, §2.4, §3.3)
 *   AFMG_STEP_RESID_RESTRICT  boxes of `level` >= 2: r = rho - L u; each
 *                             parent's octant receives mean(u) in u and
 *                             mean(r) in rho (eq. residual, §2.5)
 *   AFMG_STEP_COARSE_RHS      boxes of `level` >= 2: uold <- u; on parents
 *                             rho <- rho + L u (eq. coarse-rhs; rho holds the
 *                             restricted residual on input)
 *   AFMG_STEP_PROLONG         boxes of `level` >= 2: u += P211(u - uold of the
 *                             parent) (eq. coarse-corr, §2.5); uold of the
 *                             parents holds v' as copied by COARSE_RHS
 *   AFMG_STEP_COARSE          the root box right after a restriction from
 *                             level 2 (rho of the root = restricted residual):
 *                             its FAS right-hand side, copy v', and the
 *                             V-cycle from level 1 through the coarse grids
 *                             below it; `level` is ignored; needs lmax >= 2
 * u, rho, uold: device [n_boxes][N^D] in the layout of afmg_solve (uold
 * full-size too); every box is read and only the step's outputs change.  bc:
 * the leaf Dirichlet rows or NULL (zero); homog = 1 uses zero values.  opts:
 * n_down / n_up / n_base of AFMG_STEP_COARSE (NULL: defaults).  workspace:
 * afmg_workspace_bytes for FP64.  Synchronises the stream.
 */
typedef enum {
    AFMG_STEP_HALF_SWEEP = 0,
    AFMG_STEP_RESID_RESTRICT = 1,
    AFMG_STEP_COARSE_RHS = 2,
    AFMG_STEP_PROLONG = 3,
    AFMG_STEP_COARSE = 4
} afmg_step_op;
int afmg_step(afmg_tree *tree, void *stream, int op, int level, int colour, int homog, double *u,
              double *rho, double *uold, const double *bc, void *workspace, size_t workspace_bytes,
              const afmg_opts *opts);

/* Message for the last failing call on this thread. */
const char *afmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AFMG_H */
