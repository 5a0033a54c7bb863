// Cycle scheduler and C-ABI of the afmg library.
//
// The scheduler issues the kernels of one FAS V-cycle level by level (paper
// §3.2): smoothing, residual + restriction, FAS right-hand side and the copy
// v'_H, the kernel for the root box and the coarse grids below it, then
// prolongation + correction and smoothing on the way up.  After each cycle the
// composite leaf residual is reduced on the device and its max-norm is read
// back for the stop test.
//
// A batch is a forest: the boxes of all its trees in one list (level, tree,
// Morton), so every launch covers one level of every tree.  Each tree keeps
// its own stop test; a per-tree mask on the device removes stopped trees from
// later cycles, so each tree runs exactly the iteration it would run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "afmg.h"
#include "afmg_internal.h"
#include "afmg_kernels.h"

using namespace afmg;

// Workspace of afmg_solve_noalloc, one copy on every GPU the library runs on
// (held until the process ends).  In host code this name is only a handle
// for hipGetSymbolAddress: the device address of each GPU's copy is looked up
// once per device and used everywhere the host needs the array.
static __device__ __align__(256) unsigned char scratch[AFMG_SCRATCH_BYTES];

namespace {
thread_local std::string g_err;

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES] = {};
}

void afmg::set_error(const std::string &m) { g_err = m; }
extern "C" const char *afmg_last_error(void) { return g_err.c_str(); }

namespace {
// Launch shape of one kernel class on one level: workgroup size (64, 128 or
// 256 threads) and whether workgroups take boxes in XCD-contiguous runs.
// Every shape computes bitwise the same values.
struct Shape {
    int wg = 256;
    int no_remap = 0;
};
enum { SK_GSRB, SK_RESID, SK_CRHS, SK_PROLONG, SK_FINAL, SK_KINDS };
constexpr int SHAPE_WGS[3] = {256, 128, 64};

// The repeated cycle recorded as a HIP graph (opts.graph), with the
// arguments it was recorded for.
struct Recorded {
    hipStream_t cap = nullptr;  // private stream, used only for recording
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> key;

    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
};
}  // namespace

struct afmg_tree {
    HostTree h;
    int device = -1;
    BoxInfo *d_info = nullptr;
    int32_t *d_child = nullptr;      // [n_boxes][8] child ids (adjoint, coarse kernel)
    double *h_norm = nullptr;        // (max, L2) per tree: pinned, coherent host memory
                                     // that the norm kernels write directly
    double *d_norm_host = nullptr;   // h_norm's device address
    std::vector<int64_t> part_off;   // first k_final partial of each level (one tree)
    int64_t n_parts = 0;
    int64_t n_parts_max = 0;         // partials for the smallest workgroups
    std::vector<Shape> shapes[2][SK_KINDS];  // [FP64, FP32][kernel class][level]
    int tune_epoch = 0;              // bumped by every autotune
    std::vector<hipEvent_t> events;  // event pairs for opts.profile
    hipEvent_t span[2] = {nullptr, nullptr};  // first kernel .. last norm of a solve
    Recorded rec;
    // forests (batches): per-tree mask and tables, and the caller's layout
    bool forest = false;
    int *h_active = nullptr;              // pinned per-tree mask
    int *d_active = nullptr;              // mask of the trees still iterating
    int *d_mask = nullptr;                // mask of one FMG step
    int32_t *d_tree_lmax = nullptr;
    int64_t *d_tree_leaf_ptr = nullptr;
    int32_t *d_tree_leaf_box = nullptr;
    std::vector<int32_t> box_map;         // caller's box of each working box
    std::vector<int32_t> row_map;         // caller's Dirichlet row of each leaf row
    int32_t *d_box_map = nullptr, *d_row_map = nullptr;
    // forests: the stop rule on the device and the compacted box lists
    double *d_tnorm = nullptr;            // (max, L2) per tree after a cycle
    TreeStop *d_tstop = nullptr, *h_tstop = nullptr;  // per-tree state (h_: pinned)
    double *d_thist = nullptr, *h_thist = nullptr;    // [n][2][AFMG_HIST] history
    int64_t *d_ltoff = nullptr;           // [(lmax+2)][n+1] first box of tree t on level l
    int64_t *d_lvloff = nullptr;          // first box of each level
    int32_t *d_act = nullptr;             // per level: boxes of the trees still iterating
    int *d_nact = nullptr;                // their count per level
    int64_t user_boxes = 0, user_rows = 0, user_unknowns = 0;
    // operator (afmg_tree_set_operator): OPK_* bits, the cell coefficients
    // (colour-split, [n_boxes][N^D] plus a flag word), the x index of every
    // box, and whether the domain itself needs the general coarse path
    int opk = 0;
    double *d_eps = nullptr;
    int32_t *d_bx = nullptr;
    int32_t *d_dnbr = nullptr;  // [n_boxes][27] same-level boxes across edges and corners
    int op_kind = 0, op_prolong = 0, ghost_scheme = 0;
    int domain_general = -1;  // -1 until the first set_operator
};

struct afmg_batch {
    afmg_tree f;
};

namespace {

// Boxes of 8^D or 16^D cells (paper §2.1: N is a parameter of the grid); the
// kernels and the scheduler are instantiated for both: FN<dim, N> ARGS.
#define AFMG_BOX_DISPATCH(h, FN, ARGS)                               \
    do {                                                             \
        if ((h).dim == 3) {                                          \
            if ((h).N == 16) FN<3, 16> ARGS;                         \
            else FN<3, 8> ARGS;                                      \
        } else {                                                     \
            if ((h).N == 16) FN<2, 16> ARGS;                         \
            else FN<2, 8> ARGS;                                      \
        }                                                            \
    } while (0)
#define AFMG_BOX_RETURN(h, FN, ARGS)                                      \
    return (h).dim == 3 ? ((h).N == 16 ? FN<3, 16> ARGS : FN<3, 8> ARGS)  \
                        : ((h).N == 16 ? FN<2, 16> ARGS : FN<2, 8> ARGS)

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(AFMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t cells_per_box(int dim, int n) { return dim == 3 ? (int64_t)n * n * n : (int64_t)n * n; }
int64_t cells_per_face(int dim, int n) { return dim == 3 ? (int64_t)n * n : n; }
// cell size of level l (level-1 boxes are unit cubes, paper §2.2)
double level_h(int l, int n) { return 1.0 / ((double)n * std::ldexp(1.0, l - 1)); }

// x bits of the Morton key of level l when the level is complete (one tree,
// all 2^(D (l-1)) boxes present, so that box index = key); 0 otherwise
int cube_xmask(const HostTree &h, int l) {
    const int lg = l - 1;
    if (h.n_trees != 1 || h.general || lg < 1 || h.dim * lg > 30) return 0;
    if (h.level_count(l) != ((int64_t)1 << (h.dim * lg))) return 0;
    int m = 0;
    for (int b = 0; b < lg; b++) m |= 1 << (h.dim * b);
    return m;
}

struct WsLayout {
    // FP64: rho, uold; mixed: rho (FP64 leaf rho), e, rho_e, uold_e (FP32);
    // forests also hold the working u; general domains the grids of the
    // coarse kernel
    size_t rho, uold, bc, partial, e, rho_e, uold_e, u, cg, total;
};

// Levels <= 1 take the general coarse kernel (grids in global memory) on
// general domains, the one-tree coarse kernel (LDS) otherwise.
bool coarse_general(const HostTree &h) { return h.general; }

// The coarsest level the box kernels run: 2 on general domains and where the
// one-tree coarse kernel's LDS cannot hold level 2 as well (3D boxes of 16^3
// cells), else 3 (level 2 inside the coarse kernel).
int box_lo(const HostTree &h) { return (h.general || !coarse_kernel_level2(h.dim, h.N)) ? 2 : 3; }

// The byte model of one FP64 solve with the Laplacian (see
// afmg_solve_bytes_model): every array a kernel touches, once per launch,
// over the launch sequence of Cycler::fmg / vcycle and Solver.
double solve_bytes_model(const HostTree &h, int v_cycles, bool fmg, int n_down, int n_up) {
    const double s = 8.0, r = 1.0 / (double)(1 << h.dim), C = (double)cells_per_box(h.dim, h.N);
    std::vector<double> all((size_t)h.lmax + 2, 0.0), leaf((size_t)h.lmax + 2, 0.0);
    for (const BoxInfo &bi : h.info) {
        if (bi.level < 1) continue;
        all[(size_t)bi.level] += C;
        if (bi.flags & FLAG_LEAF) leaf[(size_t)bi.level] += C;
    }
    double n_all = 0.0, n_leaf = 0.0;
    int lmin_leaf = h.lmax;
    for (int l = 1; l <= h.lmax; l++) {
        n_all += all[(size_t)l];
        n_leaf += leaf[(size_t)l];
        if (leaf[(size_t)l] > 0.0 && l < lmin_leaf) lmin_leaf = l;
    }
    const int lo = box_lo(h);
    auto finalize = [&](int lfirst) {
        double b = 0.0;
        for (int l = std::max(1, lfirst); l <= h.lmax; l++) {
            if (l == 1 && leaf[1] == 0.0) continue;
            b += leaf[(size_t)l] * (2 * s + s * r) + (all[(size_t)l] - leaf[(size_t)l]) * (s + s * r);
        }
        return b;
    };
    const double coarse = 4 * s * all[(size_t)(lo == 3 && h.lmax >= 2 ? 2 : 1)];
    auto vcycle = [&](int top) {
        if (top < lo) return coarse;
        double b = 0.0;
        for (int l = top; l >= lo; l--) {
            b += 2 * n_down * 1.5 * s * all[(size_t)l] + (2 * s + 2 * s * r) * all[(size_t)l];
            if (l - 1 >= lo) b += 4 * s * all[(size_t)l - 1];
        }
        b += coarse;
        for (int l = lo; l <= top; l++) b += (2 * s + 2 * s * r) * all[(size_t)l] + 2 * n_up * 1.5 * s * all[(size_t)l];
        return b;
    };
    double b = 2 * s * n_leaf + s * n_all + finalize(1);  // rho layout, u = 0, initial residual
    if (fmg) {
        for (int l = 2; l <= h.lmax; l++) b += (s + s * r) * all[(size_t)l];  // rho restricted down
        b += coarse;
        for (int l = 2; l <= h.lmax; l++) {
            if (l < h.lmax) b += 2 * s * all[(size_t)l];  // the copy v'
            b += (2 * s + 2 * s * r) * all[(size_t)l] + vcycle(l);
        }
        b += finalize(lmin_leaf);
    }
    b += v_cycles * (vcycle(h.lmax) + finalize(lmin_leaf));
    b += 2 * s * n_all;  // layout conversion of u on return
    return b;
}

// bytes of the general coarse kernel's grids (0 where it is not used)
size_t coarse_gen_bytes(const HostTree &h, int opk) {
    if (!coarse_general(h)) return 0;
    size_t n = 0;
    AFMG_BOX_DISPATCH(h, n = coarse_gen_doubles, (h.n_roots, opk));
    return sizeof(double) * n;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout ws_layout(const afmg_tree *t, int precision) {
    const HostTree &h = t->h;
    const size_t C = (size_t)cells_per_box(h.dim, h.N), F = (size_t)cells_per_face(h.dim, h.N);
    const size_t nlt = (size_t)h.n_below_lmax(), nb = (size_t)h.n_boxes;
    const bool mixed = precision == AFMG_MIXED;
    const size_t np = t->forest ? nb : (size_t)std::max<int64_t>(1, t->n_parts_max);
    WsLayout L{};
    size_t off = 0;
    L.rho = off; off = align256(off + nb * C * sizeof(double));
    L.uold = off; off = align256(off + (mixed ? 0 : nlt * C * sizeof(double)));
    L.bc = off; off = align256(off + (size_t)std::max<int64_t>(1, h.n_bfaces_all) * F * sizeof(double));
    L.partial = off; off = align256(off + np * 2 * sizeof(double));
    L.e = off; off = align256(off + (mixed ? nb * C * sizeof(float) : 0));
    L.rho_e = off; off = align256(off + (mixed ? nb * C * sizeof(float) : 0));
    L.uold_e = off; off = align256(off + (mixed ? nlt * C * sizeof(float) : 0));
    L.u = off; off = align256(off + (t->forest ? nb * C * sizeof(double) : 0));
    L.cg = off; off = align256(off + coarse_gen_bytes(h, t->opk));
    L.total = off;
    return L;
}

// Workspace of the autotuner: the arrays of both precisions and a working u.
struct TuneLayout {
    size_t u, rho, uold, bc, partial, e, rho_e, uold_e, total;
};

TuneLayout tune_layout(const afmg_tree *t) {
    const HostTree &h = t->h;
    const size_t C = (size_t)cells_per_box(h.dim, h.N), F = (size_t)cells_per_face(h.dim, h.N);
    const size_t nlt = (size_t)h.n_below_lmax(), nb = (size_t)h.n_boxes;
    TuneLayout L{};
    size_t off = 0;
    L.u = off; off = align256(off + nb * C * sizeof(double));
    L.rho = off; off = align256(off + nb * C * sizeof(double));
    L.uold = off; off = align256(off + std::max<size_t>(1, nlt) * C * sizeof(double));
    L.bc = off; off = align256(off + (size_t)std::max<int64_t>(1, h.n_bfaces_all) * F * sizeof(double));
    L.partial = off; off = align256(off + std::max<size_t>(nb, (size_t)t->n_parts_max) * 2 * sizeof(double));
    L.e = off; off = align256(off + nb * C * sizeof(float));
    L.rho_e = off; off = align256(off + nb * C * sizeof(float));
    L.uold_e = off; off = align256(off + std::max<size_t>(1, nlt) * C * sizeof(float));
    L.total = off;
    return L;
}

template <int D, int N>
int64_t final_wgs_d(int64_t nb, int wg) { return final_wgs<D, N>(nb, wg); }


// k_final partial offsets per level for the current shapes, and the count
// for the smallest workgroups (the workspace is sized for that)
void compute_partials(afmg_tree *t) {
    const HostTree &h = t->h;
    for (auto &pk : t->shapes)
        for (auto &v : pk)
            if (v.size() != (size_t)h.lmax + 2) v.assign((size_t)h.lmax + 2, Shape{});
    t->part_off.assign((size_t)h.lmax + 2, 0);
    int64_t n = 0, nmax = 0;
    for (int l = h.lmax; l >= 1; l--) {
        t->part_off[(size_t)l] = n;
        if (l >= 2 || h.level1_leaf) {
            // (trees with an operator: the operator kernels' workgroups)
            const int wg = t->opk ? op_wg(h.dim, h.N) : t->shapes[0][SK_FINAL][(size_t)l].wg;
            AFMG_BOX_DISPATCH(h, n += final_wgs_d, (h.level_count(l), wg));
            AFMG_BOX_DISPATCH(h, nmax += final_wgs_d, (h.level_count(l), 64));
        }
    }
    t->n_parts = n;
    t->n_parts_max = nmax;
}

template <class V>
int upload(V *&dst, const std::vector<V> &src, const char *what) {
    const size_t bytes = sizeof(V) * std::max<size_t>(1, src.size());
    hipError_t e = hipMalloc(&dst, bytes);
    if (e != hipSuccess) return fail(AFMG_ERR_OOM, std::string("hipMalloc of ") + what + " failed");
    if (src.empty()) return AFMG_OK;
    e = hipMemcpy(dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
    return AFMG_OK;
}

int bind_device(afmg_tree *t) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (t->device >= 0) {
        if (dev != t->device) return fail(AFMG_ERR_ARG, "tree was first used on another device");
        return AFMG_OK;
    }
    const HostTree &h = t->h;
    int rc;
    if ((rc = upload(t->d_info, h.info, "the box table")) != AFMG_OK) return rc;
    if ((rc = upload(t->d_child, h.child, "the child table")) != AFMG_OK) return rc;
    e = hipHostMalloc(&t->h_norm, 2 * sizeof(double) * (size_t)h.n_trees,
                      hipHostMallocCoherent | hipHostMallocMapped);
    if (e != hipSuccess) return fail(AFMG_ERR_OOM, "hipHostMalloc failed");
    e = hipHostGetDevicePointer((void **)&t->d_norm_host, t->h_norm, 0);
    if (e != hipSuccess) return hip_fail(e, "hipHostGetDevicePointer");
    for (hipEvent_t &ev : t->span) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (t->forest) {
        e = hipHostMalloc(&t->h_active, sizeof(int) * (size_t)h.n_trees, hipHostMallocDefault);
        if (e != hipSuccess) return fail(AFMG_ERR_OOM, "hipHostMalloc failed");
        const std::vector<int> ones((size_t)h.n_trees, 1);
        if ((rc = upload(t->d_active, ones, "the tree mask")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_mask, ones, "the tree mask")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_tree_lmax, h.tree_lmax, "the tree levels")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_tree_leaf_ptr, h.tree_leaf_ptr, "the tree leaf lists")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_tree_leaf_box, h.tree_leaf_box, "the tree leaf lists")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_box_map, t->box_map, "the box map")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_row_map, t->row_map, "the row map")) != AFMG_OK) return rc;
        const size_t n = (size_t)h.n_trees, L = (size_t)h.lmax + 2;
        if ((rc = upload(t->d_tnorm, std::vector<double>(2 * n, 0.0), "the tree norms")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_tstop, std::vector<TreeStop>(n, TreeStop{}), "the tree states")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_thist, std::vector<double>(2 * n * AFMG_HIST, 0.0), "the tree histories")) != AFMG_OK)
            return rc;
        e = hipHostMalloc(&t->h_tstop, sizeof(TreeStop) * n, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&t->h_thist, sizeof(double) * 2 * n * AFMG_HIST, hipHostMallocDefault);
        if (e != hipSuccess) return fail(AFMG_ERR_OOM, "hipHostMalloc failed");
        // boxes of one tree on one level are contiguous (level, tree, Morton)
        std::vector<int64_t> ltoff(L * (n + 1), 0);
        for (int l = 1; l <= h.lmax; l++) {
            int64_t *to = ltoff.data() + (size_t)l * (n + 1);
            int64_t b = h.lvl_off[(size_t)l];
            for (size_t tr = 0; tr <= n; tr++) {
                while (b < h.lvl_off[(size_t)l + 1] && (size_t)h.info[(size_t)b].tree < tr) b++;
                to[tr] = b;
            }
        }
        if ((rc = upload(t->d_ltoff, ltoff, "the tree offsets")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_lvloff, h.lvl_off, "the level offsets")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_act, std::vector<int32_t>((size_t)h.n_boxes, 0), "the box lists")) != AFMG_OK) return rc;
        if ((rc = upload(t->d_nact, std::vector<int>(L, 0), "the box counts")) != AFMG_OK) return rc;
        // every tree listed until a solve sets the mask
        launch_compact(t->d_active, t->d_ltoff, t->d_lvloff, h.n_trees, h.lmax, t->d_act, t->d_nact, nullptr);
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "box lists");
    }
    t->device = dev;
    return AFMG_OK;
}

void release(afmg_tree *t) {
    t->rec.drop();
    if (t->rec.cap) (void)hipStreamDestroy(t->rec.cap);
    for (void *p : {(void *)t->d_info, (void *)t->d_child, (void *)t->d_active, (void *)t->d_mask,
                    (void *)t->d_tree_lmax, (void *)t->d_tree_leaf_ptr, (void *)t->d_tree_leaf_box,
                    (void *)t->d_box_map, (void *)t->d_row_map, (void *)t->d_tnorm, (void *)t->d_tstop,
                    (void *)t->d_thist, (void *)t->d_ltoff, (void *)t->d_lvloff, (void *)t->d_act,
                    (void *)t->d_nact, (void *)t->d_eps, (void *)t->d_bx, (void *)t->d_dnbr})
        if (p) (void)hipFree(p);
    if (t->h_norm) (void)hipHostFree(t->h_norm);
    if (t->h_active) (void)hipHostFree(t->h_active);
    if (t->h_tstop) (void)hipHostFree(t->h_tstop);
    if (t->h_thist) (void)hipHostFree(t->h_thist);
    for (auto ev : t->events) (void)hipEventDestroy(ev);
    for (auto ev : t->span)
        if (ev) (void)hipEventDestroy(ev);
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_opts(const afmg_opts *o) {
    if (!o) return fail(AFMG_ERR_ARG, "opts is null");
    if (o->cycle != AFMG_CYCLE_V && o->cycle != AFMG_CYCLE_FMG_V) return fail(AFMG_ERR_ARG, "bad cycle");
    if (o->n_down < 0 || o->n_up < 0 || o->n_base < 1 || o->n_down > 64 || o->n_up > 64 || o->n_base > 1024)
        return fail(AFMG_ERR_ARG, "smoothing counts out of range");
    if (!(o->tol >= 0.0) || o->max_cycles < 0 || o->max_cycles > 100000 || o->fixed_cycles < 0 ||
        o->fixed_cycles > 100000)
        return fail(AFMG_ERR_ARG, "tol / max_cycles / fixed_cycles out of range");
    if (o->precision != AFMG_FP64 && o->precision != AFMG_MIXED) return fail(AFMG_ERR_ARG, "bad precision");
    if (o->check_every < 0 || o->check_every > 1000) return fail(AFMG_ERR_ARG, "check_every out of range");
    if (o->prof_level < 0 || o->prof_level > 64) return fail(AFMG_ERR_ARG, "prof_level out of range");
    return AFMG_OK;
}

// ---------------------------------------------------------------------------
// kernel timing for opts.profile
// ---------------------------------------------------------------------------
constexpr int PROF_PAIRS = 64;

struct Prof {
    afmg_tree *t;
    hipStream_t st;
    bool on;
    int lmax;  // the level whose launches are timed (opts.prof_level, else the finest)
    afmg_stats *stats;
    std::vector<std::array<int, 3>> pending;  // (kernel class, event pair, launches)

    // Bracket `count` consecutive finest-level launches of one kernel class
    // with an event pair when profiling (s: the stream of the launches).
    template <class Fn>
    void timed(int kind, int l, Fn fn, hipStream_t s = nullptr, int count = 1) {
        const int pair = (int)pending.size();
        if (!on || kind < 0 || l != lmax || pair >= PROF_PAIRS || count < 1) {
            fn();
            return;
        }
        hipStream_t es = s ? s : st;
        (void)hipEventRecord(t->events[(size_t)(2 * pair)], es);
        fn();
        (void)hipEventRecord(t->events[(size_t)(2 * pair + 1)], es);
        pending.push_back({kind, pair, count});
    }
    // after a stream synchronisation: add the timed launches to the stats
    void collect() {
        for (const auto &p : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, t->events[(size_t)(2 * p[1])], t->events[(size_t)(2 * p[1] + 1)]) ==
                hipSuccess) {
                stats->prof_ms[p[0]] += ms;
                stats->prof_n[p[0]] += p[2];
            }
        }
        pending.clear();
    }
};

// ---------------------------------------------------------------------------
// the FAS cycles (paper §3.2) on arrays of type T
// ---------------------------------------------------------------------------
template <int D, int N, typename T>
struct Cycler {
    const HostTree &h;
    hipStream_t st;
    const afmg_opts &o;
    Prof &prof;
    LevelArgs<T> base;
    const double *bc64;  // boundary rows for the coarse kernel (null when homogeneous)
    afmg_tree *t;        // forests: tree levels and the FMG step mask
    double *cg = nullptr;  // general domains: the grids of the coarse kernel
    // mixed-precision correction on a tree whose leaves all lie on level
    // lmax (complete): the last half sweep of a V-cycle from lmax adds e to
    // this FP64 solution and clears e (see fuses_update)
    double *add_to = nullptr;
    // set for a V-cycle that follows one with the fused update: its first
    // half sweep on lmax takes the updated colour's old values as zero (the
    // fused update cleared only the other colour of e)
    bool zero_start = false;

    // whether a V-cycle from level top ends with the fused update
    bool fuses_update(int top) const {
        return add_to != nullptr && top == h.lmax && top >= 3 && o.n_up > 0 && o.n_down > 0;
    }

    LevelArgs<T> lev(int l) const {
        LevelArgs<T> a = base;
        a.b0 = h.lvl_off[(size_t)l];
        a.nb = (int)h.level_count(l);
        a.xmask = cube_xmask(h, l);
        const double hh = level_h(l, N);
        a.h2 = (T)(hh * hh);
        a.ih2 = (T)(1.0 / (hh * hh));
        a.h = (T)hh;
        if (t->forest) {
            a.act = t->d_act + h.lvl_off[(size_t)l];
            a.nact = t->d_nact + l;
        }
        return a;
    }
    void level(Op op, int l, int colour = 0, bool time = true, double *add = nullptr, bool own_zero = false) {
        const int kind = !time ? -1
                         : op == Op::GSRB ? AFMG_PROF_GSRB
                         : op == Op::RESID_RESTRICT ? AFMG_PROF_RESID
                         : op == Op::PROLONG ? AFMG_PROF_PROLONG : -1;
        const int sk = op == Op::GSRB ? SK_GSRB
                       : op == Op::RESID_RESTRICT ? SK_RESID
                       : op == Op::COARSE_RHS ? SK_CRHS
                       : op == Op::PROLONG ? SK_PROLONG : -1;
        Shape sh;
        if (sk >= 0) sh = t->shapes[sizeof(T) == 4 ? 1 : 0][sk][(size_t)l];
        LevelArgs<T> a = lev(l);
        a.no_remap = sh.no_remap;
        a.add_to = add;
        a.own_zero = own_zero ? 1 : 0;
        prof.timed(kind, l, [&] { launch_level<D, N, T>(op, a, colour, sh.wg, st); }, st);
    }
    // n sweeps; their 2n half sweeps are timed as one group.  add: the last
    // half sweep adds the level's values to this FP64 array and clears its
    // colour; own_zero: the first half sweep takes its colour's old values
    // as zero.
    // With add, the last half sweep (which also does the refinement update)
    // is left out of the timed group.
    void gsrb(int l, int n, double *add = nullptr, bool own_zero = false) {
        const int timed_n = add ? 2 * n - 1 : 2 * n;
        prof.timed(
            AFMG_PROF_GSRB, l,
            [&] {
                for (int q = 0; q < n; q++) {
                    level(Op::GSRB, l, 0, false, nullptr, q == 0 && own_zero);
                    if (q < n - 1 || !add) level(Op::GSRB, l, 1, false);
                }
            },
            st, timed_n);
        if (add) level(Op::GSRB, l, 1, false, add);
    }
    // one workgroup per tree; a tree that is its root box alone takes the
    // top-level-1 path inside the kernel.  General domains: one workgroup for
    // all level-1 boxes and the grids below them.
    void coarse(int mode) {
        if (coarse_general(h)) {
            CoarseGenArgs<T> c{base.info, base.u, base.rho, h.lmax >= 2 ? base.uold : nullptr, bc64, cg,
                               h.n_roots, mode, base.homog, o.n_down, o.n_up, o.n_base};
            c.eps = t->d_eps;
            c.bx = t->d_bx;
            c.opk = t->opk;
            c.dnbr = t->d_dnbr;
            launch_coarse_gen<D, N, T>(c, st);
            return;
        }
        CoarseArgs<T> c{base.info, base.u, base.rho, base.uold, bc64, mode, base.homog,
                        o.n_down, o.n_up, o.n_base, base.active};
        if (h.lmax == 1) c.uold = nullptr;
        if (h.lmax >= 2) {
            const LevelArgs<T> a2 = lev(2);
            c.child = t->d_child;
            c.h2_2 = a2.h2;
            c.ih2_2 = a2.ih2;
        }
        launch_coarse<D, N, T>(c, h.n_trees, st);
    }
    // V-cycle from level top: levels >= 3 box by box, levels <= 2 in the
    // coarse kernel (level 2, the 2^D children of the root, as one grid);
    // general domains: levels >= 2 box by box, levels <= 1 in their coarse
    // kernel
    void vcycle(int top) {
        if (top < 2) {
            coarse(COARSE_V_TOP1);
            return;
        }
        const int lo = box_lo(h);
        for (int l = top; l >= lo; l--) {
            gsrb(l, o.n_down, nullptr, l == top && zero_start && fuses_update(top));
            level(Op::RESID_RESTRICT, l);
            if (l - 1 >= lo) level(Op::COARSE_RHS, l - 1);
        }
        coarse(lo == 2 ? COARSE_V_FROM_2 : top >= 3 ? COARSE_V2_FROM_3 : COARSE_V2_TOP);
        for (int l = lo; l <= top; l++) {
            level(Op::PROLONG, l);
            gsrb(l, o.n_up, l == top && fuses_update(top) ? add_to : nullptr);
        }
    }
    // FMG from a zero guess: restrict rho down, then per level store v',
    // correct from the coarser level and run a V-cycle from it.  In a forest
    // the step at level l involves only the trees that reach level l.
    // zero_u = false: u is zero already.
    void fmg(bool zero_u = true) {
        if (zero_u) launch_fill<T>(base.u, h.n_boxes * cells_per_box(D, N), T(0), st);
        for (int l = h.lmax; l >= 2; l--) level(Op::RESTRICT_RHO, l);
        coarse(COARSE_FMG);
        const int64_t C = cells_per_box(D, N);
        const LevelArgs<T> saved = base;
        for (int l = 2; l <= h.lmax; l++) {
            if (saved.active) {
                launch_level_mask(saved.active, t->d_tree_lmax, l, t->d_mask, h.n_trees, st);
                base.active = t->d_mask;
                compact(t->d_mask);
            }
            if (l < h.lmax)
                launch_copy<T>(base.u + h.lvl_off[(size_t)l] * C, base.uold + h.lvl_off[(size_t)l] * C,
                               h.level_count(l) * C, st);
            level(Op::PROLONG, l);
            vcycle(l);
        }
        base = saved;
        if (saved.active) compact(saved.active);
    }
    // forests: the compacted box lists of the trees set in `mask`
    void compact(const int *mask) {
        launch_compact(mask, t->d_ltoff, t->d_lvloff, h.n_trees, h.lmax, t->d_act, t->d_nact, st);
    }
};

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
template <int D, int N>
struct Solver {
    afmg_tree *t;
    const HostTree &h;
    hipStream_t st;
    const afmg_opts &o;
    Prof prof;
    LevelArgs<double> base;  // FP64 state: u, rho, uold (FP64 path), Dirichlet rows
    double *partial;

    Solver(afmg_tree *t_, hipStream_t s, const afmg_opts &o_, afmg_stats *S)
        : t(t_), h(t_->h), st(s), o(o_),
          prof{t_, s, o_.profile != 0, o_.prof_level > 0 ? o_.prof_level : t_->h.lmax, S, {}} {}

    // Restriction of u into parents and the composite leaf residual (FP64),
    // reduced to (max, L2) per tree in norm; rout receives the FP32 leaf
    // residual for the mixed refinement.
    // Levels below lfirst are skipped: with no leaf at or below a level, its
    // restriction into the parents feeds no residual, and the next V-cycle
    // restricts into those parents again before it reads them
    // (restrict_parents() fills them at the end of a solve).
    void finalize_launch(float *rout, hipStream_t s, int lfirst = 1, double *norm_out = nullptr) {
        for (int l = h.lmax; l >= std::max(1, lfirst); l--) {
            if (l == 1 && !t->forest && !h.level1_leaf) continue;
            const double hh = level_h(l, N);
            const double hD = D == 3 ? hh * hh * hh : hh * hh;
            LevelArgs<double> a = base;
            a.b0 = h.lvl_off[(size_t)l];
            a.nb = (int)h.level_count(l);
            a.h2 = hh * hh;
            a.ih2 = 1.0 / (hh * hh);
            a.h = hh;
            if (t->forest) {
                a.act = t->d_act + h.lvl_off[(size_t)l];
                a.nact = t->d_nact + l;
            }
            const Shape sh = t->shapes[0][SK_FINAL][(size_t)l];
            a.no_remap = sh.no_remap;
            prof.timed(
                AFMG_PROF_FINAL, l,
                [&] {
                    launch_final<D, N, double>(a, partial, t->forest ? -1 : t->part_off[(size_t)l], hD, rout,
                                                   sh.wg, s);
                },
                s);
        }
        double *out = norm_out ? norm_out : t->d_norm_host;
        if (t->forest)
            launch_reduce_trees(partial, t->d_tree_leaf_ptr, t->d_tree_leaf_box, base.active, out, h.n_trees, s);
        else
            launch_reduce(partial, t->n_parts, out, s);
    }
    // parents of the levels that the per-cycle finalize skips receive the
    // restriction of the solution (k_final's arithmetic and order)
    void restrict_parents() {
        for (int l = h.lmin_leaf - 1; l >= 2; l--) {
            if (t->opk)
                launch_restrict_field_op<D, N>(t->d_info, base.u, h.lvl_off[(size_t)l], h.level_count(l), t->opk,
                                                   t->d_bx, level_h(l, N), st);
            else
                launch_restrict_field<D, N>(t->d_info, base.u, h.lvl_off[(size_t)l], h.level_count(l), st);
        }
    }
    // the norms in t->h_norm (written there by the reduction kernels, no
    // copy); synchronises the stream
    int read_norms() {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "stream synchronize");
        prof.collect();
        return AFMG_OK;
    }
    int finalize(float *rout) {
        finalize_launch(rout, st);
        return read_norms();
    }
    // single tree: the two norms
    int finalize(double &rmax, double &rl2, float *rout) {
        const int rc = finalize(rout);
        rmax = t->h_norm[0];
        rl2 = t->h_norm[1];
        return rc;
    }
    // Enqueue the launches of fn(stream) on st, through the recorded graph
    // when opts.graph is set (recorded on first use or when key changes).
    // Profiled solves launch eagerly: event pairs recorded inside a graph do
    // not bracket the kernel nodes' execution reliably.
    template <class Fn>
    int run(const std::vector<uintptr_t> &key, Fn fn) {
        if (!o.graph || o.profile) {
            fn(st);
            return AFMG_OK;
        }
        Recorded &r = t->rec;
        hipError_t e;
        if (!r.exec || r.key != key) {
            r.drop();
            if (!r.cap) {
                e = hipStreamCreateWithFlags(&r.cap, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
            }
            e = hipStreamBeginCapture(r.cap, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            fn(r.cap);
            e = hipStreamEndCapture(r.cap, &r.graph);
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&r.exec, r.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                r.drop();
                return hip_fail(e, "hipGraphInstantiate");
            }
            r.key = key;
        }
        e = hipGraphLaunch(r.exec, st);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return AFMG_OK;
    }
    // per-tree mask of the next launches (forests); h_active is rewritten
    // only after the stream has synchronised
    int upload_mask() {
        if (!t->forest) return AFMG_OK;
        hipError_t e = hipMemcpyAsync(t->d_active, t->h_active, sizeof(int) * (size_t)h.n_trees,
                                      hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "mask upload");
        return AFMG_OK;
    }
};

// Outer loop of the adjoint solve: `step` runs one iteration and leaves the
// residual norms in S.r_max / S.r_l2.
template <class Step>
int iterate(const afmg_opts &o, afmg_stats &S, Step step) {
    const bool fixed = o.fixed_cycles > 0;
    const int nmax = fixed ? o.fixed_cycles : o.max_cycles;
    bool conv = !fixed && S.r_max <= o.tol * S.r0_max;
    int grow = 0;
    double prev = S.r_max;
    while (!conv && S.cycles < nmax) {
        const int rc = step(S.cycles);
        if (rc != AFMG_OK) return rc;
        if (S.cycles < AFMG_HIST) {
            S.hist_max[S.cycles] = S.r_max;
            S.hist_l2[S.cycles] = S.r_l2;
        }
        S.cycles++;
        if (!std::isfinite(S.r_max)) return AFMG_ERR_NONFINITE;
        if (!fixed) {
            grow = S.r_max > prev ? grow + 1 : 0;
            if (grow >= 3) return AFMG_ERR_DIVERGED;
            conv = S.r_max <= o.tol * S.r0_max;
        }
        prev = S.r_max;
    }
    return (!fixed && !conv) ? AFMG_NOT_CONVERGED : AFMG_OK;
}

// Stop rule of one tree: cycles until max|r| <= tol max|r0|, max_cycles,
// a non-finite norm or 3 consecutive growths; exactly fixed_cycles if set.
struct Track {
    bool done = false, conv = false;
    int grow = 0;
    double prev = 0.0;
};

// Outer loop of the solve over the trees of t: `step(k, m)` runs cycles
// k .. k+m-1 on the trees whose mask entry is set and leaves their norms
// after the last one in t->h_norm.  The norms are read, and the stop test
// applied, every check_every cycles (and after the last allowed cycle); the
// history of the cycles in between holds NaN.  Running trees have run the
// same number of cycles, so one m serves them all.
template <int D, int N, class Step>
int iterate_trees(Solver<D, N> &s, afmg_stats *S, std::vector<Track> &tr, Step step) {
    afmg_tree *t = s.t;
    const afmg_opts &o = s.o;
    const int n = t->h.n_trees;
    const bool fixed = o.fixed_cycles > 0;
    const int nmax = fixed ? o.fixed_cycles : o.max_cycles;
    const int every = std::max(1, o.check_every);
    for (int i = 0; i < n; i++) {
        tr[(size_t)i].prev = S[i].r_max;
        if (S[i].status != AFMG_OK) tr[(size_t)i].done = true;
        tr[(size_t)i].conv = !fixed && S[i].r_max <= o.tol * S[i].r0_max;
        if (tr[(size_t)i].conv) tr[(size_t)i].done = true;
    }
    for (int k = 0;;) {
        bool any = false;
        for (int i = 0; i < n; i++) {
            Track &q = tr[(size_t)i];
            if (!q.done && S[i].cycles >= nmax) q.done = true;
            if (t->forest) t->h_active[i] = q.done ? 0 : 1;
            any |= !q.done;
        }
        if (!any) break;
        const int m = std::min(every, nmax - k);
        int rc = s.upload_mask();
        if (rc == AFMG_OK) rc = step(k, m);
        if (rc != AFMG_OK) return rc;
        k += m;
        for (int i = 0; i < n; i++) {
            Track &q = tr[(size_t)i];
            if (q.done) continue;
            afmg_stats &x = S[i];
            for (int c = 1; c < m; c++, x.cycles++)
                if (x.cycles < AFMG_HIST) x.hist_max[x.cycles] = x.hist_l2[x.cycles] = NAN;
            x.r_max = t->h_norm[2 * i];
            x.r_l2 = t->h_norm[2 * i + 1];
            if (x.cycles < AFMG_HIST) {
                x.hist_max[x.cycles] = x.r_max;
                x.hist_l2[x.cycles] = x.r_l2;
            }
            x.cycles++;
            if (!std::isfinite(x.r_max)) {
                x.status = AFMG_ERR_NONFINITE;
                q.done = true;
                continue;
            }
            if (!fixed) {
                q.grow = x.r_max > q.prev ? q.grow + 1 : 0;
                if (q.grow >= 3) {
                    x.status = AFMG_ERR_DIVERGED;
                    q.done = true;
                    continue;
                }
                q.conv = x.r_max <= o.tol * x.r0_max;
                if (q.conv) q.done = true;
            }
            q.prev = x.r_max;
        }
    }
    for (int i = 0; i < n; i++)
        if (S[i].status == AFMG_OK && !fixed && !tr[(size_t)i].conv) S[i].status = AFMG_NOT_CONVERGED;
    return AFMG_OK;
}

// Outer loop of a forest (batch).  Each tree's stop rule runs on the device
// after every cycle (k_tree_stop): a tree that stops leaves the mask and the
// compacted box lists, so it runs exactly the cycles of its own solve.  The
// host waits for the device only every check_every cycles (the cycles in
// between replay one recorded graph) and then reads the trees' states back:
// no per-cycle synchronisation or mask upload.  cycle(stream, first)
// enqueues one cycle, with the trees' norms into t->d_tnorm; first: the
// mixed path's FMG step, run eagerly as the first cycle.
template <int D, int N, class Cycle>
int iterate_forest(Solver<D, N> &s, afmg_stats *S, const std::vector<uintptr_t> &key, bool first_fmg, Cycle cycle) {
    afmg_tree *t = s.t;
    const afmg_opts &o = s.o;
    const HostTree &h = t->h;
    const int n = h.n_trees;
    const bool fixed = o.fixed_cycles > 0;
    const int nmax = fixed ? o.fixed_cycles : o.max_cycles;
    const int every = std::max(1, o.check_every);
    hipStream_t st = s.st;
    bool any = false;
    for (int i = 0; i < n; i++) {
        TreeStop &q = t->h_tstop[i];
        q = TreeStop{};
        q.status = S[i].status;
        q.prev = S[i].r_max;
        q.r0 = S[i].r0_max;
        q.rmax = S[i].r_max;
        q.rl2 = S[i].r_l2;
        q.conv = (!fixed && S[i].r_max <= o.tol * S[i].r0_max) ? 1 : 0;
        const bool go = q.status == AFMG_OK && !q.conv && nmax > 0;
        t->h_active[i] = go ? 1 : 0;
        any |= go;
    }
    hipError_t e = hipMemcpyAsync(t->d_tstop, t->h_tstop, sizeof(TreeStop) * (size_t)n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "tree state upload");
    if (s.upload_mask() != AFMG_OK) return AFMG_ERR_HIP;
    auto stop_and_compact = [&](hipStream_t cs) {
        launch_tree_stop(t->d_tnorm, t->d_active, t->d_tstop, t->d_thist, n, o.tol, fixed ? 1 : 0, nmax, cs);
        launch_compact(t->d_active, t->d_ltoff, t->d_lvloff, n, h.lmax, t->d_act, t->d_nact, cs);
    };
    launch_compact(t->d_active, t->d_ltoff, t->d_lvloff, n, h.lmax, t->d_act, t->d_nact, st);
    auto read = [&]() -> int {
        hipError_t err = hipMemcpyAsync(t->h_tstop, t->d_tstop, sizeof(TreeStop) * (size_t)n,
                                        hipMemcpyDeviceToHost, st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(t->h_active, t->d_active, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, st);
        if (err != hipSuccess) return hip_fail(err, "tree state readback");
        const int rc = s.read_norms();
        if (rc != AFMG_OK) return rc;
        any = false;
        for (int i = 0; i < n; i++) any |= t->h_active[i] != 0;
        return AFMG_OK;
    };
    int done = 0;  // cycles run by every tree still iterating
    if (any && first_fmg) {
        cycle(st, true);
        stop_and_compact(st);
        const int rc = read();
        if (rc != AFMG_OK) return rc;
        done = 1;
    }
    while (any) {
        const int m = std::max(1, std::min(every, nmax - done));
        std::vector<uintptr_t> km = key;
        km.push_back((uintptr_t)m);
        int rc = s.run(km, [&](hipStream_t cs) {
            for (int c = 0; c < m; c++) {
                cycle(cs, false);
                stop_and_compact(cs);
            }
        });
        if (rc == AFMG_OK) rc = read();
        if (rc != AFMG_OK) return rc;
        done += m;
    }
    e = hipMemcpyAsync(t->h_thist, t->d_thist, sizeof(double) * 2 * (size_t)n * AFMG_HIST, hipMemcpyDeviceToHost,
                       st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "tree history readback");
    for (int i = 0; i < n; i++) {
        const TreeStop &q = t->h_tstop[i];
        afmg_stats &x = S[i];
        x.cycles = q.cycles;
        x.status = q.status;
        if (q.cycles > 0) {
            x.r_max = q.rmax;
            x.r_l2 = q.rl2;
        }
        for (int c = 0; c < std::min(q.cycles, AFMG_HIST); c++) {
            x.hist_max[c] = t->h_thist[((size_t)i * 2 + 0) * AFMG_HIST + c];
            x.hist_l2[c] = t->h_thist[((size_t)i * 2 + 1) * AFMG_HIST + c];
        }
        if (x.status == AFMG_OK && !fixed && !q.conv) x.status = AFMG_NOT_CONVERGED;
    }
    return AFMG_OK;
}

// norms of the trees marked in t->h_active (all trees for one tree) from
// t->h_norm into the stats
void take_norms(const afmg_tree *t, afmg_stats *S, bool initial) {
    for (int i = 0; i < t->h.n_trees; i++) {
        if (t->forest && !t->h_active[i]) continue;
        if (initial) {
            S[i].r0_max = t->h_norm[2 * i];
            S[i].r0_l2 = t->h_norm[2 * i + 1];
        }
        S[i].r_max = t->h_norm[2 * i];
        S[i].r_l2 = t->h_norm[2 * i + 1];
    }
}

template <int D, int N>
int solve(afmg_tree *t, hipStream_t st, const double *rho, const double *bc, double *u, char *ws,
          const afmg_opts &o, afmg_stats *S) {
    const HostTree &h = t->h;
    const int n = h.n_trees;
    const bool mixed = o.precision == AFMG_MIXED;
    const WsLayout L = ws_layout(t, o.precision);
    Solver<D, N> s(t, st, o, &S[0]);
    if (o.profile && t->events.empty()) {
        t->events.resize(2 * PROF_PAIRS);
        for (auto &ev : t->events)
            if (hipEventCreate(&ev) != hipSuccess) return fail(AFMG_ERR_HIP, "hipEventCreate failed");
    }
    double *rho_i = (double *)(ws + L.rho);
    double *bc_w = (double *)(ws + L.bc);
    double *uw = t->forest ? (double *)(ws + L.u) : u;  // working u (colour-split)
    s.partial = (double *)(ws + L.partial);
    s.base = LevelArgs<double>{t->d_info, uw, rho_i, mixed ? nullptr : (double *)(ws + L.uold), bc_w, 0, 0, 0,
                               0.0, 0.0, t->d_active};
    s.base.eps = t->d_eps;
    s.base.bx = t->d_bx;
    s.base.opk = t->opk;
    s.base.dnbr = t->d_dnbr;
    const int64_t F = cells_per_face(D, N), C = cells_per_box(D, N);

    hipEvent_t ev0 = t->span[0], ev1 = t->span[1];
    (void)hipEventRecord(ev0, st);
    // Dirichlet rows: caller's leaf rows, then parent rows from fine to coarse
    if (h.n_bfaces_leaf > 0) {
        if (!bc) {
            launch_fill<double>(bc_w, h.n_bfaces_leaf * F, 0.0, st);
        } else if (t->forest) {
            launch_gather_rows(t->d_row_map, bc, bc_w, h.n_bfaces_leaf, (int)F, st);
        } else {
            hipError_t e = hipMemcpyAsync(bc_w, bc, (size_t)(h.n_bfaces_leaf * F) * sizeof(double),
                                          hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "copy of Dirichlet values");
        }
    }
    for (int l = h.lmax; l >= 2; l--)
        launch_bc_derive<D, N>(t->d_info, h.lvl_off[(size_t)l], h.level_count(l), bc_w, st);
    // working copies in the colour-split box layout: rho of the leaves, and
    // u (in place for one tree; a zero guess needs no conversion)
    const int32_t *map = t->forest ? t->d_box_map : nullptr;
    launch_load_rho<D, N, double>(t->d_info, map, rho, rho_i, h.n_boxes, 1, st);
    const bool guess = o.use_guess && (mixed || o.cycle == AFMG_CYCLE_V);
    if (!guess) launch_fill<double>(uw, h.n_boxes * C, 0.0, st);
    else if (t->forest) launch_load_rho<D, N, double>(t->d_info, map, u, uw, h.n_boxes, 0, st);
    else launch_permute<D, N, double>(t->d_info, u, 0, h.n_boxes, 1, 0, st);

    float *e32 = mixed ? (float *)(ws + L.e) : nullptr;
    float *rho32 = mixed ? (float *)(ws + L.rho_e) : nullptr;
    // initial residual of every tree
    if (t->forest)
        for (int i = 0; i < n; i++) t->h_active[i] = 1;
    int rc = s.upload_mask();
    if (t->forest) launch_compact(t->d_active, t->d_ltoff, t->d_lvloff, n, h.lmax, t->d_act, t->d_nact, st);
    if (rc == AFMG_OK) rc = s.finalize(rho32);
    if (rc != AFMG_OK) return rc;
    take_norms(t, S, true);
    bool any = false;
    for (int i = 0; i < n; i++) {
        if (!std::isfinite(S[i].r0_max)) S[i].status = AFMG_ERR_NONFINITE;
        any |= S[i].status == AFMG_OK;
        if (t->forest) t->h_active[i] = S[i].status == AFMG_OK;
    }
    std::vector<Track> tr((size_t)n);
    const uintptr_t wsk = (uintptr_t)ws, uk = (uintptr_t)uw;
    const std::vector<uintptr_t> key{(uintptr_t)o.precision, wsk, uk, (uintptr_t)o.n_down, (uintptr_t)o.n_up,
                                     (uintptr_t)o.n_base, (uintptr_t)t->tune_epoch, (uintptr_t)o.profile};
    if (!any) {
        // nothing to iterate
    } else if (!mixed) {
        Cycler<D, N, double> cy{h, st, o, s.prof, s.base, bc_w, t};
        cy.cg = (double *)(ws + L.cg);
        if (o.cycle == AFMG_CYCLE_FMG_V) {
            rc = s.upload_mask();
            if (rc != AFMG_OK) return rc;
            if (t->forest) cy.compact(t->d_active);
            cy.fmg(guess);  // without a guess u was zeroed above and is still zero
            s.finalize_launch(nullptr, st, h.lmin_leaf);
            if ((rc = s.read_norms()) != AFMG_OK) return rc;
            take_norms(t, S, false);
        }
        if (t->forest) {
            rc = iterate_forest(s, S, key, false, [&](hipStream_t cs, bool) {
                Cycler<D, N, double> c2 = cy;
                c2.st = cs;
                c2.vcycle(h.lmax);
                s.finalize_launch(nullptr, cs, h.lmin_leaf, t->d_tnorm);
            });
        } else {
            rc = iterate_trees(s, S, tr, [&](int, int m) {
                std::vector<uintptr_t> km = key;
                km.push_back((uintptr_t)m);
                const int q = s.run(km, [&](hipStream_t cs) {
                    Cycler<D, N, double> c2 = cy;
                    c2.st = cs;
                    for (int c = 0; c < m; c++) c2.vcycle(h.lmax);
                    s.finalize_launch(nullptr, cs, h.lmin_leaf);
                });
                return q != AFMG_OK ? q : s.read_norms();
            });
        }
    } else {
        // FP32 V-cycles inside FP64 iterative refinement: solve L e = r with
        // homogeneous Dirichlet values in FP32 (coarsest grids in FP64),
        // u += e on the leaves, new FP64 residual.  Each correction solve
        // starts from e = 0: the first from this fill (or FMG's own), the
        // others from the update, which clears e on the leaves it adds.  On
        // one tree whose leaves all lie on its complete finest level, the
        // update rides on the last half sweep of the correction's V-cycle,
        // which clears one colour of e; the next V-cycle's first half sweep
        // takes the other colour's old values as zero.
        LevelArgs<float> b32{t->d_info, e32, rho32, (float *)(ws + L.uold_e), nullptr, 0, 0, 1, 0.f, 0.f,
                             t->d_active};
        Cycler<D, N, float> cy{h, st, o, s.prof, b32, nullptr, t};
        cy.cg = (double *)(ws + L.cg);
        if (!t->forest && h.uniform && cube_xmask(h, h.lmax) != 0) cy.add_to = uw;
        if (o.cycle != AFMG_CYCLE_FMG_V) launch_fill<float>(e32, h.n_boxes * C, 0.f, st);
        auto refine = [&](hipStream_t cs, bool first_fmg) {
            Cycler<D, N, float> c2 = cy;
            c2.st = cs;
            if (first_fmg) {
                c2.fmg();
            } else {
                c2.zero_start = true;  // after the fill, or after a fused update
                c2.vcycle(h.lmax);
            }
            if (!c2.fuses_update(h.lmax))
                launch_ir_update<D, N>(t->d_info, uw, e32, h.n_boxes, t->d_active, cs);
            s.finalize_launch(rho32, cs, h.lmin_leaf, t->forest ? t->d_tnorm : nullptr);
        };
        if (t->forest) {
            rc = iterate_forest(s, S, key, o.cycle == AFMG_CYCLE_FMG_V,
                                [&](hipStream_t cs, bool first) { refine(cs, first); });
        } else {
            rc = iterate_trees(s, S, tr, [&](int k, int m) {
                int q = AFMG_OK;
                if (k == 0 && o.cycle == AFMG_CYCLE_FMG_V) {
                    for (int c = 0; c < m; c++) refine(st, c == 0);
                } else {
                    std::vector<uintptr_t> km = key;
                    km.push_back((uintptr_t)m);
                    q = s.run(km, [&](hipStream_t cs) {
                        for (int c = 0; c < m; c++) refine(cs, false);
                    });
                }
                return q != AFMG_OK ? q : s.read_norms();
            });
        }
    }
    if (rc != AFMG_OK) return rc;
    if (any) s.restrict_parents();
    if (t->forest) launch_store_boxes<D, N, double>(t->d_box_map, uw, u, h.n_boxes, st);
    else launch_permute<D, N, double>(t->d_info, u, 0, h.n_boxes, 0, 0, st);
    (void)hipEventRecord(ev1, st);
    (void)hipEventSynchronize(ev1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "solve");
    int status = AFMG_OK;
    for (int i = 0; i < n; i++) {
        S[i].t_ms = ms;
        S[i].bytes_model = (!t->forest && !t->opk && !mixed)
                               ? solve_bytes_model(h, S[i].cycles, o.cycle == AFMG_CYCLE_FMG_V, o.n_down, o.n_up)
                               : 0.0;
        if (S[i].status < 0 && status >= 0) status = S[i].status;
        if (S[i].status == AFMG_NOT_CONVERGED && status == AFMG_OK) status = AFMG_NOT_CONVERGED;
    }
    if (status == AFMG_ERR_NONFINITE) set_error("residual norm is not finite");
    if (status == AFMG_ERR_DIVERGED) set_error("residual grew for 3 consecutive cycles");
    if (status == AFMG_NOT_CONVERGED) set_error("max_cycles reached before the tolerance");
    return status;
}

// ---------------------------------------------------------------------------
// operator application and the adjoint solve
// ---------------------------------------------------------------------------
struct AdjLayout {
    // Krylov vectors and preconditioner arrays, each [n_boxes][N^D] FP64
    enum { X, R, RH, P, V, SV, T, PH, SH, B, PU, PRHO, NVEC };
    size_t vec[NVEC];
    size_t puold, bc, partial, norm, cg, total;
};

AdjLayout adj_layout(const afmg_tree *t) {
    const HostTree &h = t->h;
    const size_t C = (size_t)cells_per_box(h.dim, h.N), F = (size_t)cells_per_face(h.dim, h.N);
    const size_t nb = (size_t)h.n_boxes, nlt = (size_t)h.n_below_lmax();
    AdjLayout L{};
    size_t off = 0;
    for (int v = 0; v < AdjLayout::NVEC; v++) {
        L.vec[v] = off;
        off = align256(off + nb * C * sizeof(double));
    }
    L.puold = off; off = align256(off + nlt * C * sizeof(double));
    L.bc = off; off = align256(off + (size_t)std::max<int64_t>(1, h.n_bfaces_all) * F * sizeof(double));
    const size_t np = (size_t)std::max<int64_t>(t->n_parts_max, DOT_WGS);
    L.partial = off; off = align256(off + np * 2 * sizeof(double));
    L.norm = off; off = align256(off + 2 * sizeof(double));
    L.cg = off; off = align256(off + coarse_gen_bytes(h, t->opk));
    L.total = off;
    return L;
}

template <int D, int N>
struct Adj {
    afmg_tree *t;
    const HostTree &h;
    hipStream_t st;
    char *ws;
    AdjLayout L;
    int64_t n;  // values per field
    double *partial, *norm;

    double *vec(int v) const { return (double *)(ws + L.vec[v]); }

    // (max |a|, sum a b) over all cells; synchronises the stream
    int dot(const double *a, const double *b, double &mx, double &sum) {
        launch_dot(a, b, n, partial, norm, st);
        hipError_t e = hipMemcpyAsync(t->h_norm, norm, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "dot product");
        mx = t->h_norm[0];
        sum = t->h_norm[1];
        return AFMG_OK;
    }
    void apply_lt(const double *y, double *out) {
        launch_apply_lt<D, N>(t->d_info, t->d_child, y, out, h.n_boxes, st);
    }
    // x must be zero on parents; its restriction is written there first
    void apply_l(double *x, double *out) {
        for (int l = h.lmax; l >= 2; l--)
            launch_restrict_field<D, N>(t->d_info, x, h.lvl_off[(size_t)l], h.level_count(l), st);
        launch_apply_l<D, N>(t->d_info, x, out, h.n_boxes, st);
    }
};

template <int D, int N>
int apply_op(afmg_tree *t, hipStream_t st, int op, const double *x, double *y, char *ws) {
    const HostTree &h = t->h;
    Adj<D, N> A{t, h, st, ws, adj_layout(t), h.n_boxes * cells_per_box(D, N), nullptr, nullptr};
    double *X = A.vec(AdjLayout::X), *Y = A.vec(AdjLayout::R);
    launch_fill<double>(X, A.n, 0.0, st);
    launch_load_rho<D, N, double>(t->d_info, nullptr, x, X, h.n_boxes, 1, st);
    if (op == AFMG_OP_L) A.apply_l(X, Y);
    else A.apply_lt(X, Y);
    launch_store_leaves<D, N>(t->d_info, Y, y, h.n_boxes, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "operator application");
    return AFMG_OK;
}

// lambda = L^-T ubar on the leaf cells; rho_bar = lambda, bc_bar = -2 lambda / h^2
// on the leaf cells next to the Dirichlet rows.
template <int D, int N>
int adjoint(afmg_tree *t, hipStream_t st, const double *ubar, double *rho_bar, double *bc_bar, char *ws,
            const afmg_opts &o, afmg_stats &S) {
    const HostTree &h = t->h;
    Adj<D, N> A{t, h, st, ws, adj_layout(t), h.n_boxes * cells_per_box(D, N), nullptr, nullptr};
    A.partial = (double *)(ws + A.L.partial);
    A.norm = (double *)(ws + A.L.norm);
    double *X = A.vec(AdjLayout::X), *B = A.vec(AdjLayout::B);
    double *bcz = (double *)(ws + A.L.bc);
    const int64_t n = A.n, F = cells_per_face(D, N);
    hipEvent_t ev0 = t->span[0], ev1 = t->span[1];
    (void)hipEventRecord(ev0, st);
    // u_bar in the working layout; values on parent boxes (the restriction of
    // the leaves) are pushed to the leaves through the transposed restriction
    launch_copy<double>(ubar, B, n, st);
    launch_permute<D, N, double>(t->d_info, B, 0, h.n_boxes, 1, 0, st);
    for (int l = 2; l <= h.lmax; l++)
        launch_push_down<D, N>(t->d_info, B, h.lvl_off[(size_t)l], h.level_count(l), st);
    launch_scale_leaves<D, N>(t->d_info, B, B, 0, h.n_boxes, st);
    launch_fill<double>(bcz, std::max<int64_t>(1, h.n_bfaces_all) * F, 0.0, st);
    launch_fill<double>(X, n, 0.0, st);
    Solver<D, N> s(t, st, o, &S);
    s.partial = A.partial;
    int status = AFMG_OK, rc;
    if (h.uniform) {
        // the operator is symmetric: lambda solves L lambda = ubar with zero
        // Dirichlet values, one more multigrid solve
        s.base = LevelArgs<double>{t->d_info, X, B, (double *)(ws + A.L.puold), bcz, 0, 0, 1, 0.0, 0.0};
        Cycler<D, N, double> cy{h, st, o, s.prof, s.base, nullptr, t};
        cy.cg = (double *)(ws + A.L.cg);
        rc = s.finalize(S.r0_max, S.r0_l2, nullptr);
        if (rc != AFMG_OK) return rc;
        S.r_max = S.r0_max;
        S.r_l2 = S.r0_l2;
        status = iterate(o, S, [&](int) {
            cy.vcycle(h.lmax);
            return s.finalize(S.r_max, S.r_l2, nullptr);
        });
    } else {
        // L^T = V L* V^-1 with V = diag(h^D) and L* close to L away from
        // refinement boundaries, so M = V Vcycle(V^-1 .) approximates L^-T:
        // BiCGSTAB on L^T lambda = ubar, right-preconditioned with M
        double *R = A.vec(AdjLayout::R), *RH = A.vec(AdjLayout::RH), *P = A.vec(AdjLayout::P);
        double *Vv = A.vec(AdjLayout::V), *SV = A.vec(AdjLayout::SV), *T = A.vec(AdjLayout::T);
        double *PH = A.vec(AdjLayout::PH), *SH = A.vec(AdjLayout::SH);
        double *PU = A.vec(AdjLayout::PU), *PRHO = A.vec(AdjLayout::PRHO);
        LevelArgs<double> pb{t->d_info, PU, PRHO, (double *)(ws + A.L.puold), bcz, 0, 0, 1, 0.0, 0.0};
        Cycler<D, N, double> cy{h, st, o, s.prof, pb, nullptr, t};
        cy.cg = (double *)(ws + A.L.cg);
        auto precond = [&](const double *in, double *out) {
            launch_scale_leaves<D, N>(t->d_info, PRHO, in, -1, h.n_boxes, st);
            launch_fill<double>(PU, n, 0.0, st);
            cy.vcycle(h.lmax);
            launch_scale_leaves<D, N>(t->d_info, out, PU, +1, h.n_boxes, st);
        };
        launch_copy<double>(B, R, n, st);
        double mx, sum;
        if ((rc = A.dot(R, R, mx, sum)) != AFMG_OK) return rc;
        S.r0_max = mx;
        S.r0_l2 = std::sqrt(sum);
        S.r_max = mx;
        S.r_l2 = S.r0_l2;
        // BiCGSTAB judges convergence by its recursive residual; the true
        // residual u_bar - L^T lambda is computed afterwards, and where it
        // misses the tolerance the iteration restarts from it (twice at
        // most, within max_cycles iterations in all)
        for (int restart = 0;; restart++) {
            launch_copy<double>(R, RH, n, st);
            launch_fill<double>(P, n, 0.0, st);
            launch_fill<double>(Vv, n, 0.0, st);
            double rho_old = 1.0, alpha = 1.0, omega = 1.0;
            status = iterate(o, S, [&](int) -> int {
                double rho_new, dummy;
                int q;
                if ((q = A.dot(RH, R, dummy, rho_new)) != AFMG_OK) return q;
                if (rho_new == 0.0) return fail(AFMG_ERR_DIVERGED, "BiCGSTAB breakdown (rho = 0)");
                const double beta = (rho_new / rho_old) * (alpha / omega);
                launch_lc3(P, 1.0, R, beta, P, -beta * omega, Vv, n, st);
                precond(P, PH);
                A.apply_lt(PH, Vv);
                double rv;
                if ((q = A.dot(RH, Vv, dummy, rv)) != AFMG_OK) return q;
                if (rv == 0.0) return fail(AFMG_ERR_DIVERGED, "BiCGSTAB breakdown (r.v = 0)");
                alpha = rho_new / rv;
                launch_lc3(SV, 1.0, R, -alpha, Vv, 0.0, nullptr, n, st);
                precond(SV, SH);
                A.apply_lt(SH, T);
                double tt, ts;
                if ((q = A.dot(T, T, dummy, tt)) != AFMG_OK) return q;
                if ((q = A.dot(T, SV, dummy, ts)) != AFMG_OK) return q;
                omega = tt > 0.0 ? ts / tt : 0.0;
                launch_lc3(X, 1.0, X, alpha, PH, omega, SH, n, st);
                launch_lc3(R, 1.0, SV, -omega, T, 0.0, nullptr, n, st);
                double rs;
                if ((q = A.dot(R, R, S.r_max, rs)) != AFMG_OK) return q;
                S.r_l2 = std::sqrt(rs);
                rho_old = rho_new;
                if (omega == 0.0) return fail(AFMG_ERR_DIVERGED, "BiCGSTAB breakdown (omega = 0)");
                return AFMG_OK;
            });
            if (status < 0 && status != AFMG_ERR_NONFINITE && status != AFMG_ERR_DIVERGED) return status;
            // true residual of the result
            A.apply_lt(X, T);
            launch_lc3(T, 1.0, B, -1.0, T, 0.0, nullptr, n, st);
            double tmx, tsum;
            if ((rc = A.dot(T, T, tmx, tsum)) != AFMG_OK) return rc;
            S.r_max = tmx;
            S.r_l2 = std::sqrt(tsum);
            const bool fixed = o.fixed_cycles > 0;
            const bool missed = !(tmx <= o.tol * S.r0_max);
            if (status != AFMG_OK || fixed || !missed || restart == 2 || S.cycles >= o.max_cycles) {
                if (status == AFMG_OK && !fixed && missed) status = AFMG_NOT_CONVERGED;
                break;
            }
            launch_copy<double>(T, R, n, st);
        }
    }
    if (status < 0 && status != AFMG_ERR_NONFINITE && status != AFMG_ERR_DIVERGED) return status;
    launch_store_leaves<D, N>(t->d_info, X, rho_bar, h.n_boxes, st);
    if (bc_bar && h.n_bfaces_leaf > 0) launch_bc_grad<D, N>(t->d_info, X, bc_bar, h.n_boxes, st);
    (void)hipEventRecord(ev1, st);
    (void)hipEventSynchronize(ev1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    S.t_ms = ms;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint");
    S.status = status;
    if (status == AFMG_NOT_CONVERGED) set_error("max_cycles reached before the tolerance");
    if (status == AFMG_ERR_NONFINITE) set_error("residual norm is not finite");
    return status;
}

// ---------------------------------------------------------------------------
// one step of the cycle on caller arrays (kernel-by-kernel checks)
// ---------------------------------------------------------------------------
template <int D, int N>
int step(afmg_tree *t, hipStream_t st, int op, int level, int colour, int homog, double *u, double *rho,
         double *uold, const double *bc, char *ws, const afmg_opts &o) {
    const HostTree &h = t->h;
    const WsLayout L = ws_layout(t, AFMG_FP64);
    const int64_t F = cells_per_face(D, N);
    double *bc_w = (double *)(ws + L.bc);
    if (h.n_bfaces_leaf > 0) {
        if (bc) {
            hipError_t e = hipMemcpyAsync(bc_w, bc, (size_t)(h.n_bfaces_leaf * F) * sizeof(double),
                                          hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "copy of Dirichlet values");
        } else {
            launch_fill<double>(bc_w, h.n_bfaces_leaf * F, 0.0, st);
        }
    }
    for (int l = h.lmax; l >= 2; l--)
        launch_bc_derive<D, N>(t->d_info, h.lvl_off[(size_t)l], h.level_count(l), bc_w, st);
    for (double *f : {u, rho, uold}) launch_permute<D, N, double>(t->d_info, f, 0, h.n_boxes, 1, 0, st);
    LevelArgs<double> a{t->d_info, u, rho, uold, bc_w, h.lvl_off[(size_t)level], (int)h.level_count(level),
                        homog, 0.0, 0.0, nullptr, 0};
    a.xmask = cube_xmask(h, level);
    a.eps = t->d_eps;
    a.bx = t->d_bx;
    a.opk = t->opk;
    a.dnbr = t->d_dnbr;
    const double hh = level_h(level, N);
    a.h2 = hh * hh;
    a.ih2 = 1.0 / (hh * hh);
    a.h = hh;
    switch (op) {
    case AFMG_STEP_HALF_SWEEP: launch_level<D, N, double>(Op::GSRB, a, colour, 256, st); break;
    case AFMG_STEP_RESID_RESTRICT: launch_level<D, N, double>(Op::RESID_RESTRICT, a, 0, 256, st); break;
    case AFMG_STEP_COARSE_RHS: launch_level<D, N, double>(Op::COARSE_RHS, a, 0, 256, st); break;
    case AFMG_STEP_PROLONG: launch_level<D, N, double>(Op::PROLONG, a, 0, 256, st); break;
    default:
        if (coarse_general(h)) {
            CoarseGenArgs<double> c{t->d_info, u, rho, uold, homog ? nullptr : bc_w, (double *)(ws + L.cg),
                                    h.n_roots, COARSE_V_FROM_2, homog, o.n_down, o.n_up, o.n_base};
            c.eps = t->d_eps;
            c.bx = t->d_bx;
            c.opk = t->opk;
            c.dnbr = t->d_dnbr;
            launch_coarse_gen<D, N, double>(c, st);
        } else {
            CoarseArgs<double> c{t->d_info, u, rho, uold, homog ? nullptr : bc_w, COARSE_V_FROM_2, homog,
                                 o.n_down, o.n_up, o.n_base, nullptr};
            launch_coarse<D, N, double>(c, 1, st);
        }
    }
    for (double *f : {u, rho, uold}) launch_permute<D, N, double>(t->d_info, f, 0, h.n_boxes, 0, 0, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "step");
    return AFMG_OK;
}

// ---------------------------------------------------------------------------
// autotuning of the launch shapes
// ---------------------------------------------------------------------------
// Every candidate shape of one kernel class on one level is timed on the
// tree's own boxes (REPS launches between two events, best of two rounds);
// the fastest wins, the default (256 threads, XCD runs) unless another is at
// least TUNE_MARGIN faster.  Half sweeps alternate the colours as in a
// smoothing sweep (one colour repeated would find all its data in the
// caches).  The trials still run in other cache states than the solve's
// launches, and smaller measured gains did not carry over: on a level of
// 4096 boxes the three workgroup sizes timed within 5% of each other, and a
// 64-thread pick then ran 30% slower inside the solve.  Arrays are
// zero-filled scratch: timing does not depend on the values.
constexpr int TUNE_REPS = 10;
constexpr float TUNE_MARGIN = 0.10f;

template <class Fn>
float time_launches(hipStream_t st, hipEvent_t a, hipEvent_t b, Fn fn) {
    fn(1);  // warm-up
    (void)hipEventRecord(a, st);
    for (int r = 0; r < TUNE_REPS; r++) fn(r & 1);
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms / TUNE_REPS;
}

template <int D, int N, typename T>
void tune_precision(afmg_tree *t, hipStream_t st, LevelArgs<T> base, double *partial, hipEvent_t e0, hipEvent_t e1) {
    const HostTree &h = t->h;
    const int pi = sizeof(T) == 4 ? 1 : 0;
    for (int kind = 0; kind < SK_KINDS; kind++) {
        if (kind == SK_FINAL && pi == 1) continue;  // the residual is always FP64
        const int l0 = kind == SK_FINAL ? 1 : 2;
        const int l1 = kind == SK_CRHS ? h.lmax - 1 : h.lmax;
        for (int l = l0; l <= l1; l++) {
            if (h.level_count(l) == 0) continue;
            LevelArgs<T> a = base;
            a.b0 = h.lvl_off[(size_t)l];
            a.nb = (int)h.level_count(l);
            a.xmask = cube_xmask(h, l);
            const double hh = level_h(l, N);
            a.h2 = (T)(hh * hh);
            a.ih2 = (T)(1.0 / (hh * hh));
            a.h = (T)hh;
            if (t->forest) {
                a.act = t->d_act + h.lvl_off[(size_t)l];
                a.nact = t->d_nact + l;
            }
            const Op op = kind == SK_GSRB ? Op::GSRB
                          : kind == SK_RESID ? Op::RESID_RESTRICT
                          : kind == SK_CRHS ? Op::COARSE_RHS : Op::PROLONG;
            auto run = [&](const Shape &sh, int colour) {
                LevelArgs<T> b = a;
                b.no_remap = sh.no_remap;
                if (kind == SK_FINAL) {
                    const double hD = D == 3 ? hh * hh * hh : hh * hh;
                    launch_final<D, N, T>(b, partial, t->forest ? -1 : 0, hD, nullptr, sh.wg, st);
                } else {
                    launch_level<D, N, T>(op, b, colour, sh.wg, st);
                }
            };
            Shape best{};
            float t_def = 0.f, t_best = 0.f;
            for (int round = 0; round < 2; round++) {
                for (int wi = 0; wi < 3; wi++) {
                    if (SHAPE_WGS[wi] < cells_per_face(D, N)) continue;  // a workgroup holds whole boxes
                    for (int nr = 0; nr < 2; nr++) {
                        const Shape sh{SHAPE_WGS[wi], nr};
                        const float ms = time_launches(st, e0, e1, [&](int c) { run(sh, c); });
                        const bool is_def = wi == 0 && nr == 0;
                        if (round == 0 && is_def) {
                            t_def = ms;
                            t_best = ms;
                            best = sh;
                            continue;
                        }
                        if (is_def) t_def = std::min(t_def, ms);
                        if (ms < t_best) {
                            t_best = ms;
                            best = sh;
                        }
                    }
                }
            }
            if (!(t_best < (1.0f - TUNE_MARGIN) * t_def)) best = Shape{};
            t->shapes[pi][kind][(size_t)l] = best;
        }
    }
}

template <int D, int N>
int autotune(afmg_tree *t, hipStream_t st, char *ws) {
    const HostTree &h = t->h;
    const TuneLayout L = tune_layout(t);
    const int64_t C = cells_per_box(D, N), F = cells_per_face(D, N);
    const int64_t nb = h.n_boxes, nlt = std::max<int64_t>(1, h.n_below_lmax());
    double *u = (double *)(ws + L.u), *rho = (double *)(ws + L.rho), *uold = (double *)(ws + L.uold);
    double *bc = (double *)(ws + L.bc), *partial = (double *)(ws + L.partial);
    float *e = (float *)(ws + L.e), *re = (float *)(ws + L.rho_e), *uo = (float *)(ws + L.uold_e);
    launch_fill<double>(u, nb * C, 0.0, st);
    launch_fill<double>(rho, nb * C, 0.0, st);
    launch_fill<double>(uold, nlt * C, 0.0, st);
    launch_fill<double>(bc, std::max<int64_t>(1, h.n_bfaces_all) * F, 0.0, st);
    launch_fill<float>(e, nb * C, 0.f, st);
    launch_fill<float>(re, nb * C, 0.f, st);
    launch_fill<float>(uo, nlt * C, 0.f, st);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(AFMG_ERR_HIP, "hipEventCreate failed");
    LevelArgs<double> b64{t->d_info, u, rho, uold, bc, 0, 0, 0, 0.0, 0.0, nullptr, 0};
    LevelArgs<float> b32{t->d_info, e, re, uo, nullptr, 0, 0, 1, 0.f, 0.f, nullptr, 0};
    if (t->forest) {
        // the trials run every tree: lists of all boxes
        launch_level_mask(nullptr, t->d_tree_lmax, 1, t->d_mask, h.n_trees, st);
        launch_compact(t->d_mask, t->d_ltoff, t->d_lvloff, h.n_trees, h.lmax, t->d_act, t->d_nact, st);
        b64.active = t->d_mask;
        b32.active = t->d_mask;
    }
    tune_precision<D, N, double>(t, st, b64, partial, e0, e1);
    tune_precision<D, N, float>(t, st, b32, partial, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipError_t err = hipStreamSynchronize(st);
    if (err == hipSuccess) err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "autotune");
    compute_partials(t);
    t->tune_epoch++;
    return AFMG_OK;
}

int tree_autotune(afmg_tree *t, void *stream, void *workspace, size_t workspace_bytes) {
    if (!t || !workspace) return fail(AFMG_ERR_ARG, "null argument");
    if (t->opk) return fail(AFMG_ERR_ARG, "the autotuner covers the Laplacian's kernels");
    if (!aligned(workspace, 256)) return fail(AFMG_ERR_ARG, "misaligned array");
    if (workspace_bytes < tune_layout(t).total) return fail(AFMG_ERR_ARG, "workspace too small");
    int rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(t->h, autotune, (t, st, (char *)workspace));
}

int get_shape(const afmg_tree *t, int precision, int kind, int level, int *wg, int *no_remap) {
    if (!t || !wg || !no_remap) return fail(AFMG_ERR_ARG, "null argument");
    if (precision < 0 || precision > 1 || kind < 0 || kind >= SK_KINDS || level < 1 || level > t->h.lmax)
        return fail(AFMG_ERR_ARG, "shape index out of range");
    const Shape &sh = t->shapes[precision][kind][(size_t)level];
    *wg = sh.wg;
    *no_remap = sh.no_remap;
    return AFMG_OK;
}

int set_shape(afmg_tree *t, int precision, int kind, int level, int wg, int no_remap) {
    if (!t) return fail(AFMG_ERR_ARG, "null argument");
    if (t->opk && (wg != 256 || no_remap != 0))
        return fail(AFMG_ERR_ARG, "a tree with an operator set runs the default launch shapes");
    if (precision < -1 || precision > 1 || kind < -1 || kind >= SK_KINDS || level < -1 || level == 0 ||
        level > t->h.lmax || (wg != 64 && wg != 128 && wg != 256) || (no_remap != 0 && no_remap != 1))
        return fail(AFMG_ERR_ARG, "shape out of range");
    if (wg < cells_per_face(t->h.dim, t->h.N))
        return fail(AFMG_ERR_ARG, "a workgroup must hold whole boxes (one thread per row of cells)");
    for (int p = 0; p < 2; p++)
        for (int k = 0; k < SK_KINDS; k++)
            for (int l = 1; l <= t->h.lmax; l++)
                if ((precision < 0 || p == precision) && (kind < 0 || k == kind) && (level < 0 || l == level))
                    t->shapes[p][k][(size_t)l] = Shape{wg, no_remap};
    compute_partials(t);
    t->tune_epoch++;
    return AFMG_OK;
}

// device address of the current GPU's copy of `scratch`, looked up on the
// first call on that device
int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(AFMG_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
        if (!p || !aligned(p, 256)) return fail(AFMG_ERR_HIP, "scratch array has no aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AFMG_OK;
}

}  // namespace

// The operator's coefficients: the caller's eps (leaf boxes) in the
// colour-split layout, (volume) means into the parents, and a check that
// every leaf value is positive and finite.
template <int D, int N>
int load_eps(afmg_tree *t, hipStream_t st, const double *eps, int opk, int *flag) {
    const HostTree &h = t->h;
    launch_load_rho<D, N, double>(t->d_info, nullptr, eps, t->d_eps, h.n_boxes, 1, st);
    for (int l = h.lmax; l >= 2; l--)
        launch_restrict_field_op<D, N>(t->d_info, t->d_eps, h.lvl_off[(size_t)l], h.level_count(l), opk, t->d_bx,
                                           level_h(l, N), st);
    launch_fill<int>(flag, 1, 0, st);
    launch_check_positive<D, N>(t->d_info, t->d_eps, h.n_boxes, flag, st);
    int bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "eps");
    if (bad) return fail(AFMG_ERR_ARG, "eps must be positive and finite on every leaf cell");
    return AFMG_OK;
}

// Workspace of afmg_tree_transfer: the from-tree's field (colour-split, with
// its parents), its boundary rows with the derived parent rows, and the
// box lists of the transfer.
struct XferLayout {
    size_t u, bc, lists, total;
};
XferLayout xfer_layout(const afmg_tree *from, const afmg_tree *to) {
    const size_t C = (size_t)cells_per_box(from->h.dim, from->h.N), F = (size_t)cells_per_face(from->h.dim, from->h.N);
    XferLayout L{};
    size_t off = 0;
    L.u = off; off = align256(off + (size_t)from->h.n_boxes * C * sizeof(double));
    L.bc = off; off = align256(off + (size_t)std::max<int64_t>(1, from->h.n_bfaces_all) * F * sizeof(double));
    L.lists = off; off = align256(off + (size_t)std::max<int64_t>(1, to->h.n_boxes) * 4 * sizeof(int32_t));
    L.total = off;
    return L;
}

template <int D, int N>
int transfer(afmg_tree *from, afmg_tree *to, hipStream_t st, const double *u_from, const double *bc, double *u_to,
             char *ws) {
    const HostTree &hf = from->h, &ht = to->h;
    const XferLayout L = xfer_layout(from, to);
    const int64_t C = cells_per_box(D, N), F = cells_per_face(D, N);
    // the box lists: a leaf of `to` that is a box of `from` takes its values
    // (the mean of its children if it was refined there); a new leaf is
    // prolonged from its parent, a leaf of `from`.  Both trees hold each level
    // in increasing Morton order, so one merge per level finds the boxes.
    std::vector<uint64_t> kf((size_t)hf.n_boxes);
    for (int64_t m = 0; m < hf.n_boxes; m++) kf[(size_t)m] = box_morton(hf, m);
    std::vector<int32_t> cdst, csrc, pdst, psrc;
    for (int l = 1; l <= ht.lmax; l++) {
        int64_t a = l <= hf.lmax ? hf.lvl_off[(size_t)l] : 0, a_end = l <= hf.lmax ? hf.lvl_off[(size_t)l + 1] : 0;
        int64_t p = l - 1 >= 1 && l - 1 <= hf.lmax ? hf.lvl_off[(size_t)l - 1] : 0;
        const int64_t p_end = l - 1 >= 1 && l - 1 <= hf.lmax ? hf.lvl_off[(size_t)l] : 0;
        for (int64_t m = ht.lvl_off[(size_t)l]; m < ht.lvl_off[(size_t)l + 1]; m++) {
            if (!(ht.info[(size_t)m].flags & FLAG_LEAF)) continue;
            const uint64_t km = box_morton(ht, m);
            while (a < a_end && kf[(size_t)a] < km) a++;
            if (a < a_end && kf[(size_t)a] == km) {
                cdst.push_back((int32_t)m);
                csrc.push_back((int32_t)a);
                continue;
            }
            const uint64_t kp = km >> D;
            while (p < p_end && kf[(size_t)p] < kp) p++;
            if (p >= p_end || kf[(size_t)p] != kp || !(hf.info[(size_t)p].flags & FLAG_LEAF))
                return fail(AFMG_ERR_ARG, "a leaf of the target lies two or more levels below the source's leaves");
            pdst.push_back((int32_t)m);
            psrc.push_back((int32_t)p);
        }
    }
    int32_t *lists = (int32_t *)(ws + L.lists);
    std::vector<int32_t> all;
    all.reserve(2 * (size_t)ht.n_boxes);
    all.insert(all.end(), cdst.begin(), cdst.end());
    all.insert(all.end(), csrc.begin(), csrc.end());
    all.insert(all.end(), pdst.begin(), pdst.end());
    all.insert(all.end(), psrc.begin(), psrc.end());
    hipError_t e = hipMemcpyAsync(lists, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "transfer lists");
    const int64_t nc = (int64_t)cdst.size(), np = (int64_t)pdst.size();
    // the from-field with its parents, and its boundary rows
    double *uf = (double *)(ws + L.u), *bc_w = (double *)(ws + L.bc);
    launch_load_rho<D, N, double>(from->d_info, nullptr, u_from, uf, hf.n_boxes, 1, st);
    for (int l = hf.lmax; l >= 2; l--)
        launch_restrict_field<D, N>(from->d_info, uf, hf.lvl_off[(size_t)l], hf.level_count(l), st);
    if (hf.n_bfaces_leaf > 0 && bc) {
        e = hipMemcpyAsync(bc_w, bc, (size_t)(hf.n_bfaces_leaf * F) * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "copy of boundary values");
        for (int l = hf.lmax; l >= 2; l--)
            launch_bc_derive<D, N>(from->d_info, hf.lvl_off[(size_t)l], hf.level_count(l), bc_w, st);
    }
    launch_transfer<D, N>(to->d_info, from->d_info, lists, lists + nc, nc, lists + 2 * nc, lists + 2 * nc + np, np,
                              uf, bc_w, bc ? 0 : 1, u_to, st);
    for (int l = ht.lmax; l >= 2; l--)
        launch_restrict_field<D, N>(to->d_info, u_to, ht.lvl_off[(size_t)l], ht.level_count(l), st);
    launch_permute<D, N, double>(to->d_info, u_to, 0, ht.n_boxes, 0, 0, st);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host lists above must outlive their copy
    if (e != hipSuccess) return hip_fail(e, "transfer");
    (void)C;
    return AFMG_OK;
}

// The kernel bits of a tree's operator, prolongation and ghost scheme; a
// tree with any of them takes the operator kernels, the general coarse path
// and the default launch shapes (one norm partial per 256-thread workgroup).
int apply_schemes(afmg_tree *t) {
    HostTree &h = t->h;
    int opk = 0;
    if (t->op_kind & AFMG_OPERATOR_EPS) opk |= OPK_EPS;
    if (t->op_kind & AFMG_OPERATOR_CYL) opk |= OPK_CYL;
    if (t->op_prolong == AFMG_PROLONG_EPS) opk |= OPK_PROLONG_EPS;
    if (t->op_prolong == AFMG_PROLONG_LINEAR) opk |= OPK_PROLONG_LIN;
    if (t->ghost_scheme == AFMG_GHOST_BILINEAR) opk |= OPK_GHOST_BIL;
    t->rec.drop();  // a recorded cycle holds the old launches
    t->opk = opk;
    h.general = opk != 0 || (t->domain_general >= 0 ? t->domain_general != 0 : h.general);
    if (opk) {
        for (auto &pk : t->shapes)
            for (auto &v : pk) v.assign((size_t)h.lmax + 2, Shape{});
        t->tune_epoch++;
    }
    compute_partials(t);  // the norm partials follow the final kernel's workgroups
    return AFMG_OK;
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

void afmg_default_opts(afmg_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->cycle = AFMG_CYCLE_V;
    o->n_down = 2;
    o->n_up = 2;
    o->n_base = 4;
    o->tol = 1e-10;
    o->max_cycles = 100;
    o->fixed_cycles = 0;
    o->use_guess = 0;
    o->precision = AFMG_FP64;
    o->profile = 0;
    o->prof_level = 0;
    o->graph = 0;
    o->check_every = 1;
}

int afmg_tree_create_domain(int dim, int box_n, const int32_t *bc_type, int64_t n_leaves, const int32_t *level,
                            const int32_t *idx, afmg_tree **out) {
    if (!out) return fail(AFMG_ERR_ARG, "out is null");
    *out = nullptr;
    afmg_tree *t = nullptr;
    try {
        t = new afmg_tree();
        std::string msg;
        const int64_t off[2] = {0, n_leaves};
        int rc = build_tree(dim, box_n, 1, off, level, idx, t->h, msg, bc_type);
        if (rc != AFMG_OK) {
            delete t;
            return fail(rc, msg);
        }
        compute_partials(t);
    } catch (const std::bad_alloc &) {
        delete t;
        return fail(AFMG_ERR_OOM, "host allocation failed");
    }
    *out = t;
    return AFMG_OK;
}

int afmg_tree_create(int dim, int box_n, int64_t n_leaves, const int32_t *level, const int32_t *idx,
                     afmg_tree **out) {
    if (!out) return fail(AFMG_ERR_ARG, "out is null");
    *out = nullptr;
    if (!level || !idx || n_leaves <= 0) return fail(AFMG_ERR_ARG, "empty or null leaf list");
    // one level-1 box at (1, 1, 1): every leaf index within 2^(level - 1)
    for (int64_t q = 0; q < n_leaves; q++) {
        const int l = level[q];
        if (l < 1 || l > 30) return fail(AFMG_ERR_ARG, "leaf level out of range");
        for (int d = 0; d < (dim == 3 ? 3 : 2); d++)
            if (idx[3 * q + d] > (1 << (l - 1))) return fail(AFMG_ERR_ARG, "leaf spatial index out of range");
    }
    return afmg_tree_create_domain(dim, box_n, nullptr, n_leaves, level, idx, out);
}

void afmg_tree_destroy(afmg_tree *t) {
    if (!t) return;
    release(t);
    delete t;
}

int afmg_tree_info(const afmg_tree *t, afmg_tree_desc *out) {
    if (!t || !out) return fail(AFMG_ERR_ARG, "null argument");
    const HostTree &h = t->h;
    out->dim = h.dim;
    out->box_n = h.N;
    out->n_boxes = h.n_boxes;
    out->n_leaves = h.n_leaves;
    out->n_bfaces = h.n_bfaces_leaf;
    out->lmin = h.lmin;
    out->lmax = h.lmax;
    out->cells_per_box = cells_per_box(h.dim, h.N);
    out->n_unknowns = h.n_leaves * cells_per_box(h.dim, h.N);
    out->n_roots = h.n_roots;
    for (int d = 0; d < 3; d++) out->ext[d] = h.ext[d];
    for (int s = 0; s < 6; s++) out->bc_type[s] = h.bc_type[s];
    out->singular = h.singular ? 1 : 0;
    out->op = t->op_kind;
    out->prolong = t->op_prolong;
    out->ghost = t->ghost_scheme;
    return AFMG_OK;
}

int afmg_tree_leaf_boxes(const afmg_tree *t, int32_t *out) {
    if (!t || !out) return fail(AFMG_ERR_ARG, "null argument");
    std::memcpy(out, t->h.leaf_box.data(), sizeof(int32_t) * t->h.leaf_box.size());
    return AFMG_OK;
}

int afmg_tree_bfaces(const afmg_tree *t, int32_t *out) {
    if (!t || !out) return fail(AFMG_ERR_ARG, "null argument");
    for (int64_t f = 0; f < t->h.n_bfaces_leaf; f++) {
        out[2 * f] = t->h.bface_box[(size_t)f];
        out[2 * f + 1] = t->h.bface_side[(size_t)f];
    }
    return AFMG_OK;
}

int afmg_tree_box(const afmg_tree *t, int64_t b, afmg_box_desc *out) {
    if (!t || !out) return fail(AFMG_ERR_ARG, "null argument");
    if (b < 0 || b >= t->h.n_boxes) return fail(AFMG_ERR_ARG, "box id out of range");
    const BoxInfo &bi = t->h.info[(size_t)b];
    out->level = bi.level;
    out->idx[0] = t->h.ix[(size_t)b];
    out->idx[1] = t->h.iy[(size_t)b];
    out->idx[2] = t->h.iz[(size_t)b];
    out->parent = bi.parent;
    out->leaf = bi.flags & FLAG_LEAF;
    for (int s = 0; s < 6; s++) out->nbr[s] = s < 2 * t->h.dim ? bi.nbr[s] : -1;
    for (int c = 0; c < 8; c++) out->children[c] = c < (1 << t->h.dim) ? t->h.child[(size_t)b * 8 + c] : -1;
    const double h = level_h(bi.level, t->h.N);
    out->h = h;
    out->x_lo[0] = (out->idx[0] - 1) * t->h.N * h;
    out->x_lo[1] = (out->idx[1] - 1) * t->h.N * h;
    out->x_lo[2] = t->h.dim == 3 ? (out->idx[2] - 1) * t->h.N * h : 0.0;
    return AFMG_OK;
}

int afmg_tree_refine(const afmg_tree *t, const int32_t *ids, int64_t n, int balance, afmg_tree **out) {
    if (!t || !out) return fail(AFMG_ERR_ARG, "null argument");
    *out = nullptr;
    if (t->forest) return fail(AFMG_ERR_ARG, "not a tree");
    try {
        std::vector<int32_t> level, idx;
        std::string msg;
        const int rc = refine_leaves(t->h, ids, n, balance, level, idx, msg);
        if (rc != AFMG_OK) return fail(rc, msg);
        // the domain's own kind (an operator makes the solve take the general
        // path, but the new tree starts with the Laplacian)
        const bool general = t->domain_general >= 0 ? t->domain_general != 0 : t->h.general;
        return afmg_tree_create_domain(t->h.dim, t->h.N, general ? t->h.bc_type : nullptr,
                                       (int64_t)level.size(), level.data(), idx.data(), out);
    } catch (const std::bad_alloc &) {
        return fail(AFMG_ERR_OOM, "host allocation failed");
    }
}

int afmg_tree_adapt(afmg_tree *t, void *stream, const int8_t *flags, int n_buf, afmg_tree **out, int64_t *counts) {
    if (!t || !flags || !out) return fail(AFMG_ERR_ARG, "null argument");
    *out = nullptr;
    if (t->forest) return fail(AFMG_ERR_ARG, "not a tree");
    if (n_buf < 0 || n_buf > t->h.N) return fail(AFMG_ERR_ARG, "n_buf must lie in [0, box_n]");
    int rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    const HostTree &h = t->h;
    hipStream_t st = (hipStream_t)stream;
    try {
        std::vector<int32_t> words((size_t)h.n_boxes);
        int32_t *d_words = nullptr;
        hipError_t e = hipMalloc(&d_words, sizeof(int32_t) * words.size());
        if (e != hipSuccess) return fail(AFMG_ERR_OOM, "hipMalloc of the box words failed");
        AFMG_BOX_DISPATCH(h, launch_box_flags, (t->d_info, flags, h.n_boxes, n_buf, d_words, st));
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(words.data(), d_words, sizeof(int32_t) * words.size(),
                                                hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(d_words);
        if (e != hipSuccess) return hip_fail(e, "cell flags");
        std::vector<int32_t> level, idx;
        std::string msg;
        int64_t cnt[2] = {0, 0};
        rc = adapt_leaves(h, words.data(), level, idx, cnt, msg);
        if (rc != AFMG_OK) return fail(rc, msg);
        if (counts) {
            counts[0] = cnt[0];
            counts[1] = cnt[1];
        }
        const bool general = t->domain_general >= 0 ? t->domain_general != 0 : h.general;
        return afmg_tree_create_domain(h.dim, h.N, general ? h.bc_type : nullptr, (int64_t)level.size(),
                                       level.data(), idx.data(), out);
    } catch (const std::bad_alloc &) {
        return fail(AFMG_ERR_OOM, "host allocation failed");
    }
}

int afmg_transfer_workspace_bytes(const afmg_tree *from, const afmg_tree *to, size_t *bytes) {
    if (!from || !to || !bytes) return fail(AFMG_ERR_ARG, "null argument");
    *bytes = xfer_layout(from, to).total;
    return AFMG_OK;
}

int afmg_tree_transfer(afmg_tree *from, afmg_tree *to, void *stream, const double *u_from, const double *bc_from,
                       double *u_to, void *workspace, size_t workspace_bytes) {
    if (!from || !to || !u_from || !u_to || !workspace) return fail(AFMG_ERR_ARG, "null argument");
    if (from->forest || to->forest) return fail(AFMG_ERR_ARG, "not a tree");
    const HostTree &a = from->h, &b = to->h;
    bool same = a.dim == b.dim && a.N == b.N && a.n_roots == b.n_roots;
    for (int d = 0; d < 3; d++) same = same && a.ext[d] == b.ext[d];
    for (int s = 0; s < 6; s++) same = same && a.bc_type[s] == b.bc_type[s];
    if (!same) return fail(AFMG_ERR_ARG, "the trees must share the domain");
    if (!aligned(u_from, 8) || !aligned(u_to, 8) || (bc_from && !aligned(bc_from, 8)) || !aligned(workspace, 256))
        return fail(AFMG_ERR_ARG, "misaligned array");
    if (workspace_bytes < xfer_layout(from, to).total) return fail(AFMG_ERR_ARG, "workspace too small");
    int rc = bind_device(from);
    if (rc == AFMG_OK) rc = bind_device(to);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    try {
        AFMG_BOX_RETURN(a, transfer, (from, to, st, u_from, bc_from, u_to, (char *)workspace));
    } catch (const std::bad_alloc &) {
        return fail(AFMG_ERR_OOM, "host allocation failed");
    }
}

int afmg_tree_set_operator(afmg_tree *t, void *stream, int op, const double *eps, int prolong) {
    if (!t) return fail(AFMG_ERR_ARG, "null tree");
    if (t->forest) return fail(AFMG_ERR_ARG, "not a tree");
    if (op < AFMG_OPERATOR_LAPLACIAN || op > AFMG_OPERATOR_CYL_EPS) return fail(AFMG_ERR_ARG, "bad operator");
    if (prolong < AFMG_PROLONG_DEFAULT || prolong > AFMG_PROLONG_LINEAR) return fail(AFMG_ERR_ARG, "bad prolongation");
    const bool has_eps = op & AFMG_OPERATOR_EPS;
    if ((op & AFMG_OPERATOR_CYL) && t->h.dim != 2) return fail(AFMG_ERR_ARG, "the cylindrical form is 2D (r, z)");
    if (prolong == AFMG_PROLONG_EPS && !has_eps) return fail(AFMG_ERR_ARG, "the eps prolongation needs eps");
    if (has_eps && !eps) return fail(AFMG_ERR_ARG, "eps is null");
    if (eps && !aligned(eps, 8)) return fail(AFMG_ERR_ARG, "misaligned array");
    int rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    HostTree &h = t->h;
    if (t->domain_general < 0) t->domain_general = h.general ? 1 : 0;
    const int opk = (has_eps ? OPK_EPS : 0) | ((op & AFMG_OPERATOR_CYL) ? OPK_CYL : 0);
    t->op_kind = 0;
    t->op_prolong = 0;
    if ((rc = apply_schemes(t)) != AFMG_OK) return rc;
    const size_t C = (size_t)cells_per_box(h.dim, h.N);
    if (opk && !t->d_bx && (rc = upload(t->d_bx, h.ix, "the box x indices")) != AFMG_OK) return rc;
    if (prolong == AFMG_PROLONG_LINEAR && !t->d_dnbr) {
        std::vector<int32_t> dn;
        diagonal_neighbours(h, dn);
        if ((rc = upload(t->d_dnbr, dn, "the diagonal neighbours")) != AFMG_OK) return rc;
    }
    if (has_eps) {
        if (!t->d_eps) {
            // the coefficients, then one word for the check's flag
            hipError_t e = hipMalloc(&t->d_eps, sizeof(double) * ((size_t)h.n_boxes * C + 1));
            if (e != hipSuccess) {
                t->d_eps = nullptr;
                return fail(AFMG_ERR_OOM, "hipMalloc of the coefficients failed");
            }
        }
        hipStream_t st = (hipStream_t)stream;
        int *flag = (int *)(t->d_eps + (size_t)h.n_boxes * C);
        AFMG_BOX_DISPATCH(h, rc = load_eps, (t, st, eps, opk, flag));
        if (rc != AFMG_OK) return rc;
    }
    t->op_kind = op;
    t->op_prolong = prolong;
    return apply_schemes(t);
}

int afmg_tree_set_ghost_scheme(afmg_tree *t, void *stream, int scheme) {
    (void)stream;
    if (!t) return fail(AFMG_ERR_ARG, "null tree");
    if (t->forest) return fail(AFMG_ERR_ARG, "not a tree");
    if (scheme != AFMG_GHOST_DEFAULT && scheme != AFMG_GHOST_BILINEAR) return fail(AFMG_ERR_ARG, "bad ghost scheme");
    int rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    if (t->domain_general < 0) t->domain_general = t->h.general ? 1 : 0;
    t->ghost_scheme = scheme;
    return apply_schemes(t);
}

int afmg_tree_finalize(afmg_tree *t, void *stream) {
    (void)stream;
    if (!t) return fail(AFMG_ERR_ARG, "null argument");
    return bind_device(t);
}

int afmg_tree_level_list(const afmg_tree *t, int level, int kind, int32_t *ids, int64_t *n) {
    if (!t || !n) return fail(AFMG_ERR_ARG, "null argument");
    if (level < 1 || level > t->h.lmax || kind < AFMG_LIST_ALL || kind > AFMG_LIST_LEAF)
        return fail(AFMG_ERR_ARG, "level or kind out of range");
    int64_t c = 0;
    for (int64_t b = t->h.lvl_off[(size_t)level]; b < t->h.lvl_off[(size_t)level + 1]; b++) {
        const bool leaf = t->h.info[(size_t)b].flags & FLAG_LEAF;
        if (kind == AFMG_LIST_ALL || (kind == AFMG_LIST_LEAF) == leaf) {
            if (ids) ids[c] = (int32_t)b;
            c++;
        }
    }
    *n = c;
    return AFMG_OK;
}

int afmg_workspace_bytes(const afmg_tree *t, const afmg_opts *o, size_t *bytes) {
    if (!t || !bytes) return fail(AFMG_ERR_ARG, "null argument");
    if (o) {
        int rc = check_opts(o);
        if (rc != AFMG_OK) return rc;
    }
    *bytes = ws_layout(t, o ? o->precision : AFMG_FP64).total;
    return AFMG_OK;
}

int afmg_solve_bytes_model(const afmg_tree *t, const afmg_opts *opts, int v_cycles, double *bytes) {
    if (!t || !bytes || v_cycles < 0) return fail(AFMG_ERR_ARG, "null argument or negative cycle count");
    if (t->forest || t->opk) return fail(AFMG_ERR_ARG, "the byte model covers one tree with the Laplacian");
    afmg_opts o;
    afmg_default_opts(&o);
    if (opts) o = *opts;
    *bytes = solve_bytes_model(t->h, v_cycles, o.cycle == AFMG_CYCLE_FMG_V, o.n_down, o.n_up);
    return AFMG_OK;
}

int afmg_adjoint_workspace_bytes(const afmg_tree *t, const afmg_opts *o, size_t *bytes) {
    if (!t || !bytes) return fail(AFMG_ERR_ARG, "null argument");
    if (o) {
        int rc = check_opts(o);
        if (rc != AFMG_OK) return rc;
    }
    *bytes = adj_layout(t).total;
    return AFMG_OK;
}

int afmg_apply(afmg_tree *t, void *stream, int op, const double *x, double *y, void *workspace,
               size_t workspace_bytes) {
    if (!t || !x || !y || !workspace) return fail(AFMG_ERR_ARG, "null argument");
    if (op != AFMG_OP_L && op != AFMG_OP_LT) return fail(AFMG_ERR_ARG, "bad operator");
    if (t->opk) return fail(AFMG_ERR_ARG, "afmg_apply covers the Laplacian only");
    if (!aligned(x, 8) || !aligned(y, 8) || !aligned(workspace, 256)) return fail(AFMG_ERR_ARG, "misaligned array");
    if (workspace_bytes < adj_layout(t).total) return fail(AFMG_ERR_ARG, "workspace too small");
    int rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(t->h, apply_op, (t, st, op, x, y, (char *)workspace));
}

int afmg_adjoint(afmg_tree *t, void *stream, const double *u_bar, double *rho_bar, double *bc_bar,
                 void *workspace, size_t workspace_bytes, const afmg_opts *opts, afmg_stats *stats) {
    if (!t || !u_bar || !rho_bar || !workspace || !stats) return fail(AFMG_ERR_ARG, "null argument");
    int rc = check_opts(opts);
    if (rc != AFMG_OK) return rc;
    if (!aligned(u_bar, 8) || !aligned(rho_bar, 8) || (bc_bar && !aligned(bc_bar, 8)) || !aligned(workspace, 256))
        return fail(AFMG_ERR_ARG, "misaligned array");
    if (workspace_bytes < adj_layout(t).total) return fail(AFMG_ERR_ARG, "workspace too small");
    if (t->h.singular)
        return fail(AFMG_ERR_ARG, "afmg_adjoint: without a Dirichlet side the operator is singular");
    if (t->opk) return fail(AFMG_ERR_ARG, "afmg_adjoint covers the Laplacian only");
    std::memset(stats, 0, sizeof(*stats));
    rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(t->h, adjoint, (t, st, u_bar, rho_bar, bc_bar, (char *)workspace, *opts, *stats));
}

int afmg_solve(afmg_tree *t, void *stream, const double *rho, const double *bc, double *u,
               void *workspace, size_t workspace_bytes, const afmg_opts *opts, afmg_stats *stats) {
    if (!t || !rho || !u || !workspace || !stats) return fail(AFMG_ERR_ARG, "null argument");
    int rc = check_opts(opts);
    if (rc != AFMG_OK) return rc;
    if (!aligned(rho, 8) || !aligned(u, 8) || (bc && !aligned(bc, 8)) || !aligned(workspace, 256))
        return fail(AFMG_ERR_ARG, "misaligned array");
    const WsLayout L = ws_layout(t, opts->precision);
    if (workspace_bytes < L.total) return fail(AFMG_ERR_ARG, "workspace too small");
    if (t->opk && opts->precision != AFMG_FP64)
        return fail(AFMG_ERR_ARG, "a tree with an operator set solves in FP64");
    std::memset(stats, 0, sizeof(*stats));
    rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(t->h, solve, (t, st, rho, bc, u, (char *)workspace, *opts, stats));
}

int afmg_solve_noalloc(afmg_tree *t, void *stream, const double *rho, const double *bc, double *u,
                       const afmg_opts *opts, afmg_stats *stats) {
    if (!t || !rho || !u || !stats) return fail(AFMG_ERR_ARG, "null argument");
    if (t->forest) return fail(AFMG_ERR_ARG, "not a tree");
    int rc = check_opts(opts);
    if (rc != AFMG_OK) return rc;
    if (opts->graph || opts->profile)
        return fail(AFMG_ERR_ARG, "afmg_solve_noalloc: graph recording and profiling allocate; set both to 0");
    if (!aligned(rho, 8) || !aligned(u, 8) || (bc && !aligned(bc, 8))) return fail(AFMG_ERR_ARG, "misaligned array");
    const size_t need = ws_layout(t, opts->precision).total;
    if (need > AFMG_SCRATCH_BYTES)
        return fail(AFMG_ERR_ARG, "afmg_solve_noalloc: the tree needs " + std::to_string(need) +
                                      " bytes of workspace, more than the " + std::to_string(AFMG_SCRATCH_BYTES) +
                                      " of the scratch array; use afmg_solve with a caller workspace");
    if (t->device < 0) return fail(AFMG_ERR_ARG, "afmg_solve_noalloc: prepare the tree first (afmg_tree_finalize)");
    if (t->opk && opts->precision != AFMG_FP64)
        return fail(AFMG_ERR_ARG, "a tree with an operator set solves in FP64");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (t->device != dev) return fail(AFMG_ERR_ARG, "tree was first used on another device");
    void *ws = nullptr;
    if ((rc = scratch_address(dev, &ws)) != AFMG_OK) return rc;
    std::memset(stats, 0, sizeof(*stats));
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(t->h, solve, (t, st, rho, bc, u, (char *)ws, *opts, stats));
}

int afmg_batch_create(afmg_tree *const *trees, int n_trees, afmg_batch **out) {
    if (!out) return fail(AFMG_ERR_ARG, "out is null");
    *out = nullptr;
    if (!trees || n_trees < 1) return fail(AFMG_ERR_ARG, "empty batch");
    for (int i = 0; i < n_trees; i++) {
        if (!trees[i]) return fail(AFMG_ERR_ARG, "null tree");
        if (trees[i]->forest) return fail(AFMG_ERR_ARG, "not a tree");
        if (trees[i]->h.general)
            return fail(AFMG_ERR_ARG, "batches take trees of one level-1 box with Dirichlet sides");
        if (trees[i]->opk) return fail(AFMG_ERR_ARG, "batches take trees with the Laplacian");
        if (trees[i]->h.dim != trees[0]->h.dim || trees[i]->h.N != trees[0]->h.N)
            return fail(AFMG_ERR_ARG, "trees of one batch must share dim and box_n");
    }
    afmg_batch *b = nullptr;
    try {
        b = new afmg_batch();
        afmg_tree &f = b->f;
        const int dim = trees[0]->h.dim;
        // the trees' leaves, each tree in its own input order
        std::vector<int64_t> off((size_t)n_trees + 1, 0), box_base((size_t)n_trees), row_base((size_t)n_trees);
        for (int i = 0; i < n_trees; i++) {
            const HostTree &h = trees[i]->h;
            off[(size_t)i + 1] = off[(size_t)i] + h.n_leaves;
            box_base[(size_t)i] = f.user_boxes;
            row_base[(size_t)i] = f.user_rows;
            f.user_boxes += h.n_boxes;
            f.user_rows += h.n_bfaces_leaf;
            f.user_unknowns += h.n_leaves * cells_per_box(dim, h.N);
        }
        if (f.user_boxes >= ((int64_t)1 << 30) || f.user_rows >= ((int64_t)1 << 31)) {
            delete b;
            return fail(AFMG_ERR_ARG, "batch too large");
        }
        std::vector<int32_t> level((size_t)off[(size_t)n_trees]), idx(3 * (size_t)off[(size_t)n_trees]);
        for (int i = 0; i < n_trees; i++) {
            const HostTree &h = trees[i]->h;
            for (int64_t q = 0; q < h.n_leaves; q++) {
                const size_t m = (size_t)h.leaf_box[(size_t)q], g = (size_t)(off[(size_t)i] + q);
                level[g] = h.info[m].level;
                idx[3 * g] = h.ix[m];
                idx[3 * g + 1] = h.iy[m];
                idx[3 * g + 2] = h.iz[m];
            }
        }
        std::string msg;
        int rc = build_tree(dim, trees[0]->h.N, n_trees, off.data(), level.data(), idx.data(), f.h, msg);
        if (rc != AFMG_OK) {
            delete b;
            return fail(rc, msg);
        }
        f.forest = true;
        compute_partials(&f);
        // caller's box of each working box: inside one tree the working order
        // is the tree's own order, level by level
        const HostTree &fh = f.h;
        f.box_map.assign((size_t)fh.n_boxes, 0);
        std::vector<int64_t> seen((size_t)n_trees, 0);
        int cur_level = 0;
        for (int64_t m = 0; m < fh.n_boxes; m++) {
            const BoxInfo &bi = fh.info[(size_t)m];
            if (bi.level != cur_level) {
                std::fill(seen.begin(), seen.end(), 0);
                cur_level = bi.level;
            }
            const HostTree &h = trees[bi.tree]->h;
            const int64_t local = h.lvl_off[(size_t)bi.level] + seen[(size_t)bi.tree]++;
            if (local >= h.lvl_off[(size_t)bi.level + 1] || h.ix[(size_t)local] != fh.ix[(size_t)m] ||
                h.iy[(size_t)local] != fh.iy[(size_t)m] || h.iz[(size_t)local] != fh.iz[(size_t)m]) {
                delete b;
                return fail(AFMG_ERR_TREE, "inconsistent box order in a batch");
            }
            f.box_map[(size_t)m] = (int32_t)(box_base[(size_t)bi.tree] + local);
        }
        f.row_map.assign((size_t)fh.n_bfaces_leaf, 0);
        for (int64_t r = 0; r < fh.n_bfaces_leaf; r++) {
            const int32_t m = fh.bface_box[(size_t)r];
            const int tr = fh.info[(size_t)m].tree;
            const int64_t local = f.box_map[(size_t)m] - box_base[(size_t)tr];
            const int32_t row = trees[tr]->h.info[(size_t)local].bcoff[fh.bface_side[(size_t)r]];
            f.row_map[(size_t)r] = (int32_t)(row_base[(size_t)tr] + row);
        }
    } catch (const std::bad_alloc &) {
        delete b;
        return fail(AFMG_ERR_OOM, "host allocation failed");
    }
    *out = b;
    return AFMG_OK;
}

void afmg_batch_destroy(afmg_batch *b) {
    if (!b) return;
    release(&b->f);
    delete b;
}

int afmg_batch_info(const afmg_batch *b, afmg_batch_desc *out) {
    if (!b || !out) return fail(AFMG_ERR_ARG, "null argument");
    const HostTree &h = b->f.h;
    out->dim = h.dim;
    out->box_n = h.N;
    out->n_trees = h.n_trees;
    out->lmax = h.lmax;
    out->n_boxes = b->f.user_boxes;
    out->n_bfaces = b->f.user_rows;
    out->n_unknowns = b->f.user_unknowns;
    return AFMG_OK;
}

int afmg_batch_workspace_bytes(const afmg_batch *b, const afmg_opts *o, size_t *bytes) {
    if (!b || !bytes) return fail(AFMG_ERR_ARG, "null argument");
    if (o) {
        int rc = check_opts(o);
        if (rc != AFMG_OK) return rc;
    }
    *bytes = ws_layout(&b->f, o ? o->precision : AFMG_FP64).total;
    return AFMG_OK;
}

int afmg_batch_solve(afmg_batch *b, void *stream, const double *rho, const double *bc, double *u,
                     void *workspace, size_t workspace_bytes, const afmg_opts *opts, afmg_stats *stats) {
    if (!b || !rho || !u || !workspace || !stats) return fail(AFMG_ERR_ARG, "null argument");
    int rc = check_opts(opts);
    if (rc != AFMG_OK) return rc;
    if (!aligned(rho, 8) || !aligned(u, 8) || (bc && !aligned(bc, 8)) || !aligned(workspace, 256))
        return fail(AFMG_ERR_ARG, "misaligned array");
    afmg_tree *f = &b->f;
    if (workspace_bytes < ws_layout(f, opts->precision).total) return fail(AFMG_ERR_ARG, "workspace too small");
    std::memset(stats, 0, sizeof(afmg_stats) * (size_t)f->h.n_trees);
    rc = bind_device(f);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(f->h, solve, (f, st, rho, bc, u, (char *)workspace, *opts, stats));
}

int afmg_autotune_workspace_bytes(const afmg_tree *t, size_t *bytes) {
    if (!t || !bytes) return fail(AFMG_ERR_ARG, "null argument");
    *bytes = tune_layout(t).total;
    return AFMG_OK;
}

int afmg_tree_autotune(afmg_tree *t, void *stream, void *workspace, size_t workspace_bytes) {
    return tree_autotune(t, stream, workspace, workspace_bytes);
}

int afmg_tree_shape(const afmg_tree *t, int precision, int kind, int level, int *wg, int *no_remap) {
    return get_shape(t, precision, kind, level, wg, no_remap);
}

int afmg_tree_set_shape(afmg_tree *t, int precision, int kind, int level, int wg, int no_remap) {
    return set_shape(t, precision, kind, level, wg, no_remap);
}

int afmg_batch_autotune_workspace_bytes(const afmg_batch *b, size_t *bytes) {
    if (!b || !bytes) return fail(AFMG_ERR_ARG, "null argument");
    *bytes = tune_layout(&b->f).total;
    return AFMG_OK;
}

int afmg_batch_autotune(afmg_batch *b, void *stream, void *workspace, size_t workspace_bytes) {
    if (!b) return fail(AFMG_ERR_ARG, "null argument");
    return tree_autotune(&b->f, stream, workspace, workspace_bytes);
}

int afmg_batch_shape(const afmg_batch *b, int precision, int kind, int level, int *wg, int *no_remap) {
    if (!b) return fail(AFMG_ERR_ARG, "null argument");
    return get_shape(&b->f, precision, kind, level, wg, no_remap);
}

int afmg_batch_set_shape(afmg_batch *b, int precision, int kind, int level, int wg, int no_remap) {
    if (!b) return fail(AFMG_ERR_ARG, "null argument");
    return set_shape(&b->f, precision, kind, level, wg, no_remap);
}

int afmg_step(afmg_tree *t, void *stream, int op, int level, int colour, int homog, double *u, double *rho,
              double *uold, const double *bc, void *workspace, size_t workspace_bytes, const afmg_opts *opts) {
    if (!t || !u || !rho || !uold || !workspace) return fail(AFMG_ERR_ARG, "null argument");
    if (t->forest) return fail(AFMG_ERR_ARG, "not a tree");
    afmg_opts o;
    afmg_default_opts(&o);
    if (opts) {
        const int rc = check_opts(opts);
        if (rc != AFMG_OK) return rc;
        o = *opts;
    }
    if (op < AFMG_STEP_HALF_SWEEP || op > AFMG_STEP_COARSE) return fail(AFMG_ERR_ARG, "bad step");
    const int lo = op == AFMG_STEP_HALF_SWEEP ? 1 : 2;
    if (op == AFMG_STEP_COARSE) {
        if (t->h.lmax < 2) return fail(AFMG_ERR_ARG, "the coarse step needs a refined root");
    } else if (level < lo || level > t->h.lmax) {
        return fail(AFMG_ERR_ARG, "level out of range for this step");
    }
    if (colour != 0 && colour != 1) return fail(AFMG_ERR_ARG, "colour must be 0 or 1");
    if (!aligned(u, 8) || !aligned(rho, 8) || !aligned(uold, 8) || (bc && !aligned(bc, 8)) ||
        !aligned(workspace, 256))
        return fail(AFMG_ERR_ARG, "misaligned array");
    if (workspace_bytes < ws_layout(t, AFMG_FP64).total) return fail(AFMG_ERR_ARG, "workspace too small");
    int rc = bind_device(t);
    if (rc != AFMG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    AFMG_BOX_RETURN(t->h, step, (t, st, op, level, colour, homog != 0, u, rho, uold, bc, (char *)workspace, o));
}

}  // extern "C"
