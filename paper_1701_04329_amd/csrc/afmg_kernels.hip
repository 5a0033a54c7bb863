// HIP kernels (gfx950) of the FAS multigrid Poisson solve on box grids.
//
// Storage: every box holds its N^D cells colour-split, red cells (1-based
// index sum even, paper §3.1) first, then black; within a colour z, y, x
// (x fastest, every other cell).  A red-black half sweep therefore reads the
// other colour and the right-hand side of its own colour and writes its own
// colour, each as one contiguous run per box.  The caller's arrays keep the
// natural x-fastest order; k_permute converts at the solve boundary.
//
// No ghost layer is stored: side ghosts (paper §2.4, §3.3) are computed on
// the fly from the neighbouring boxes.  Workgroups are 256 threads (four
// wave64) and one thread owns one x-row of a box, so a workgroup holds four
// boxes of 8^3 cells in 3D (one wave per box) and 32 of 8^2 in 2D; a box of
// 16^3 cells fills the workgroup, 16 boxes of 16^2 share one.  Workgroup ids are
// remapped so that each of the eight XCDs processes a contiguous run of boxes:
// Morton-ordered siblings and neighbours then share one L2.
#include <hip/hip_runtime.h>

#include "afmg_internal.h"
#include "afmg_kernels.h"

namespace afmg {

template <int D, int N>
struct Geo {
    static constexpr int C = D == 3 ? N * N * N : N * N;  // cells per box
    static constexpr int F = D == 3 ? N * N : N;          // cells per side
    static constexpr int P = N + 2;
    static constexpr int PC = D == 3 ? P * P * P : P * P;  // padded cells
    static constexpr int HALF = C / 2;
    static constexpr int HN = N / 2;
    static constexpr int TPB = F;          // threads per box: one per row (j, k) of x-cells
    static constexpr int BPW = 256 / TPB;  // boxes per workgroup
    static constexpr int H = N / 2;                           // parent cells per axis under a box
    static constexpr int HC = D == 3 ? H * H * H : H * H;
    static constexpr int HF = D == 3 ? H * H : H;
    static constexpr int Q = H + 2;
    static constexpr int QC = D == 3 ? Q * Q * Q : Q * Q;
};

// padded LDS index (natural order, ghost layer at -1 and N)
template <int D, int N>
__device__ __forceinline__ int padi(int i, int j, int k) {
    constexpr int P = N + 2;
    return D == 3 ? (i + 1) + P * ((j + 1) + P * (k + 1)) : (i + 1) + P * (j + 1);
}
// colour of a cell: 0 red, 1 black (0-based local indices; box offsets are even)
template <int D>
__device__ __forceinline__ int colour_of(int i, int j, int k) {
    return (i + j + (D == 3 ? k : 0) + D) & 1;
}
// position of a cell inside its colour
template <int D, int N>
__device__ __forceinline__ int in_colour(int i, int j, int k) {
    constexpr int HN = N / 2;
    return (D == 3 ? (k * N + j) * HN : j * HN) + (i >> 1);
}
// storage position of a cell in a box
template <int D, int N>
__device__ __forceinline__ int cpos(int i, int j, int k) {
    return colour_of<D>(i, j, k) * Geo<D, N>::HALF + in_colour<D, N>(i, j, k);
}
// cell of storage position e
template <int D, int N>
__device__ __forceinline__ void cell_of(int e, int &i, int &j, int &k) {
    using G = Geo<D, N>;
    const int c = e / G::HALF, r = e % G::HALF;
    j = (r / G::HN) % N;
    k = D == 3 ? r / (N * G::HN) : 0;
    i = 2 * (r % G::HN) + ((c + D + j + k) & 1);
}
__device__ __forceinline__ int obit(int flags, int axis) { return (flags >> (1 + axis)) & 1; }

// row r of a box: cells (0..N-1, j, k)
template <int D, int N>
__device__ __forceinline__ void row_of(int r, int &j, int &k) {
    j = r % N;
    k = D == 3 ? r / N : 0;
}

// fine cell q (0 .. 2^D - 1, x fastest) of the 2^D block under parent cell pc
// (0 .. (N/2)^D - 1, x fastest) of a box
template <int D, int N>
__device__ __forceinline__ void block_cell(int pc, int q, int &i, int &j, int &k) {
    constexpr int H = N / 2;
    i = 2 * (pc % H) + (q & 1);
    j = 2 * ((pc / H) % H) + ((q >> 1) & 1);
    k = D == 3 ? 2 * (pc / (H * H)) + (q >> 2) : 0;
}

// Contiguous run of workgroup ids per XCD (workgroups are dispatched to the
// eight XCDs round-robin).  Bijective on [0, G).
__device__ __forceinline__ int xcd_remap(int w, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = w & 7, p = w >> 3;
    // x < r: x (q + 1) + p; else r (q + 1) + (x - r) q + p (no branch)
    return x * q + min(x, r) + p;
}
// The same runs, each XCD taking its run from the end: a launch that follows
// one in the forward order starts on the boxes whose data the previous
// launch touched last (still in that XCD's L2)
__device__ __forceinline__ int xcd_remap_rev(int w, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = w & 7, p = w >> 3;
    const int len = q + (x < r ? 1 : 0);
    return x * q + min(x, r) + (len - 1 - p);
}

// Morton neighbours on a complete level (every box of one tree's level
// present, in Morton order, so that box index = Morton key): the x bits of a
// key are the bits of xmask, the y bits xmask << 1, the z bits xmask << 2.
// The neighbour across a side has that coordinate incremented or decremented
// in place (the carry or borrow runs through the other coordinates' bits).
__device__ __forceinline__ int mort_inc(int m, int mask) { return (((m | ~mask) + 1) & mask) | (m & ~mask); }
__device__ __forceinline__ int mort_dec(int m, int mask) { return (((m & mask) - 1) & mask) | (m & ~mask); }
// neighbour box across the low (hi = false) or high side of the axis with
// key bits `mask`, or -1 on the domain boundary
__device__ __forceinline__ int mort_nbr(int64_t b0, int m, int mask, bool hi) {
    const int c = m & mask;
    if (hi) return c != mask ? (int)b0 + mort_inc(m, mask) : -1;
    return c != 0 ? (int)b0 + mort_dec(m, mask) : -1;
}

// Box record of box b.  When a box fills whole waves (3D: one wave per box
// of 8^3 cells, four per box of 16^3) the id is made wave-uniform so that the
// record arrives through one scalar load.
template <int D, int N>
__device__ __forceinline__ BoxInfo load_box(const BoxInfo *__restrict__ info, int64_t b) {
    if (Geo<D, N>::TPB % 64 == 0) return info[__builtin_amdgcn_readfirstlane((int)b)];
    return info[b];
}

template <int D, int N>
struct Slot {
    int64_t b;   // box id (clamped to a valid box)
    bool valid;  // false for the padding slots of the last workgroup
    int slot, t; // slot in the workgroup, thread in the slot
};
// Workgroups of W threads hold W / TPB boxes; with remap set, workgroup ids
// are remapped so that each XCD takes a contiguous run of boxes.  The grid is
// ceil(nb / (W / TPB)) workgroups (wg_count); the count is derived from nb
// rather than read from the dispatch, which saves the kernel one dependent
// argument load before its first memory access.
template <int D, int N, int W = 256>
__device__ __forceinline__ Slot<D, N> slot_of(int64_t b0, int nb, bool remap = true, bool rev = false) {
    using G = Geo<D, N>;
    constexpr int BPW = W / G::TPB;
    static_assert(BPW >= 1 && W % G::TPB == 0, "workgroup must hold whole boxes");
    Slot<D, N> r;
    const int ng = (nb + BPW - 1) / BPW;
    const int wr = rev ? xcd_remap_rev((int)blockIdx.x, ng) : xcd_remap((int)blockIdx.x, ng);
    const int w = remap ? wr : (rev ? ng - 1 - (int)blockIdx.x : (int)blockIdx.x);
    r.slot = (int)threadIdx.x / G::TPB;
    r.t = (int)threadIdx.x % G::TPB;
    int bl = w * BPW + r.slot;
    if (G::TPB % 64 == 0) bl = __builtin_amdgcn_readfirstlane(bl);  // whole waves per box
    r.valid = bl < nb;
    r.b = b0 + (r.valid ? bl : 0);
    return r;
}

// Slot of a level kernel.  Level kernels come in two variants: F = false for
// one tree, whose loads start without waiting for anything but the
// arguments, and F = true for forests, which take their boxes from the
// level's compacted list of boxes of trees still iterating (a.act[0 ..
// *a.nact)): the first ceil(n / boxes per workgroup) workgroups take them, in
// contiguous runs per XCD over that count, and the other workgroups of the
// grid (sized for the whole level) find no box and exit, so that stopped
// trees cost neither memory traffic nor more than an empty workgroup.
template <int D, int N, int W, bool F, typename T>
__device__ __forceinline__ Slot<D, N> slot_lvl(const LevelArgs<T> &a, bool rev = false) {
    if (!F) return slot_of<D, N, W>(a.b0, a.nb, a.no_remap == 0, rev);
    using G = Geo<D, N>;
    constexpr int BPW = W / G::TPB;
    Slot<D, N> r;
    const int n = *a.nact;
    const int g = (n + BPW - 1) / BPW;
    const int wb = (int)blockIdx.x;
    const int w = a.no_remap ? wb : xcd_remap(wb, g);
    r.slot = (int)threadIdx.x / G::TPB;
    r.t = (int)threadIdx.x % G::TPB;
    int bl = w * BPW + r.slot;
    if (G::TPB % 64 == 0) bl = __builtin_amdgcn_readfirstlane(bl);  // whole waves per box
    r.valid = wb < g && bl < n;
    const int q = r.valid ? bl : 0;
    r.b = r.valid ? (int64_t)a.act[q] : a.b0;
    return r;
}

// ---------------------------------------------------------------------------
// side ghosts (paper §2.4, §3.3)
// ---------------------------------------------------------------------------
// A ghost next to face cell x on side S is
//   same-level neighbour v:  its face cell across the side (periodic sides
//                            have their wrapped neighbour here)
//   physical side:           2 b - u1          Dirichlet (b = 0 when homog)
//                            u1 + h q          Neumann, q the outward
//                                              derivative (q = 0 when homog)
//   refinement boundary:     2D 1/2 uH + u1 - 1/4 (u1' + u2)
//                            3D 1/2 uH + 5/4 u1 - 1/4 (u2 + u1' + u1'')
// uH: cell of the coarser neighbour box containing the ghost centre; u2: next
// cell inward; u1', u1'': tangential partners of u1 inside one coarse cell.
// The global operand (neighbour cell, b or uH) is fetched first ("raw"), the
// formula is finished once the box interior is in LDS.
template <int S>
struct SideOf {
    static constexpr int d = S >> 1, hi = S & 1;
    static constexpr int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
};

template <int D, int N, int S>
__device__ __forceinline__ void face_cell(int m, int x[3]) {
    using SD = SideOf<S>;
    x[SD::t1] = m % N;
    x[SD::t2] = D == 3 ? m / N : 0;
    x[SD::d] = SD::hi ? N - 1 : 0;
}

// raw operand of the ghost on side S next to face cell m of box bi (and, by
// ghost_ptr, its address).  The address is selected without branches (one load per ghost, so the loads of a
// thread stay in flight together), and the loaded value is not used here: a
// homogeneous Dirichlet side loads a harmless in-range value, replaced by 0
// when the ghost is finished (after the barrier, so no load waits before it).
template <int D, int N, int S, typename T>
__device__ __forceinline__ const T *ghost_ptr(const BoxInfo &bi, int m, const T *__restrict__ u,
                                              const T *__restrict__ bc, int homog, int &v) {
    using SD = SideOf<S>;
    using G = Geo<D, N>;
    int x[3];
    face_cell<D, N, S>(m, x);
    v = bi.nbr[S];
    const bool cf = v <= -2, dir = v == -1;
    const int flags = bi.flags;
    int q[3];
    q[SD::d] = SD::hi ? 0 : N - 1;
    q[SD::t1] = cf ? obit(flags, SD::t1) * G::H + (x[SD::t1] >> 1) : x[SD::t1];
    q[SD::t2] = D == 3 ? (cf ? obit(flags, SD::t2) * G::H + (x[SD::t2] >> 1) : x[SD::t2]) : 0;
    const int64_t box = v >= 0 ? (int64_t)v : (cf ? (int64_t)(-v - 2) : (int64_t)0);
    const size_t iu = (size_t)box * G::C + cpos<D, N>(q[0], q[1], q[2]);
    const bool from_bc = dir && !homog;
    const size_t ib = from_bc ? (size_t)bi.bcoff[S] * G::F + m : 0;
    return from_bc ? bc + ib : u + iu;
}
template <int D, int N, int S, typename T>
__device__ __forceinline__ T ghost_raw(const BoxInfo &bi, int m, const T *__restrict__ u,
                                       const T *__restrict__ bc, int homog, int &v) {
    return *ghost_ptr<D, N, S, T>(bi, m, u, bc, homog, v);
}

// the ghost of a physical side from its boundary value b (zero when
// homogeneous) and the face cell's value u1
template <typename T>
__device__ __forceinline__ T phys_ghost(bool neumann, T b, T u1, T h) {
    return neumann ? u1 + h * b : T(2) * b - u1;
}
__device__ __forceinline__ bool neumann_side(int flags, int s) { return (flags >> (10 + s)) & 1; }

// The bilinear-extrapolation variant of the refinement-boundary ghost
// (paper §3.3): 2D 1/2 uH + 9/8 u1 - 3/8 (u1p + u2) + 1/8 u2p; 3D, the same
// construction with the second tangential axis,
// 1/2 uH + 27/16 u1 - 9/16 (u2 + u1p + u1q) + 3/16 (u2p + u2q + u1pq)
// - 1/16 u2pq (p: partner along t1, q: along t2, pq: both).  at(depth, f1,
// f2) gives the cell of the box (or octant) at normal depth 0 (face cell)
// or 1 (next inward), flipped to the partner along t1 (f1) and t2 (f2).
template <int D, typename T, class At>
__device__ __forceinline__ T bil_ghost(T uH, const At &at) {
    const T u1 = at(0, 0, 0), u1p = at(0, 1, 0), u2 = at(1, 0, 0), u2p = at(1, 1, 0);
    if (D == 2) return T(0.5) * uH + T(1.125) * u1 - T(0.375) * (u1p + u2) + T(0.125) * u2p;
    const T u1q = at(0, 0, 1), u1pq = at(0, 1, 1), u2q = at(1, 0, 1), u2pq = at(1, 1, 1);
    return T(0.5) * uH + T(27.0 / 16.0) * u1 - T(9.0 / 16.0) * ((u2 + u1p) + u1q) +
           T(3.0 / 16.0) * ((u2p + u2q) + u1pq) - T(1.0 / 16.0) * u2pq;
}

// finish the ghost from its raw operand; s is the padded box in LDS.  RT:
// the refinement-boundary scheme is chosen at run time (bil = 1: bilinear
// extrapolation); otherwise the default scheme is compiled in.
template <int D, int N, int S, typename T, bool RT = false>
__device__ __forceinline__ T ghost_finish(const T *s, int m, T raw, int v, int homog, int flags, T h, int bil = 0) {
    using SD = SideOf<S>;
    if (v >= 0) return raw;
    int x[3];
    face_cell<D, N, S>(m, x);
    const T u1 = s[padi<D, N>(x[0], x[1], x[2])];
    if (v == -1) return phys_ghost<T>(neumann_side(flags, S), homog ? T(0) : raw, u1, h);
    if (RT && bil) {
        auto at = [&](int depth, int f1, int f2) {
            int c[3] = {x[0], x[1], x[2]};
            c[SD::d] = SD::hi ? N - 1 - depth : depth;
            c[SD::t1] ^= f1;
            if (D == 3) c[SD::t2] ^= f2;
            return s[padi<D, N>(c[0], c[1], c[2])];
        };
        return bil_ghost<D, T>(raw, at);
    }
    int y[3] = {x[0], x[1], x[2]};
    y[SD::d] = SD::hi ? N - 2 : 1;
    const T u2 = s[padi<D, N>(y[0], y[1], y[2])];
    int p[3] = {x[0], x[1], x[2]};
    p[SD::t1] ^= 1;
    const T u1p = s[padi<D, N>(p[0], p[1], p[2])];
    if (D == 2) return T(0.5) * raw + u1 - T(0.25) * (u1p + u2);
    int r[3] = {x[0], x[1], x[2]};
    r[SD::t2] ^= 1;
    const T u1pp = s[padi<D, N>(r[0], r[1], r[2])];
    return T(0.5) * raw + T(1.25) * u1 - T(0.25) * ((u2 + u1p) + u1pp);
}

template <int D, int N, int S>
__device__ __forceinline__ int ghost_slot(int m) {
    using SD = SideOf<S>;
    int x[3];
    face_cell<D, N, S>(m, x);
    x[SD::d] = SD::hi ? N : -1;
    return padi<D, N>(x[0], x[1], x[2]);
}

#define AFMG_SIDE_SWITCH(side, CALL) \
    switch (side) {                  \
    case 0: CALL(0); break;          \
    case 1: CALL(1); break;          \
    case 2: CALL(2); break;          \
    case 3: CALL(3); break;          \
    case 4: CALL(4); break;          \
    default: CALL(5); break;         \
    }

// Staging of one box with its ghosts in two phases around a barrier:
// load() fetches row t of the interior and the raw ghost operands, stage()
// writes the row into the padded LDS box (begin() = both); after
// __syncthreads, end() writes the ghost slots; one more __syncthreads and the
// box is ready.  Thread t of the box owns row t (both colours) and face cell t
// of every side (a side has F == TPB cells).  A kernel issues its other
// loads between load() and stage(), so that they are in flight together.
template <int D, int N, typename T, bool RT = false>
struct Stager {
    using G = Geo<D, N>;
    T raw[6];
    int v[6];
    int hg;
    int fl;  // box flags (Neumann sides)
    T hh;    // cell size (Neumann ghosts)
    int bil = 0;  // RT: bilinear-extrapolation refinement ghosts
    T rowv[2][G::HN];

    __device__ __forceinline__ void load(const BoxInfo &bi, const T *__restrict__ ub, const T *__restrict__ u,
                                         const T *__restrict__ bc, int homog, int t, bool ghosts, T h = T(0)) {
        hg = homog;
        fl = bi.flags;
        hh = h;
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int m = 0; m < G::HN; m++) rowv[c][m] = ub[c * G::HALF + t * G::HN + m];
        if (ghosts) {
            raw[0] = ghost_raw<D, N, 0, T>(bi, t, u, bc, homog, v[0]);
            raw[1] = ghost_raw<D, N, 1, T>(bi, t, u, bc, homog, v[1]);
            raw[2] = ghost_raw<D, N, 2, T>(bi, t, u, bc, homog, v[2]);
            raw[3] = ghost_raw<D, N, 3, T>(bi, t, u, bc, homog, v[3]);
            if (D == 3) {
                raw[4] = ghost_raw<D, N, 4, T>(bi, t, u, bc, homog, v[4]);
                raw[5] = ghost_raw<D, N, 5, T>(bi, t, u, bc, homog, v[5]);
            }
        }
    }
    __device__ __forceinline__ void stage(T *s, int t) const {
        int j, k;
        row_of<D, N>(t, j, k);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int p = (c + D + j + k) & 1;
#pragma unroll
            for (int m = 0; m < G::HN; m++) s[padi<D, N>(2 * m + p, j, k)] = rowv[c][m];
        }
    }
    __device__ __forceinline__ void begin(T *s, const BoxInfo &bi, const T *__restrict__ ub,
                                          const T *__restrict__ u, const T *__restrict__ bc, int homog, int t,
                                          bool ghosts, T h = T(0)) {
        load(bi, ub, u, bc, homog, t, ghosts, h);
        stage(s, t);
    }
    __device__ void end(T *s, int t) {
        s[ghost_slot<D, N, 0>(t)] = ghost_finish<D, N, 0, T, RT>(s, t, raw[0], v[0], hg, fl, hh, bil);
        s[ghost_slot<D, N, 1>(t)] = ghost_finish<D, N, 1, T, RT>(s, t, raw[1], v[1], hg, fl, hh, bil);
        s[ghost_slot<D, N, 2>(t)] = ghost_finish<D, N, 2, T, RT>(s, t, raw[2], v[2], hg, fl, hh, bil);
        s[ghost_slot<D, N, 3>(t)] = ghost_finish<D, N, 3, T, RT>(s, t, raw[3], v[3], hg, fl, hh, bil);
        if (D == 3) {
            s[ghost_slot<D, N, 4>(t)] = ghost_finish<D, N, 4, T, RT>(s, t, raw[4], v[4], hg, fl, hh, bil);
            s[ghost_slot<D, N, 5>(t)] = ghost_finish<D, N, 5, T, RT>(s, t, raw[5], v[5], hg, fl, hh, bil);
        }
    }
};

template <int D, int N, typename T>
__device__ __forceinline__ T nb_sum(const T *s, int i, int j, int k) {
    if (D == 2)
        return (s[padi<D, N>(i - 1, j, k)] + s[padi<D, N>(i + 1, j, k)]) +
               (s[padi<D, N>(i, j - 1, k)] + s[padi<D, N>(i, j + 1, k)]);
    return (s[padi<D, N>(i - 1, j, k)] + s[padi<D, N>(i + 1, j, k)]) +
           (s[padi<D, N>(i, j - 1, k)] + s[padi<D, N>(i, j + 1, k)]) +
           (s[padi<D, N>(i, j, k - 1)] + s[padi<D, N>(i, j, k + 1)]);
}

// ---------------------------------------------------------------------------
// Gauss-Seidel red-black half sweep (paper §3.1)
// ---------------------------------------------------------------------------
// Thread t of a box updates the N/2 cells of `colour` in row t.  Only the
// other colour is staged in LDS; the thread fetches the ghosts of its own cells
// (one x ghost at the row end, a y / z ghost per cell on the box faces) and,
// next to Dirichlet or refinement sides, the old values of its cells, which
// those ghost formulas use.

// ghost of side S next to own cell (i, j, k), other colour in s
// LDS slot of an other-colour cell: x-pair index major, row minor, so that the
// threads of a wave (consecutive rows) touch consecutive words.  In 2D a
// box's block is padded by one word so that the eight boxes of a wave do not
// share banks.
template <int D, int N>
__device__ __forceinline__ int oslot(int i, int j, int k) {
    constexpr int TPB = Geo<D, N>::TPB;
    return (i >> 1) * TPB + (D == 3 ? k * N + j : j);
}
template <int D, int N>
constexpr int oblock() { return Geo<D, N>::HALF + (D == 3 ? 0 : 1); }

template <int D, int N, int S, typename T>
__device__ __forceinline__ T gs_finish(const T *s, T raw, int v, T own, int homog, int i, int j, int k, int flags,
                                       T h) {
    using SD = SideOf<S>;
    if (v >= 0) return raw;
    if (v == -1) return phys_ghost<T>(neumann_side(flags, S), homog ? T(0) : raw, own, h);
    int y[3] = {i, j, k};
    y[SD::d] += SD::hi ? -1 : 1;
    int p1[3] = {i, j, k};
    p1[SD::t1] ^= 1;
    const T u2 = s[oslot<D, N>(y[0], y[1], y[2])];
    const T u1p = s[oslot<D, N>(p1[0], p1[1], p1[2])];
    if (D == 2) return T(0.5) * raw + own - T(0.25) * (u1p + u2);
    int p2[3] = {i, j, k};
    p2[SD::t2] ^= 1;
    const T u1pp = s[oslot<D, N>(p2[0], p2[1], p2[2])];
    return T(0.5) * raw + T(1.25) * own - T(0.25) * ((u2 + u1p) + u1pp);
}

// Slot of this workgroup holding the same-level neighbour across side s of
// box sl.b (one tree: slot q holds box sl.b + q - sl.slot), or -1.  Only the
// slot that differs in the side's axis bit can be a sibling; the box table
// decides (any box order stays correct).
// (v: the box record's neighbour entry of that side, selected with a
// compile-time index so that the record stays in registers)
template <int D, int N, int W, int AXIS>
__device__ __forceinline__ int sib_slot(int v, const Slot<D, N> &sl, int64_t b0, int nb) {
    constexpr int BPW = W / Geo<D, N>::TPB, BIT = 1 << AXIS;
    if constexpr (BIT >= BPW) {
        return -1;
    } else {
        const int q = sl.slot ^ BIT;
        const int64_t cand = sl.b + (q - sl.slot);
        return (v >= 0 && (int64_t)v == cand && cand - b0 < nb) ? q : -1;
    }
}

template <int D, int N, typename T, int W, bool F>
__global__ __launch_bounds__(W) void k_gsrb(LevelArgs<T> a, int colour) {
    using G = Geo<D, N>;
    constexpr int HN = G::HN;
    __shared__ T so[(W / G::TPB) * oblock<D, N>()];
    // the black half sweep takes each XCD's run of boxes from the end, so
    // that it starts where the red one ended (and the other way round)
    const Slot<D, N> sl = slot_lvl<D, N, W, F>(a, colour == 1);
    T *s = so + sl.slot * oblock<D, N>();
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    T *ub = a.u + (size_t)sl.b * G::C;
    const int r = sl.t;
    int j, k;
    row_of<D, N>(r, j, k);
    const int p = (colour + D + j + k) & 1;  // x parity of the updated cells in this row
    const int own0 = colour * G::HALF + r * HN;
    T rr[HN], ow[HN], gy[HN], gz[HN];
    T gx = T(0);
    int vx = 0, vy = 0, vz = 0;
#pragma unroll
    for (int m = 0; m < HN; m++) {
        ow[m] = T(0);
        gy[m] = T(0);
        gz[m] = T(0);
    }
    // one tree: the padding slots of the last workgroup load a valid box too
    // (sl.b is clamped), so that no branch separates the loads from the
    // kernel start
    const bool act = sl.valid;
    // Siblings in the workgroup: the 2^D children of a parent are consecutive
    // in a level's box order, so slot ^ (axis bit) is often the same-level
    // neighbour across a side.  Its other colour is staged in LDS by its own
    // threads, and ghosts across such a side are read there after the
    // barrier (the same values as from global memory).  qx, qy, qz: the slot
    // across the side this thread's ghosts need, or -1.
    // (decided after the box's own loads are issued: it needs the box record)
    int qx = -1, qy = -1, qz = -1;
    if (!F || act) {
        T ot[HN];
        const int oth0 = (1 - colour) * G::HALF + r * HN;
#pragma unroll
        for (int m = 0; m < HN; m++) ot[m] = ub[oth0 + m];
        const T *rb = a.rho + (size_t)sl.b * G::C + own0;
#pragma unroll
        for (int m = 0; m < HN; m++) rr[m] = rb[m];
        if (!F) {
            qx = sib_slot<D, N, W, 0>(p == 0 ? bi.nbr[0] : bi.nbr[1], sl, a.b0, a.nb);
            qy = sib_slot<D, N, W, 1>(j == 0 ? bi.nbr[2] : bi.nbr[3], sl, a.b0, a.nb);
            if (D == 3) qz = sib_slot<D, N, W, 2>(k == 0 ? bi.nbr[4] : bi.nbr[5], sl, a.b0, a.nb);
        }
        // x ghost of the row end cell (side 0 when the row starts with this colour)
        if (qx < 0) {
            if (p == 0) gx = ghost_raw<D, N, 0, T>(bi, r, a.u, a.bc, a.homog, vx);
            else gx = ghost_raw<D, N, 1, T>(bi, r, a.u, a.bc, a.homog, vx);
        }
        bool need_own = vx < 0;
        // y / z ghosts.  Across a same-level side they are the other-colour
        // cells of one row of the neighbour (row j' = N-1-j, resp. k' =
        // N-1-k), HN contiguous values like the thread's own row.  Boxes
        // with both sides of an axis at the same level take this form, the
        // others the general one, which comes later in the program so that
        // the common form's loads never wait for its loads.
        const bool yrow = (j == 0 || j == N - 1) && qy < 0, zrow = D == 3 && (k == 0 || k == N - 1) && qz < 0;
        const bool yfast = bi.nbr[2] >= 0 && bi.nbr[3] >= 0;
        const bool zfast = D == 3 && bi.nbr[4] >= 0 && bi.nbr[5] >= 0;
        if (yfast && yrow) {
            vy = bi.nbr[j == 0 ? 2 : 3];
            const T *nr = a.u + (size_t)vy * G::C + oth0 + ((D == 3 ? N * k : 0) + (N - 1 - j) - r) * HN;
#pragma unroll
            for (int m = 0; m < HN; m++) gy[m] = nr[m];
        }
        if (zfast && zrow) {
            vz = bi.nbr[k == 0 ? 4 : 5];
            const T *nr = a.u + (size_t)vz * G::C + oth0 + ((N - 1 - k) * N + j - r) * HN;
#pragma unroll
            for (int m = 0; m < HN; m++) gz[m] = nr[m];
        }
        __asm__ volatile("" ::: "memory");
        if (!yfast && yrow) {
#pragma unroll
            for (int m = 0; m < HN; m++) {
                const int fm = (2 * m + p) + (D == 3 ? N * k : 0);
                int v2, v3;
                const T *p2 = ghost_ptr<D, N, 2, T>(bi, fm, a.u, a.bc, a.homog, v2);
                const T *p3 = ghost_ptr<D, N, 3, T>(bi, fm, a.u, a.bc, a.homog, v3);
                vy = j == 0 ? v2 : v3;
                gy[m] = *(j == 0 ? p2 : p3);
            }
            need_own |= vy < 0;
        }
        if (D == 3 && !zfast && zrow) {
#pragma unroll
            for (int m = 0; m < HN; m++) {
                const int fm = (2 * m + p) + N * j;
                int v4, v5;
                const T *p4 = ghost_ptr<D, N, 4, T>(bi, fm, a.u, a.bc, a.homog, v4);
                const T *p5 = ghost_ptr<D, N, 5, T>(bi, fm, a.u, a.bc, a.homog, v5);
                vz = k == 0 ? v4 : v5;
                gz[m] = *(k == 0 ? p4 : p5);
            }
            need_own |= vz < 0;
        }
        if (need_own) {
#pragma unroll
            for (int m = 0; m < HN; m++) ow[m] = ub[own0 + m];
        }
#pragma unroll
        for (int m = 0; m < HN; m++) s[m * G::TPB + r] = ot[m];
    }
    __syncthreads();
    if (!act) return;
    // ghosts from a sibling's staged other colour: its face cell across the side
    if (qx >= 0) gx = so[qx * oblock<D, N>() + oslot<D, N>(p == 0 ? N - 1 : 0, j, k)];
    if (qy >= 0 && (j == 0 || j == N - 1)) {
#pragma unroll
        for (int m = 0; m < HN; m++) gy[m] = so[qy * oblock<D, N>() + oslot<D, N>(2 * m + p, j == 0 ? N - 1 : 0, k)];
    }
    if (D == 3 && qz >= 0 && (k == 0 || k == N - 1)) {
#pragma unroll
        for (int m = 0; m < HN; m++) gz[m] = so[qz * oblock<D, N>() + oslot<D, N>(2 * m + p, j, k == 0 ? N - 1 : 0)];
    }
#pragma unroll
    for (int m = 0; m < HN; m++) {
        const int i = 2 * m + p;
        const int fl = bi.flags;
        const T xm = i > 0 ? s[oslot<D, N>(i - 1, j, k)] : gs_finish<D, N, 0, T>(s, gx, vx, ow[m], a.homog, i, j, k, fl, a.h);
        const T xp = i < N - 1 ? s[oslot<D, N>(i + 1, j, k)] : gs_finish<D, N, 1, T>(s, gx, vx, ow[m], a.homog, i, j, k, fl, a.h);
        const T ym = j > 0 ? s[oslot<D, N>(i, j - 1, k)] : gs_finish<D, N, 2, T>(s, gy[m], vy, ow[m], a.homog, i, j, k, fl, a.h);
        const T yp = j < N - 1 ? s[oslot<D, N>(i, j + 1, k)] : gs_finish<D, N, 3, T>(s, gy[m], vy, ow[m], a.homog, i, j, k, fl, a.h);
        T sum = (xm + xp) + (ym + yp);
        if (D == 3) {
            const T zm = k > 0 ? s[oslot<D, N>(i, j, k - 1)] : gs_finish<D, N, 4, T>(s, gz[m], vz, ow[m], a.homog, i, j, k, fl, a.h);
            const T zp = k < N - 1 ? s[oslot<D, N>(i, j, k + 1)] : gs_finish<D, N, 5, T>(s, gz[m], vz, ow[m], a.homog, i, j, k, fl, a.h);
            sum = sum + (zm + zp);
        }
        rr[m] = (sum - a.h2 * rr[m]) / T(2 * D);
    }
    // the row's new values leave together (two 16-byte stores per thread in
    // FP64 instead of four scattered 8-byte ones)
#pragma unroll
    for (int m = 0; m < HN; m++) ub[own0 + m] = rr[m];
}

// Half sweep on a complete level of one tree (LevelArgs::xmask != 0): every
// side is same-level or physical, and the neighbour ids come from the Morton
// index, so that the ghost loads leave with the box's own loads instead of
// waiting for the box table.  Boxes on the domain boundary fetch their
// Dirichlet values b (rows named by the box record, a scalar load issued
// first) and the old values u1 of their own cells before the barrier as
// well (ghost 2 b - u1).  Same arithmetic and order as k_gsrb.
// Modes for a mixed-precision correction on a tree whose leaves all lie on
// this level.  CUBE_ADD (its last half sweep): instead of storing the new
// values, add e (the new values and the other colour's) to the FP64
// solution a.add_to on every cell of the box, and set the updated colour of
// e to zero: the refinement update u += e, bitwise as the separate update
// kernel computes it.  The other colour keeps its values (neighbouring boxes
// read them as ghosts during the launch).  CUBE_OWN_ZERO (the first half
// sweep of the next correction): the old values of the updated colour are
// taken as zero; they enter only through the Dirichlet ghost 2b - u1, so
// that with the other colour zero this half sweep equals the one from e = 0.
enum { CUBE_PLAIN = 0, CUBE_ADD = 1, CUBE_OWN_ZERO = 2 };
template <int D, int N, typename T, int W, int MODE>
__global__ __launch_bounds__(W) void k_gsrb_cube(LevelArgs<T> a, int colour) {
    constexpr bool ADD = MODE == CUBE_ADD;
    using G = Geo<D, N>;
    constexpr int HN = G::HN;
    __shared__ T so[(W / G::TPB) * oblock<D, N>()];
    // the arguments the loads need, fetched in one batch: an empty asm takes
    // them as operands, so that the compiler cannot sink their loads behind
    // the branches of the neighbour computation
    __asm__ volatile("" ::"s"(a.u), "s"(a.rho), "s"(a.b0), "s"(a.nb), "s"(a.no_remap), "s"(a.xmask),
                     "s"(colour));
    if (ADD) __asm__ volatile("" ::"s"(a.add_to));
    const Slot<D, N> sl = slot_lvl<D, N, W, false>(a, colour == 1);
    T *s = so + sl.slot * oblock<D, N>();
    T *ub = a.u + (size_t)sl.b * G::C;
    // the box record (boundary rows of Dirichlet sides), issued first
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const int r = sl.t;
    int j, k;
    row_of<D, N>(r, j, k);
    const int p = (colour + D + j + k) & 1;  // x parity of the updated cells in this row
    const int own0 = colour * G::HALF + r * HN, oth0 = (1 - colour) * G::HALF + r * HN;
    const int xm = a.xmask, mb = (int)(sl.b - a.b0);
    const bool yrow = j == 0 || j == N - 1, zrow = D == 3 && (k == 0 || k == N - 1);
    // neighbours across the x side of the row end cell, the y side of row j,
    // the z side of row k (-1: physical side)
    const int vx = mort_nbr(a.b0, mb, xm, p != 0);
    const int vy = yrow ? mort_nbr(a.b0, mb, xm << 1, j != 0) : 0;
    const int vz = zrow ? mort_nbr(a.b0, mb, xm << 2, k != 0) : 0;
    // the neighbour is a sibling in this workgroup (slot ^ axis bit, box
    // key ^ axis bit): its ghost comes from its staged other colour
    constexpr int BPW = W / G::TPB;
    const int rx = vx - (int)a.b0, ry = vy - (int)a.b0, rz = vz - (int)a.b0;
    const int qx = (BPW > 1 && vx >= 0 && rx == (mb ^ 1)) ? (sl.slot ^ 1) : -1;
    const int qy = (BPW > 2 && yrow && vy >= 0 && ry == (mb ^ 2)) ? (sl.slot ^ 2) : -1;
    const int qz = (D == 3 && BPW > 4 && zrow && vz >= 0 && rz == (mb ^ 4)) ? (sl.slot ^ 4) : -1;
    T rr[HN], ot[HN], gy[HN], gz[HN];
    T gx = T(0);
#pragma unroll
    for (int m = 0; m < HN; m++) {
        gy[m] = T(0);
        gz[m] = T(0);
    }
    // padding slots load a valid box too (sl.b is clamped)
#pragma unroll
    for (int m = 0; m < HN; m++) ot[m] = ub[oth0 + m];
    const T *rb = a.rho + (size_t)sl.b * G::C + own0;
#pragma unroll
    for (int m = 0; m < HN; m++) rr[m] = rb[m];
    if (vx >= 0 && qx < 0) gx = a.u[(size_t)vx * G::C + cpos<D, N>(p == 0 ? N - 1 : 0, j, k)];
    if (yrow && vy >= 0 && qy < 0) {
        const T *nr = a.u + (size_t)vy * G::C + oth0 + ((D == 3 ? N * k : 0) + (N - 1 - j) - r) * HN;
#pragma unroll
        for (int m = 0; m < HN; m++) gy[m] = nr[m];
    }
    if (zrow && vz >= 0 && qz < 0) {
        const T *nr = a.u + (size_t)vz * G::C + oth0 + ((N - 1 - k) * N + j - r) * HN;
#pragma unroll
        for (int m = 0; m < HN; m++) gz[m] = nr[m];
    }
    double fo[HN], ft[HN];  // ADD: the FP64 solution on this row's cells of each colour
    if (ADD) {
        const double *fb = a.add_to + (size_t)sl.b * G::C;
#pragma unroll
        for (int m = 0; m < HN; m++) {
            fo[m] = fb[own0 + m];
            ft[m] = fb[oth0 + m];
        }
    }
    // Dirichlet sides: ghost 2 b - u1 (b = 0 when homogeneous).  The old
    // values and the boundary values leave before the barrier; the box record
    // they need is a scalar load, so its wait holds back none of the loads
    // above
    const bool dx = vx < 0, dy = yrow && vy < 0, dz = zrow && vz < 0;
    T ow[HN], bx = T(0), by[HN], bz[HN];
#pragma unroll
    for (int m = 0; m < HN; m++) {
        ow[m] = T(0);
        by[m] = T(0);
        bz[m] = T(0);
    }
    if (dx || dy || dz) {
        if (MODE != CUBE_OWN_ZERO) {
#pragma unroll
            for (int m = 0; m < HN; m++) ow[m] = ub[own0 + m];
        }
        if (!a.homog) {
            if (dx) bx = a.bc[(size_t)(p == 0 ? bi.bcoff[0] : bi.bcoff[1]) * G::F + r];
            if (dy) {
                const T *br = a.bc + (size_t)(j == 0 ? bi.bcoff[2] : bi.bcoff[3]) * G::F + (D == 3 ? N * k : 0) + p;
#pragma unroll
                for (int m = 0; m < HN; m++) by[m] = br[2 * m];
            }
            if (dz) {
                const T *br = a.bc + (size_t)(k == 0 ? bi.bcoff[4] : bi.bcoff[5]) * G::F + N * j + p;
#pragma unroll
                for (int m = 0; m < HN; m++) bz[m] = br[2 * m];
            }
        }
    }
#pragma unroll
    for (int m = 0; m < HN; m++) s[m * G::TPB + r] = ot[m];
    __syncthreads();
    if (!sl.valid) return;
    if (qx >= 0) gx = so[qx * oblock<D, N>() + oslot<D, N>(p == 0 ? N - 1 : 0, j, k)];
    if (qy >= 0) {
#pragma unroll
        for (int m = 0; m < HN; m++) gy[m] = so[qy * oblock<D, N>() + oslot<D, N>(2 * m + p, j == 0 ? N - 1 : 0, k)];
    }
    if (qz >= 0) {
#pragma unroll
        for (int m = 0; m < HN; m++) gz[m] = so[qz * oblock<D, N>() + oslot<D, N>(2 * m + p, j, k == 0 ? N - 1 : 0)];
    }
#pragma unroll
    for (int m = 0; m < HN; m++) {
        const int i = 2 * m + p;
        const T gxm = dx ? T(2) * bx - ow[m] : gx;
        const T gym = dy ? T(2) * by[m] - ow[m] : gy[m];
        const T xm_ = i > 0 ? s[oslot<D, N>(i - 1, j, k)] : gxm;
        const T xp_ = i < N - 1 ? s[oslot<D, N>(i + 1, j, k)] : gxm;
        const T ym_ = j > 0 ? s[oslot<D, N>(i, j - 1, k)] : gym;
        const T yp_ = j < N - 1 ? s[oslot<D, N>(i, j + 1, k)] : gym;
        T sum = (xm_ + xp_) + (ym_ + yp_);
        if (D == 3) {
            const T gzm = dz ? T(2) * bz[m] - ow[m] : gz[m];
            const T zm_ = k > 0 ? s[oslot<D, N>(i, j, k - 1)] : gzm;
            const T zp_ = k < N - 1 ? s[oslot<D, N>(i, j, k + 1)] : gzm;
            sum = sum + (zm_ + zp_);
        }
        rr[m] = (sum - a.h2 * rr[m]) / T(2 * D);
    }
    if (ADD) {
        double *fb = a.add_to + (size_t)sl.b * G::C;
#pragma unroll
        for (int m = 0; m < HN; m++) {
            fo[m] = fo[m] + (double)rr[m];
            ft[m] = ft[m] + (double)ot[m];
        }
#pragma unroll
        for (int m = 0; m < HN; m++) fb[own0 + m] = fo[m];
#pragma unroll
        for (int m = 0; m < HN; m++) fb[oth0 + m] = ft[m];
#pragma unroll
        for (int m = 0; m < HN; m++) ub[own0 + m] = T(0);
        return;
    }
#pragma unroll
    for (int m = 0; m < HN; m++) ub[own0 + m] = rr[m];
}

// ---------------------------------------------------------------------------
// residual (eq. residual) and restriction by averaging (paper §2.5)
// ---------------------------------------------------------------------------
// The octant of box bi's parent receives the mean of each 2^D block of src
// (src in LDS, padded or plain natural order).
template <int D, int N, typename T, bool PADDED>
__device__ __forceinline__ void restrict_octant(const T *s, T *__restrict__ dst, const BoxInfo &bi,
                                                int t) {
    using G = Geo<D, N>;
    const T w = D == 3 ? T(0.125) : T(0.25);
    const int flags = bi.flags;
    const int64_t p = bi.parent;
    for (int pc = t; pc < G::HC; pc += G::TPB) {
        const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
        T acc = T(0);
#pragma unroll
        for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
#pragma unroll
            for (int dj = 0; dj < 2; dj++)
#pragma unroll
                for (int di = 0; di < 2; di++) {
                    const int i = 2 * I + di, j = 2 * J + dj, k = D == 3 ? 2 * K + dk : 0;
                    acc += PADDED ? s[padi<D, N>(i, j, k)] : s[D == 3 ? i + N * (j + N * k) : i + N * j];
                }
        const int X = obit(flags, 0) * G::H + I, Y = obit(flags, 1) * G::H + J,
                  Z = D == 3 ? obit(flags, 2) * G::H + K : 0;
        dst[(size_t)p * G::C + cpos<D, N>(X, Y, Z)] = w * acc;
    }
}

// Boxes of level l: r = rho - L u; the parent's octant receives mean(u) in u
// and mean(r) in rho (the restricted residual, turned into the FAS
// right-hand side by k_coarse_rhs).
template <int D, int N, typename T, int W, bool F>
__global__ __launch_bounds__(W) void k_resid_restrict(LevelArgs<T> a) {
    using G = Geo<D, N>;
    __shared__ T sm[(W / G::TPB) * G::PC];
    const Slot<D, N> sl = slot_lvl<D, N, W, F>(a);
    T *s = sm + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    // each thread: NPC parent cells (2^D blocks); their right-hand side is
    // fetched before the staging loads so that both are in flight together
    constexpr int NPC = G::HC / G::TPB, NB = D == 3 ? 8 : 4;
    T rf[NPC][NB];
    Stager<D, N, T> st;
    // one tree: padding slots (sl.b clamped to a valid box) load too, no
    // branch before the loads
    const bool act = sl.valid;
    if (!F || act) {
#pragma unroll
        for (int it = 0; it < NPC; it++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
                int i, j, k;
                block_cell<D, N>(sl.t + it * G::TPB, q, i, j, k);
                rf[it][q] = a.rho[bo + cpos<D, N>(i, j, k)];
            }
        st.begin(s, bi, a.u + bo, a.u, a.bc, a.homog, sl.t, true, a.h);
    }
    __syncthreads();
    if (act) st.end(s, sl.t);
    __syncthreads();
    if (!act) return;
    const T w = D == 3 ? T(0.125) : T(0.25);
    const int flags = bi.flags;
    const int64_t p = bi.parent;
#pragma unroll
    for (int it = 0; it < NPC; it++) {
        const int pc = sl.t + it * G::TPB;
        const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
        T su = T(0), sr = T(0);
#pragma unroll
        for (int q = 0; q < NB; q++) {
            int i, j, k;
            block_cell<D, N>(pc, q, i, j, k);
            const T uc = s[padi<D, N>(i, j, k)];
            su += uc;
            sr += rf[it][q] - (nb_sum<D, N, T>(s, i, j, k) - T(2 * D) * uc) * a.ih2;
        }
        const int X = obit(flags, 0) * G::H + I, Y = obit(flags, 1) * G::H + J,
                  Z = D == 3 ? obit(flags, 2) * G::H + K : 0;
        const size_t o = (size_t)p * G::C + cpos<D, N>(X, Y, Z);
        a.u[o] = w * su;
        a.rho[o] = w * sr;
    }
}

// ---------------------------------------------------------------------------
// FAS coarse right-hand side (eq. coarse-rhs) and the copy v'_H
// ---------------------------------------------------------------------------
// Boxes of level l-1: uold <- u; on parents rho <- rbar + L_H u (rho holds
// rbar, the restricted residual).
template <int D, int N, typename T, int W, bool F>
__global__ __launch_bounds__(W) void k_coarse_rhs(LevelArgs<T> a) {
    using G = Geo<D, N>;
    __shared__ T sm[(W / G::TPB) * G::PC];
    const Slot<D, N> sl = slot_lvl<D, N, W, F>(a);
    T *s = sm + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const bool parent = !(bi.flags & FLAG_LEAF);
    constexpr int NE = G::C / G::TPB;  // cells per thread
    T rf[NE];
    Stager<D, N, T> st;
    // rows first (one tree: padding slots load a valid box too), then what
    // depends on the box record: ghosts and rbar of parents
    const bool act = sl.valid;
    if (!F || act) {
        st.load(bi, a.u + bo, a.u, a.bc, a.homog, sl.t, parent, a.h);
        if (parent) {
#pragma unroll
            for (int it = 0; it < NE; it++) rf[it] = a.rho[bo + sl.t + it * G::TPB];
        }
        st.stage(s, sl.t);
    }
    __syncthreads();
    if (act) {
        // the copy v' from the staged interior
        for (int e = sl.t; e < G::C; e += G::TPB) {
            int i, j, k;
            cell_of<D, N>(e, i, j, k);
            a.uold[bo + e] = s[padi<D, N>(i, j, k)];
        }
    }
    if (act && parent) st.end(s, sl.t);
    __syncthreads();
    if (!act || !parent) return;
#pragma unroll
    for (int it = 0; it < NE; it++) {
        const int e = sl.t + it * G::TPB;
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        a.rho[bo + e] = rf[it] + (nb_sum<D, N, T>(s, i, j, k) - T(2 * D) * s[padi<D, N>(i, j, k)]) * a.ih2;
    }
}

// ---------------------------------------------------------------------------
// coarse-grid correction (eq. coarse-corr) with 2-1-1 prolongation (§2.5)
// ---------------------------------------------------------------------------
// Boxes of level l: u += P(delta), delta = u - uold of the parent (level
// l-1).  The parent's octant under the box plus a one-cell face halo is
// staged; halo cells outside the parent are ghosts of delta.  The ghost
// formulas are linear, so the ghost of delta is the formula applied to
// deltas, and Dirichlet values cancel (2b - u1 minus 2b - u1_old).
//   2D: 1/2 d(P) + 1/4 d(P + sx ex) + 1/4 d(P + sy ey)
//   3D: 1/4 [d(P) + d(P + sx ex) + d(P + sy ey) + d(P + sz ez)]
// with s = -1 for a fine cell in the lower half of its parent cell.
template <int D, int N>
__device__ __forceinline__ int qpad(int I, int J, int K) {
    constexpr int Q = N / 2 + 2;
    return D == 3 ? (I + 1) + Q * ((J + 1) + Q * (K + 1)) : (I + 1) + Q * (J + 1);
}

// Halo cell m of side S of the octant (o = octant origin in parent cells).
// halo_addr gives the cell whose delta is the halo value (inside the parent
// or in a same-level neighbour: v >= 0) or the global operand of its ghost
// formula (the coarser cell uH of a refinement side; v <= -2), the side type v
// and the LDS slot.  Phase 2 (after a barrier) finishes the ghosts (v < 0)
// from the staged octant.
template <int D, int N, int S>
__device__ __forceinline__ void halo_cell(int m, const int o[3], int L[3], int X[3]) {
    using SD = SideOf<S>;
    using G = Geo<D, N>;
    L[SD::t1] = m % G::H;
    L[SD::t2] = D == 3 ? m / G::H : 0;
    L[SD::d] = SD::hi ? G::H : -1;
    X[0] = o[0] + L[0];
    X[1] = o[1] + L[1];
    X[2] = D == 3 ? o[2] + L[2] : 0;
}

template <int D, int N, int S>
__device__ __forceinline__ size_t halo_addr(int m, const int o[3], const BoxInfo &pi, int64_t p, int &v,
                                            int &slot) {
    using SD = SideOf<S>;
    using G = Geo<D, N>;
    int L[3], X[3];
    halo_cell<D, N, S>(m, o, L, X);
    const bool inside = X[SD::d] >= 0 && X[SD::d] < N;
    const int nb = pi.nbr[S];
    v = inside ? 0 : nb;
    const bool cf = v <= -2;
    const int flags = pi.flags;
    const int x1 = X[SD::t1], x2 = X[SD::t2];
    if (!inside) X[SD::d] = SD::hi ? 0 : N - 1;
    X[SD::t1] = cf ? obit(flags, SD::t1) * G::H + (x1 >> 1) : x1;
    X[SD::t2] = D == 3 ? (cf ? obit(flags, SD::t2) * G::H + (x2 >> 1) : x2) : 0;
    // a Dirichlet side reads the parent's own (in-range) cell and ignores it
    const int64_t box = inside ? p : (v >= 0 ? (int64_t)v : (cf ? (int64_t)(-v - 2) : p));
    slot = qpad<D, N>(L[0], L[1], L[2]);
    return (size_t)box * G::C + cpos<D, N>(X[0], X[1], X[2]);
}

// Dirichlet: ghost of delta = -delta(face cell), Neumann: +delta(face cell)
// (the boundary values cancel); refinement side: the default scheme applied
// to deltas.
template <int D, int N, int S, typename T, bool RT = false>
__device__ __forceinline__ void halo_phase2(T *q, int m, const int o[3], T raw, int v, int pflags, int bil = 0) {
    using SD = SideOf<S>;
    if (v >= 0) return;
    int L[3], X[3];
    halo_cell<D, N, S>(m, o, L, X);
    int f[3] = {L[0], L[1], L[2]};
    f[SD::d] = SD::hi ? L[SD::d] - 1 : 0;  // face cell inside the octant
    const T d1 = q[qpad<D, N>(f[0], f[1], f[2])];
    T val;
    if (v == -1) {
        val = neumann_side(pflags, S) ? d1 : -d1;
    } else if (RT && bil) {
        auto at = [&](int depth, int f1, int f2) {
            int c[3] = {f[0], f[1], f[2]};
            c[SD::d] += SD::hi ? -depth : depth;
            c[SD::t1] ^= f1;  // octant origins are even: partners stay inside
            if (D == 3) c[SD::t2] ^= f2;
            return q[qpad<D, N>(c[0], c[1], c[2])];
        };
        val = bil_ghost<D, T>(raw, at);
    } else {
        int y[3] = {f[0], f[1], f[2]};
        y[SD::d] += SD::hi ? -1 : 1;
        int p1[3] = {f[0], f[1], f[2]};
        p1[SD::t1] ^= 1;  // octant origins are even: partners stay in the octant
        const T d2 = q[qpad<D, N>(y[0], y[1], y[2])];
        const T d1p = q[qpad<D, N>(p1[0], p1[1], p1[2])];
        if (D == 2) {
            val = T(0.5) * raw + d1 - T(0.25) * (d1p + d2);
        } else {
            int p2[3] = {f[0], f[1], f[2]};
            p2[SD::t2] ^= 1;
            const T d1pp = q[qpad<D, N>(p2[0], p2[1], p2[2])];
            val = T(0.5) * raw + T(1.25) * d1 - T(0.25) * ((d2 + d1p) + d1pp);
        }
    }
    q[qpad<D, N>(L[0], L[1], L[2])] = val;
}

template <int D, int N, typename T, int W, bool F>
__global__ __launch_bounds__(W) void k_prolong(LevelArgs<T> a) {
    using G = Geo<D, N>;
    constexpr int NH = (2 * D * G::HF + G::TPB - 1) / G::TPB;  // halo cells per thread
    constexpr int NO = G::HC / G::TPB;                           // octant cells per thread
    constexpr int NE = G::C / G::TPB;                            // fine cells per thread
    __shared__ T qs[(W / G::TPB) * G::QC];
    // reversed order: the first half sweep that follows runs forward
    const Slot<D, N> sl = slot_lvl<D, N, W, F>(a, true);
    T *q = qs + sl.slot * G::QC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    T raw[NH], uf[NE];
    int hv[NH];
    int pfl = 0;  // the parent's flags (Neumann sides of its halo)
    // the fine values (needed only after the barriers) first: they need no
    // box record; one tree: padding slots (sl.b clamped to a valid box) load
    // too
    const bool act = sl.valid;
    if (!F || act) {
#pragma unroll
        for (int it = 0; it < NE; it++) uf[it] = a.u[bo + sl.t + it * G::TPB];
    }
    const int flags = bi.flags;
    const int o[3] = {obit(flags, 0) * G::H, obit(flags, 1) * G::H, D == 3 ? obit(flags, 2) * G::H : 0};
    if (!F || act) {
        const int64_t p = bi.parent;
        const BoxInfo pi = load_box<D, N>(a.info, p);
        pfl = pi.flags;
        // every global operand (octant, halo) before the LDS stores
        T od[NO];
#pragma unroll
        for (int it = 0; it < NO; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            const size_t oo = (size_t)p * G::C + cpos<D, N>(o[0] + I, o[1] + J, o[2] + K);
            od[it] = a.u[oo] - a.uold[oo];
        }
        int hs[NH];
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int hc = sl.t + h * G::TPB;
            size_t ho = (size_t)p * G::C;
            hv[h] = 0;
            hs[h] = 0;
            if (hc < 2 * D * G::HF) {
                const int side = hc / G::HF, m = hc % G::HF;
#define AFMG_H1(S) ho = halo_addr<D, N, S>(m, o, pi, p, hv[h], hs[h])
                AFMG_SIDE_SWITCH(side, AFMG_H1)
#undef AFMG_H1
            }
            raw[h] = a.u[ho] - a.uold[ho];
        }
#pragma unroll
        for (int it = 0; it < NO; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            q[qpad<D, N>(I, J, K)] = od[it];
        }
#pragma unroll
        for (int h = 0; h < NH; h++)
            if (sl.t + h * G::TPB < 2 * D * G::HF && hv[h] >= 0) q[hs[h]] = raw[h];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int hc = sl.t + h * G::TPB;
            if (hc < 2 * D * G::HF && hv[h] < 0) {
                const int side = hc / G::HF, m = hc % G::HF;
#define AFMG_H2(S) halo_phase2<D, N, S, T>(q, m, o, raw[h], hv[h], pfl)
                AFMG_SIDE_SWITCH(side, AFMG_H2)
#undef AFMG_H2
            }
        }
    }
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int it = 0; it < NE; it++) {
        const int e = sl.t + it * G::TPB;
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        T v;
        if (D == 2) {
            v = T(0.5) * q[qpad<D, N>(I, J, 0)] + T(0.25) * q[qpad<D, N>(I + sx, J, 0)] +
                T(0.25) * q[qpad<D, N>(I, J + sy, 0)];
        } else {
            v = T(0.25) * (((q[qpad<D, N>(I, J, K)] + q[qpad<D, N>(I + sx, J, K)]) + q[qpad<D, N>(I, J + sy, K)]) +
                           q[qpad<D, N>(I, J, K + sz)]);
        }
        a.u[bo + e] = uf[it] + v;
    }
}

// ---------------------------------------------------------------------------
// end of a cycle: restriction of u and the composite leaf residual
// ---------------------------------------------------------------------------
// Boxes of level l: the octant of the parent receives mean(u) (l >= 2); on
// leaves r = rho - L u, and (max |r|, sum r^2 h^D) goes to partial: per
// workgroup at partial[part0 + workgroup], or, with part0 < 0 (forests), per
// leaf box at partial[box].  With rout set, the leaf residual is also stored
// there rounded to FP32: the right-hand side of the correction solve of the
// mixed-precision refinement.
template <int D, int N, typename T, int W, bool F>
__global__ __launch_bounds__(W) void k_final(LevelArgs<T> a, double *partial, int64_t part0, double hD,
                                             float *__restrict__ rout) {
    using G = Geo<D, N>;
    constexpr int NW = W / 64;  // waves per workgroup
    __shared__ T sm[(W / G::TPB) * G::PC];
    __shared__ double red_m[NW], red_s[NW];
    const Slot<D, N> sl = slot_lvl<D, N, W, F>(a);
    T *s = sm + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const bool leaf = bi.flags & FLAG_LEAF;
    constexpr int NPC = G::HC / G::TPB, NB = D == 3 ? 8 : 4;
    T rf[NPC][NB];
    Stager<D, N, T> st;
    // rows first (one tree: padding slots load a valid box too), then what
    // depends on the box record: ghosts and rho of leaves
    const bool act = sl.valid;
    if (!F || act) {
        st.load(bi, a.u + bo, a.u, a.bc, a.homog, sl.t, leaf, a.h);
        if (leaf) {
#pragma unroll
            for (int it = 0; it < NPC; it++)
#pragma unroll
                for (int q = 0; q < NB; q++) {
                    int i, j, k;
                    block_cell<D, N>(sl.t + it * G::TPB, q, i, j, k);
                    rf[it][q] = a.rho[bo + cpos<D, N>(i, j, k)];
                }
        }
        st.stage(s, sl.t);
    }
    __syncthreads();
    if (act && leaf) st.end(s, sl.t);
    __syncthreads();
    // each thread: 2^D blocks of cells = parent cells; the block mean of u
    // goes to the parent, the residuals of leaves stay in registers
    double mx = 0.0, ss = 0.0;
    if (act) {
        const T w = D == 3 ? T(0.125) : T(0.25);
        const int flags = bi.flags;
        const int64_t p = bi.parent;
#pragma unroll
        for (int it = 0; it < NPC; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            T su = T(0);
            if (leaf) {
                // all residuals of the block first, then the optional FP32 copies
                double r[NB];
                int e[NB];
#pragma unroll
                for (int q = 0; q < NB; q++) {
                    int i, j, k;
                    block_cell<D, N>(pc, q, i, j, k);
                    const T uc = s[padi<D, N>(i, j, k)];
                    su += uc;
                    e[q] = cpos<D, N>(i, j, k);
                    r[q] = (double)(rf[it][q] - (nb_sum<D, N, T>(s, i, j, k) - T(2 * D) * uc) * a.ih2);
                }
                if (rout) {
#pragma unroll
                    for (int q = 0; q < NB; q++) rout[bo + e[q]] = (float)r[q];
                }
#pragma unroll
                for (int q = 0; q < NB; q++) {
                    mx = fmax(mx, fabs(r[q]));
                    ss += r[q] * r[q];
                }
            } else {
                for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
                    for (int dj = 0; dj < 2; dj++)
                        for (int di = 0; di < 2; di++)
                            su += s[padi<D, N>(2 * I + di, 2 * J + dj, D == 3 ? 2 * K + dk : 0)];
            }
            if (p >= 0) {
                const int X = obit(flags, 0) * G::H + I, Y = obit(flags, 1) * G::H + J,
                          Z = D == 3 ? obit(flags, 2) * G::H + K : 0;
                a.u[(size_t)p * G::C + cpos<D, N>(X, Y, Z)] = w * su;
            }
        }
    }
    // reduce over the TPB threads of the box (8 or 16 lanes in 2D, one wave
    // in 3D with 8^3 cells), or over each wave of a box of several waves
    constexpr int LW = G::TPB < 64 ? G::TPB : 64;
    for (int o = LW / 2; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        ss += __shfl_xor(ss, o);
    }
    if (part0 < 0) {
        if constexpr (G::TPB > 64) {
            // the waves of the box through LDS, in wave order
            constexpr int WPB = G::TPB / 64;
            const int wave = (int)threadIdx.x / 64;
            if ((threadIdx.x & 63) == 0) {
                red_m[wave] = mx;
                red_s[wave] = ss;
            }
            __syncthreads();
            if (sl.t == 0) {
                for (int q = 1; q < WPB; q++) {
                    mx = fmax(mx, red_m[wave + q]);
                    ss += red_s[wave + q];
                }
            }
        }
        if (act && leaf && sl.t == 0) {
            partial[2 * sl.b + 0] = mx;
            partial[2 * sl.b + 1] = ss * hD;
        }
        return;
    }
    // then over the boxes of the wave and the waves of the workgroup
    for (int o = 32; o >= G::TPB; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        ss += __shfl_xor(ss, o);
    }
    const int wave = (int)threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red_m[wave] = mx;
        red_s[wave] = ss;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red_m[0], t = red_s[0];
        for (int q = 1; q < NW; q++) {
            m = fmax(m, red_m[q]);
            t += red_s[q];
        }
        partial[2 * (part0 + blockIdx.x) + 0] = m;
        partial[2 * (part0 + blockIdx.x) + 1] = t * hD;
    }
}

// ---------------------------------------------------------------------------
// operators (paper §3.4, §3.5)
// ---------------------------------------------------------------------------
// Level kernels of a tree with an operator (LevelArgs::opk != 0; one tree,
// 256-thread workgroups).  A box is staged in LDS with its side ghosts as in
// the Laplacian's kernels, and its coefficients eps with their own ghosts:
// the coefficient of the cell across the side, the face cell's own on a
// physical side, and on a refinement side that of the coarse cell holding
// the ghost centre (the jumps lie on coarse-grid faces, paper §3.4).

// left edge (x = r) of box b on a level with cell size h
template <int N, typename T>
__device__ __forceinline__ T box_x0(const int32_t *__restrict__ bx, int64_t b, T h) {
    return T(bx[b] - 1) * T(N) * h;
}

// sum over the 2D sides of w_s u_s, and in dg the sum of the w_s, for cell
// (i, j, k); s and se are the padded box and its coefficients in LDS
template <int D, int N, typename T>
__device__ __forceinline__ T op_sum(const T *s, const T *se, int i, int j, int k, int opk, T x0, T h, T &dg) {
    int nb[6];
    nb[0] = padi<D, N>(i - 1, j, k);
    nb[1] = padi<D, N>(i + 1, j, k);
    nb[2] = padi<D, N>(i, j - 1, k);
    nb[3] = padi<D, N>(i, j + 1, k);
    nb[4] = padi<D, N>(i, j, k - 1);
    nb[5] = padi<D, N>(i, j, k + 1);
    const bool eps = opk & OPK_EPS, cyl = opk & OPK_CYL;
    const T ec = eps ? se[padi<D, N>(i, j, k)] : T(1);
    const T rc = x0 + (T(i) + T(0.5)) * h;
    T sum = T(0), d = T(0);
#pragma unroll
    for (int q = 0; q < 2 * D; q++) {
        T w = T(1);
        if (eps) {
            const T en = se[nb[q]];
            w = T(2) * ec * en / (ec + en);
        }
        if (cyl && q < 2) w *= (x0 + T(i + q) * h) / rc;
        sum += w * s[nb[q]];
        d += w;
    }
    dg = d;
    return sum;
}

// h^2 (L u) at cell (i, j, k)
template <int D, int N, typename T>
__device__ __forceinline__ T op_h2(const T *s, const T *se, int i, int j, int k, int opk, T x0, T h) {
    T dg;
    const T sm = op_sum<D, N, T>(s, se, i, j, k, opk, x0, h, dg);
    return sm - dg * s[padi<D, N>(i, j, k)];
}

// restriction weight of fine cell column i (0-based in the box): 1, or the
// radius of its centre for the cylindrical form
template <typename T>
__device__ __forceinline__ T vol_w(bool cyl, T x0, T h, int i) {
    return cyl ? x0 + (T(i) + T(0.5)) * h : T(1);
}

// Side ghosts of the coefficients (copy rules above); load / stage / end as
// in Stager.
template <int D, int N, typename T>
struct EpsStager {
    using G = Geo<D, N>;
    T raw[6];
    int v[6];
    T rowv[2][G::HN];
    __device__ __forceinline__ void load(const BoxInfo &bi, const T *__restrict__ eb, const T *__restrict__ e,
                                         int t) {
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int m = 0; m < G::HN; m++) rowv[c][m] = eb[c * G::HALF + t * G::HN + m];
        // a physical side reads an in-range value of box 0 and ignores it
        raw[0] = ghost_raw<D, N, 0, T>(bi, t, e, nullptr, 1, v[0]);
        raw[1] = ghost_raw<D, N, 1, T>(bi, t, e, nullptr, 1, v[1]);
        raw[2] = ghost_raw<D, N, 2, T>(bi, t, e, nullptr, 1, v[2]);
        raw[3] = ghost_raw<D, N, 3, T>(bi, t, e, nullptr, 1, v[3]);
        if (D == 3) {
            raw[4] = ghost_raw<D, N, 4, T>(bi, t, e, nullptr, 1, v[4]);
            raw[5] = ghost_raw<D, N, 5, T>(bi, t, e, nullptr, 1, v[5]);
        }
    }
    __device__ __forceinline__ void stage(T *s, int t) const {
        int j, k;
        row_of<D, N>(t, j, k);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int p = (c + D + j + k) & 1;
#pragma unroll
            for (int m = 0; m < G::HN; m++) s[padi<D, N>(2 * m + p, j, k)] = rowv[c][m];
        }
    }
    template <int S>
    __device__ __forceinline__ void end1(T *s, int t) const {
        int x[3];
        face_cell<D, N, S>(t, x);
        s[ghost_slot<D, N, S>(t)] = v[S] == -1 ? s[padi<D, N>(x[0], x[1], x[2])] : raw[S];
    }
    __device__ void end(T *s, int t) const {
        end1<0>(s, t);
        end1<1>(s, t);
        end1<2>(s, t);
        end1<3>(s, t);
        if (D == 3) {
            end1<4>(s, t);
            end1<5>(s, t);
        }
    }
};

// Gauss-Seidel red-black half sweep (paper §3.1) with the operator: each
// cell of `colour` solves its own equation with the neighbours and ghosts
// of the old state, u_c = (sum w_s u_s - h^2 rho_c) / sum w_s.  The whole
// box is staged; the cells written are the updated colour, which no ghost of
// an updated cell reads (its neighbours across sides are the other colour).
// Workgroup size of the operator kernels: 128 threads (two 8^3 boxes in 3D,
// sixteen 8^2 boxes in 2D), or one box where a box needs more threads.  They
// stage padded boxes of u and eps (16 KB per 8^3 box); 128-thread workgroups
// leave more of them resident per CU than 256-thread ones (the half sweep on
// 256^3: 106 against 128 us per launch).
template <int D, int N>
constexpr int opw() { return op_wg(D, N); }

template <int D, int N, typename T>
__global__ __launch_bounds__((opw<D, N>())) void k_vgsrb(LevelArgs<T> a, int colour) {
    using G = Geo<D, N>;
    constexpr int HN = G::HN;
    __shared__ T sm[opw<D, N>() / G::TPB * G::PC];
    __shared__ T sme[opw<D, N>() / G::TPB * G::PC];
    const Slot<D, N> sl = slot_of<D, N, opw<D, N>()>(a.b0, a.nb, a.no_remap == 0);
    T *s = sm + sl.slot * G::PC, *se = sme + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const int r = sl.t;
    int j, k;
    row_of<D, N>(r, j, k);
    const int p = (colour + D + j + k) & 1;
    const int own0 = colour * G::HALF + r * HN;
    const bool act = sl.valid, eps = a.opk & OPK_EPS;
    T rr[HN];
    Stager<D, N, T, true> st;
    st.bil = (a.opk & OPK_GHOST_BIL) != 0;
    EpsStager<D, N, T> es;
    // padding slots (sl.b clamped to a valid box) load too
#pragma unroll
    for (int m = 0; m < HN; m++) rr[m] = a.rho[bo + own0 + m];
    st.load(bi, a.u + bo, a.u, a.bc, a.homog, r, true, a.h);
    if (eps) es.load(bi, a.eps + bo, a.eps, r);
    st.stage(s, r);
    if (eps) es.stage(se, r);
    __syncthreads();
    if (act) {
        st.end(s, r);
        if (eps) es.end(se, r);
    }
    __syncthreads();
    if (!act) return;
    const T x0 = (a.opk & OPK_CYL) ? box_x0<N, T>(a.bx, sl.b, a.h) : T(0);
    T out[HN];
#pragma unroll
    for (int m = 0; m < HN; m++) {
        T dg;
        const T sum = op_sum<D, N, T>(s, se, 2 * m + p, j, k, a.opk, x0, a.h, dg);
        out[m] = (sum - a.h2 * rr[m]) / dg;
    }
#pragma unroll
    for (int m = 0; m < HN; m++) a.u[bo + own0 + m] = out[m];
}

// The same half sweep with one row of a box per thread, in the Laplacian
// half sweep's form: only the other colour of u and of eps is staged in LDS
// (the cells of one colour have only the other colour as neighbours), the
// updated colour's eps, right-hand side and, next to physical or refinement
// sides, old values stay in registers, and each thread fetches the ghosts
// of u and of eps across the sides of its own cells.  Face weights, the
// cylindrical factors and the order of the sum over sides (-x, +x, -y, +y,
// -z, +z) are those of op_sum, and the ghosts those of the staging helpers
// (eps across a physical side: the face cell's own).  Default refinement
// ghosts only: the bilinear scheme reads cells of both colours and runs
// k_vgsrb.
template <int D, int N, typename T, int W>
__global__ __launch_bounds__(W) void k_vgsrb_row(LevelArgs<T> a, int colour) {
    using G = Geo<D, N>;
    constexpr int HN = G::HN;
    __shared__ T so[(W / G::TPB) * oblock<D, N>()];
    __shared__ T soe[(W / G::TPB) * oblock<D, N>()];
    const Slot<D, N> sl = slot_of<D, N, W>(a.b0, a.nb, a.no_remap == 0, colour == 1);
    T *s = so + sl.slot * oblock<D, N>();
    T *se = soe + sl.slot * oblock<D, N>();
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const int r = sl.t;
    int j, k;
    row_of<D, N>(r, j, k);
    const int p = (colour + D + j + k) & 1;  // x parity of the updated cells in this row
    const int own0 = colour * G::HALF + r * HN, oth0 = (1 - colour) * G::HALF + r * HN;
    const bool eps = a.opk & OPK_EPS, cyl = a.opk & OPK_CYL;
    T rr[HN], ow[HN], eo[HN], gy[HN], gz[HN], ey[HN], ez[HN];
    T gx = T(0), ex = T(0);
    int vx = 0, vy = 0, vz = 0;
#pragma unroll
    for (int m = 0; m < HN; m++) {
        ow[m] = T(0);
        eo[m] = T(1);
        gy[m] = gz[m] = ey[m] = ez[m] = T(0);
    }
    // ghosts across a side whose neighbour is a sibling in this workgroup
    // come from its staged other colour of u and eps (as in k_gsrb; decided
    // after the box's own loads are issued: it needs the box record)
    int qx = -1, qy = -1, qz = -1;
    // padding slots (sl.b clamped to a valid box) load too
    {
        T ot[HN], et[HN];
#pragma unroll
        for (int m = 0; m < HN; m++) ot[m] = a.u[bo + oth0 + m];
#pragma unroll
        for (int m = 0; m < HN; m++) rr[m] = a.rho[bo + own0 + m];
        if (eps) {
#pragma unroll
            for (int m = 0; m < HN; m++) eo[m] = a.eps[bo + own0 + m];
#pragma unroll
            for (int m = 0; m < HN; m++) et[m] = a.eps[bo + oth0 + m];
        }
        qx = sib_slot<D, N, W, 0>(p == 0 ? bi.nbr[0] : bi.nbr[1], sl, a.b0, a.nb);
        qy = sib_slot<D, N, W, 1>(j == 0 ? bi.nbr[2] : bi.nbr[3], sl, a.b0, a.nb);
        if (D == 3) qz = sib_slot<D, N, W, 2>(k == 0 ? bi.nbr[4] : bi.nbr[5], sl, a.b0, a.nb);
        // x ghost of the row end cell (side 0 when the row starts with this colour)
        int dv;
        if (qx < 0) {
            if (p == 0) {
                gx = ghost_raw<D, N, 0, T>(bi, r, a.u, a.bc, a.homog, vx);
                if (eps) ex = ghost_raw<D, N, 0, T>(bi, r, a.eps, nullptr, 1, dv);
            } else {
                gx = ghost_raw<D, N, 1, T>(bi, r, a.u, a.bc, a.homog, vx);
                if (eps) ex = ghost_raw<D, N, 1, T>(bi, r, a.eps, nullptr, 1, dv);
            }
        }
        bool need_own = vx < 0;
        // y / z ghosts: across a same-level side, one row of the neighbour's
        // other colour (row j' = N-1-j, resp. k' = N-1-k); else per cell
        const bool yrow = (j == 0 || j == N - 1) && qy < 0, zrow = D == 3 && (k == 0 || k == N - 1) && qz < 0;
        const bool yfast = bi.nbr[2] >= 0 && bi.nbr[3] >= 0;
        const bool zfast = D == 3 && bi.nbr[4] >= 0 && bi.nbr[5] >= 0;
        if (yfast && yrow) {
            vy = bi.nbr[j == 0 ? 2 : 3];
            const size_t o = (size_t)vy * G::C + oth0 + ((D == 3 ? N * k : 0) + (N - 1 - j) - r) * HN;
#pragma unroll
            for (int m = 0; m < HN; m++) gy[m] = a.u[o + m];
            if (eps) {
#pragma unroll
                for (int m = 0; m < HN; m++) ey[m] = a.eps[o + m];
            }
        }
        if (zfast && zrow) {
            vz = bi.nbr[k == 0 ? 4 : 5];
            const size_t o = (size_t)vz * G::C + oth0 + ((N - 1 - k) * N + j - r) * HN;
#pragma unroll
            for (int m = 0; m < HN; m++) gz[m] = a.u[o + m];
            if (eps) {
#pragma unroll
                for (int m = 0; m < HN; m++) ez[m] = a.eps[o + m];
            }
        }
        __asm__ volatile("" ::: "memory");
        // (the coefficient ghost is the u ghost's cell in eps: a physical
        // side reads an in-range value of box 0 and ignores it)
        if (!yfast && yrow) {
#pragma unroll
            for (int m = 0; m < HN; m++) {
                const int fm = (2 * m + p) + (D == 3 ? N * k : 0);
                const T *pu, *pe;
                if (j == 0) {
                    pu = ghost_ptr<D, N, 2, T>(bi, fm, a.u, a.bc, a.homog, vy);
                    pe = ghost_ptr<D, N, 2, T>(bi, fm, a.eps, nullptr, 1, vy);
                } else {
                    pu = ghost_ptr<D, N, 3, T>(bi, fm, a.u, a.bc, a.homog, vy);
                    pe = ghost_ptr<D, N, 3, T>(bi, fm, a.eps, nullptr, 1, vy);
                }
                gy[m] = *pu;
                if (eps) ey[m] = *pe;
            }
            need_own |= vy < 0;
        }
        if (D == 3 && !zfast && zrow) {
#pragma unroll
            for (int m = 0; m < HN; m++) {
                const int fm = (2 * m + p) + N * j;
                const T *pu, *pe;
                if (k == 0) {
                    pu = ghost_ptr<D, N, 4, T>(bi, fm, a.u, a.bc, a.homog, vz);
                    pe = ghost_ptr<D, N, 4, T>(bi, fm, a.eps, nullptr, 1, vz);
                } else {
                    pu = ghost_ptr<D, N, 5, T>(bi, fm, a.u, a.bc, a.homog, vz);
                    pe = ghost_ptr<D, N, 5, T>(bi, fm, a.eps, nullptr, 1, vz);
                }
                gz[m] = *pu;
                if (eps) ez[m] = *pe;
            }
            need_own |= vz < 0;
        }
        if (need_own) {
#pragma unroll
            for (int m = 0; m < HN; m++) ow[m] = a.u[bo + own0 + m];
        }
#pragma unroll
        for (int m = 0; m < HN; m++) s[m * G::TPB + r] = ot[m];
        if (eps) {
#pragma unroll
            for (int m = 0; m < HN; m++) se[m * G::TPB + r] = et[m];
        }
    }
    __syncthreads();
    if (!sl.valid) return;
    if (qx >= 0) {
        gx = so[qx * oblock<D, N>() + oslot<D, N>(p == 0 ? N - 1 : 0, j, k)];
        if (eps) ex = soe[qx * oblock<D, N>() + oslot<D, N>(p == 0 ? N - 1 : 0, j, k)];
    }
    if (qy >= 0 && (j == 0 || j == N - 1)) {
#pragma unroll
        for (int m = 0; m < HN; m++) {
            const int o = qy * oblock<D, N>() + oslot<D, N>(2 * m + p, j == 0 ? N - 1 : 0, k);
            gy[m] = so[o];
            if (eps) ey[m] = soe[o];
        }
    }
    if (D == 3 && qz >= 0 && (k == 0 || k == N - 1)) {
#pragma unroll
        for (int m = 0; m < HN; m++) {
            const int o = qz * oblock<D, N>() + oslot<D, N>(2 * m + p, j, k == 0 ? N - 1 : 0);
            gz[m] = so[o];
            if (eps) ez[m] = soe[o];
        }
    }
    const T x0 = cyl ? box_x0<N, T>(a.bx, sl.b, a.h) : T(0);
    const int fl = bi.flags;
    const T h = a.h;
    T out[HN];
#pragma unroll
    for (int m = 0; m < HN; m++) {
        const int i = 2 * m + p;
        T un[6], en[6];
        un[0] = i > 0 ? s[oslot<D, N>(i - 1, j, k)] : gs_finish<D, N, 0, T>(s, gx, vx, ow[m], a.homog, i, j, k, fl, h);
        un[1] = i < N - 1 ? s[oslot<D, N>(i + 1, j, k)] : gs_finish<D, N, 1, T>(s, gx, vx, ow[m], a.homog, i, j, k, fl, h);
        un[2] = j > 0 ? s[oslot<D, N>(i, j - 1, k)] : gs_finish<D, N, 2, T>(s, gy[m], vy, ow[m], a.homog, i, j, k, fl, h);
        un[3] = j < N - 1 ? s[oslot<D, N>(i, j + 1, k)] : gs_finish<D, N, 3, T>(s, gy[m], vy, ow[m], a.homog, i, j, k, fl, h);
        if (D == 3) {
            un[4] = k > 0 ? s[oslot<D, N>(i, j, k - 1)] : gs_finish<D, N, 4, T>(s, gz[m], vz, ow[m], a.homog, i, j, k, fl, h);
            un[5] = k < N - 1 ? s[oslot<D, N>(i, j, k + 1)] : gs_finish<D, N, 5, T>(s, gz[m], vz, ow[m], a.homog, i, j, k, fl, h);
        }
        const T ec = eo[m];
        if (eps) {
            en[0] = i > 0 ? se[oslot<D, N>(i - 1, j, k)] : (vx == -1 ? ec : ex);
            en[1] = i < N - 1 ? se[oslot<D, N>(i + 1, j, k)] : (vx == -1 ? ec : ex);
            en[2] = j > 0 ? se[oslot<D, N>(i, j - 1, k)] : (vy == -1 ? ec : ey[m]);
            en[3] = j < N - 1 ? se[oslot<D, N>(i, j + 1, k)] : (vy == -1 ? ec : ey[m]);
            if (D == 3) {
                en[4] = k > 0 ? se[oslot<D, N>(i, j, k - 1)] : (vz == -1 ? ec : ez[m]);
                en[5] = k < N - 1 ? se[oslot<D, N>(i, j, k + 1)] : (vz == -1 ? ec : ez[m]);
            }
        }
        const T rc = x0 + (T(i) + T(0.5)) * h;
        T sum = T(0), d = T(0);
#pragma unroll
        for (int q = 0; q < 2 * D; q++) {
            T w = T(1);
            if (eps) w = T(2) * ec * en[q] / (ec + en[q]);
            if (cyl && q < 2) w *= (x0 + T(i + q) * h) / rc;
            sum += w * un[q];
            d += w;
        }
        out[m] = (sum - a.h2 * rr[m]) / d;
        // one cell's neighbours in registers at a time
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int m = 0; m < HN; m++) a.u[bo + own0 + m] = out[m];
}

// residual r = rho - L u on the boxes of level l; the parent's octant
// receives the means of u and of r (volume means in the cylindrical form)
template <int D, int N, typename T>
__global__ __launch_bounds__((opw<D, N>())) void k_vresid_restrict(LevelArgs<T> a) {
    using G = Geo<D, N>;
    __shared__ T sm[opw<D, N>() / G::TPB * G::PC];
    __shared__ T sme[opw<D, N>() / G::TPB * G::PC];
    const Slot<D, N> sl = slot_of<D, N, opw<D, N>()>(a.b0, a.nb, a.no_remap == 0);
    T *s = sm + sl.slot * G::PC, *se = sme + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    constexpr int NPC = G::HC / G::TPB, NB = D == 3 ? 8 : 4;
    const bool act = sl.valid, eps = a.opk & OPK_EPS, cyl = a.opk & OPK_CYL;
    T rf[NPC][NB];
    Stager<D, N, T, true> st;
    st.bil = (a.opk & OPK_GHOST_BIL) != 0;
    EpsStager<D, N, T> es;
#pragma unroll
    for (int it = 0; it < NPC; it++)
#pragma unroll
        for (int q = 0; q < NB; q++) {
            int i, j, k;
            block_cell<D, N>(sl.t + it * G::TPB, q, i, j, k);
            rf[it][q] = a.rho[bo + cpos<D, N>(i, j, k)];
        }
    st.load(bi, a.u + bo, a.u, a.bc, a.homog, sl.t, true, a.h);
    if (eps) es.load(bi, a.eps + bo, a.eps, sl.t);
    st.stage(s, sl.t);
    if (eps) es.stage(se, sl.t);
    __syncthreads();
    if (act) {
        st.end(s, sl.t);
        if (eps) es.end(se, sl.t);
    }
    __syncthreads();
    if (!act) return;
    const T x0 = cyl ? box_x0<N, T>(a.bx, sl.b, a.h) : T(0);
    const T w = D == 3 ? T(0.125) : T(0.25);
    const int flags = bi.flags;
    const int64_t p = bi.parent;
#pragma unroll
    for (int it = 0; it < NPC; it++) {
        const int pc = sl.t + it * G::TPB;
        const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
        T su = T(0), sr = T(0), vol = T(0);
        // two fine cells at a time: the full unroll needs 220 VGPRs
#pragma unroll 2
        for (int q = 0; q < NB; q++) {
            int i, j, k;
            block_cell<D, N>(pc, q, i, j, k);
            const T uc = s[padi<D, N>(i, j, k)];
            const T res = rf[it][q] - op_h2<D, N, T>(s, se, i, j, k, a.opk, x0, a.h) * a.ih2;
            const T wq = vol_w<T>(cyl, x0, a.h, i);
            su += cyl ? wq * uc : uc;
            sr += cyl ? wq * res : res;
            vol += wq;
        }
        const int X = obit(flags, 0) * G::H + I, Y = obit(flags, 1) * G::H + J,
                  Z = D == 3 ? obit(flags, 2) * G::H + K : 0;
        const size_t o = (size_t)p * G::C + cpos<D, N>(X, Y, Z);
        a.u[o] = cyl ? su / vol : w * su;
        a.rho[o] = cyl ? sr / vol : w * sr;
    }
}

// boxes of level l-1: uold <- u; on parents rho <- rbar + L_H u
template <int D, int N, typename T>
__global__ __launch_bounds__((opw<D, N>())) void k_vcoarse_rhs(LevelArgs<T> a) {
    using G = Geo<D, N>;
    __shared__ T sm[opw<D, N>() / G::TPB * G::PC];
    __shared__ T sme[opw<D, N>() / G::TPB * G::PC];
    const Slot<D, N> sl = slot_of<D, N, opw<D, N>()>(a.b0, a.nb, a.no_remap == 0);
    T *s = sm + sl.slot * G::PC, *se = sme + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const bool parent = !(bi.flags & FLAG_LEAF);
    const bool act = sl.valid, eps = (a.opk & OPK_EPS) && parent;
    constexpr int NE = G::C / G::TPB;
    T rf[NE];
    Stager<D, N, T, true> st;
    st.bil = (a.opk & OPK_GHOST_BIL) != 0;
    EpsStager<D, N, T> es;
    st.load(bi, a.u + bo, a.u, a.bc, a.homog, sl.t, parent, a.h);
    if (parent) {
#pragma unroll
        for (int it = 0; it < NE; it++) rf[it] = a.rho[bo + sl.t + it * G::TPB];
    }
    if (eps) es.load(bi, a.eps + bo, a.eps, sl.t);
    st.stage(s, sl.t);
    if (eps) es.stage(se, sl.t);
    __syncthreads();
    if (act) {
        for (int e = sl.t; e < G::C; e += G::TPB) {
            int i, j, k;
            cell_of<D, N>(e, i, j, k);
            a.uold[bo + e] = s[padi<D, N>(i, j, k)];
        }
    }
    if (act && parent) {
        st.end(s, sl.t);
        if (eps) es.end(se, sl.t);
    }
    __syncthreads();
    if (!act || !parent) return;
    const T x0 = (a.opk & OPK_CYL) ? box_x0<N, T>(a.bx, sl.b, a.h) : T(0);
#pragma unroll
    for (int it = 0; it < NE; it++) {
        const int e = sl.t + it * G::TPB;
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        a.rho[bo + e] = rf[it] + op_h2<D, N, T>(s, se, i, j, k, a.opk, x0, a.h) * a.ih2;
    }
}

// end of a cycle with the operator: the parent's octant receives the mean of
// u (volume mean in the cylindrical form); on leaves r = rho - L u and its
// (max |r|, sum r^2 h^D) per workgroup at partial[part0 + workgroup]
template <int D, int N, typename T>
__global__ __launch_bounds__((opw<D, N>())) void k_vfinal(LevelArgs<T> a, double *partial, int64_t part0, double hD) {
    using G = Geo<D, N>;
    constexpr int NW = opw<D, N>() / 64;
    __shared__ T sm[opw<D, N>() / G::TPB * G::PC];
    __shared__ T sme[opw<D, N>() / G::TPB * G::PC];
    __shared__ double red_m[NW], red_s[NW];
    const Slot<D, N> sl = slot_of<D, N, opw<D, N>()>(a.b0, a.nb, a.no_remap == 0);
    T *s = sm + sl.slot * G::PC, *se = sme + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const bool leaf = bi.flags & FLAG_LEAF;
    const bool act = sl.valid, eps = (a.opk & OPK_EPS) && leaf, cyl = a.opk & OPK_CYL;
    constexpr int NPC = G::HC / G::TPB, NB = D == 3 ? 8 : 4;
    T rf[NPC][NB];
    Stager<D, N, T, true> st;
    st.bil = (a.opk & OPK_GHOST_BIL) != 0;
    EpsStager<D, N, T> es;
    st.load(bi, a.u + bo, a.u, a.bc, a.homog, sl.t, leaf, a.h);
    if (leaf) {
#pragma unroll
        for (int it = 0; it < NPC; it++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
                int i, j, k;
                block_cell<D, N>(sl.t + it * G::TPB, q, i, j, k);
                rf[it][q] = a.rho[bo + cpos<D, N>(i, j, k)];
            }
    }
    if (eps) es.load(bi, a.eps + bo, a.eps, sl.t);
    st.stage(s, sl.t);
    if (eps) es.stage(se, sl.t);
    __syncthreads();
    if (act && leaf) {
        st.end(s, sl.t);
        if (eps) es.end(se, sl.t);
    }
    __syncthreads();
    double mx = 0.0, ss = 0.0;
    if (act) {
        const T x0 = cyl ? box_x0<N, T>(a.bx, sl.b, a.h) : T(0);
        const T w = D == 3 ? T(0.125) : T(0.25);
        const int flags = bi.flags;
        const int64_t p = bi.parent;
#pragma unroll
        for (int it = 0; it < NPC; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            T su = T(0), vol = T(0);
#pragma unroll
            for (int q = 0; q < NB; q++) {
                int i, j, k;
                block_cell<D, N>(pc, q, i, j, k);
                const T uc = s[padi<D, N>(i, j, k)];
                const T wq = vol_w<T>(cyl, x0, a.h, i);
                su += cyl ? wq * uc : uc;
                vol += wq;
                if (leaf) {
                    const double r = (double)(rf[it][q] - op_h2<D, N, T>(s, se, i, j, k, a.opk, x0, a.h) * a.ih2);
                    mx = fmax(mx, fabs(r));
                    ss += r * r;
                }
            }
            if (p >= 0) {
                const int X = obit(flags, 0) * G::H + I, Y = obit(flags, 1) * G::H + J,
                          Z = D == 3 ? obit(flags, 2) * G::H + K : 0;
                a.u[(size_t)p * G::C + cpos<D, N>(X, Y, Z)] = cyl ? su / vol : w * su;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        ss += __shfl_xor(ss, o);
    }
    const int wave = (int)threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red_m[wave] = mx;
        red_s[wave] = ss;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red_m[0], t = red_s[0];
        for (int q = 1; q < NW; q++) {
            m = fmax(m, red_m[q]);
            t += red_s[q];
        }
        partial[2 * (part0 + blockIdx.x) + 0] = m;
        partial[2 * (part0 + blockIdx.x) + 1] = t * hD;
    }
}

// coarse-grid correction with the eps-weighted prolongation: along each
// axis d the fine cell lies a quarter coarse cell from its coarse cell P
// towards P + s_d e_d; the piecewise-linear profile that is continuous in
// value and in flux eps du/dx across the face between them (the local
// reconstruction of paper §3.4) gives
//   u += d(P) + sum_d eps_d / (2 (eps_P + eps_d)) (d(P + s_d e_d) - d(P)),
// d = u - uold of the parent level; with equal eps this is the default
// interpolation.  The coefficients of the parent's octant and its halo are
// staged beside the deltas, with the copy rules of the coefficient ghosts.
template <int D, int N, typename T>
__global__ __launch_bounds__((opw<D, N>())) void k_vprolong(LevelArgs<T> a) {
    using G = Geo<D, N>;
    constexpr int NH = (2 * D * G::HF + G::TPB - 1) / G::TPB;
    constexpr int NO = G::HC / G::TPB;
    constexpr int NE = G::C / G::TPB;
    __shared__ T qs[opw<D, N>() / G::TPB * G::QC];
    __shared__ T qes[opw<D, N>() / G::TPB * G::QC];
    const Slot<D, N> sl = slot_of<D, N, opw<D, N>()>(a.b0, a.nb, a.no_remap == 0);
    T *q = qs + sl.slot * G::QC, *qe = qes + sl.slot * G::QC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    const bool act = sl.valid;
    const bool eps = a.opk & OPK_PROLONG_EPS;
    const int bil = (a.opk & OPK_GHOST_BIL) ? 1 : 0;
    T raw[NH], rawe[NH], uf[NE];
    int hv[NH], hs[NH];
#pragma unroll
    for (int it = 0; it < NE; it++) uf[it] = a.u[bo + sl.t + it * G::TPB];
    const int flags = bi.flags;
    const int o[3] = {obit(flags, 0) * G::H, obit(flags, 1) * G::H, D == 3 ? obit(flags, 2) * G::H : 0};
    const int64_t p = bi.parent;
    const BoxInfo pi = load_box<D, N>(a.info, p);
    const int pfl = pi.flags;
    {
        T od[NO], oe[NO];
#pragma unroll
        for (int it = 0; it < NO; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            const size_t oo = (size_t)p * G::C + cpos<D, N>(o[0] + I, o[1] + J, o[2] + K);
            od[it] = a.u[oo] - a.uold[oo];
            oe[it] = eps ? a.eps[oo] : T(1);
        }
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int hc = sl.t + h * G::TPB;
            size_t ho = (size_t)p * G::C;
            hv[h] = 0;
            hs[h] = 0;
            if (hc < 2 * D * G::HF) {
                const int side = hc / G::HF, m = hc % G::HF;
#define AFMG_H1(S) ho = halo_addr<D, N, S>(m, o, pi, p, hv[h], hs[h])
                AFMG_SIDE_SWITCH(side, AFMG_H1)
#undef AFMG_H1
            }
            raw[h] = a.u[ho] - a.uold[ho];
            rawe[h] = eps ? a.eps[ho] : T(1);
        }
#pragma unroll
        for (int it = 0; it < NO; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            q[qpad<D, N>(I, J, K)] = od[it];
            qe[qpad<D, N>(I, J, K)] = oe[it];
        }
#pragma unroll
        for (int h = 0; h < NH; h++)
            if (sl.t + h * G::TPB < 2 * D * G::HF) {
                if (hv[h] >= 0) q[hs[h]] = raw[h];
                if (hv[h] != -1) qe[hs[h]] = rawe[h];
            }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int hc = sl.t + h * G::TPB;
            if (hc < 2 * D * G::HF && hv[h] < 0) {
                const int side = hc / G::HF, m = hc % G::HF;
#define AFMG_H2(S) halo_phase2<D, N, S, T, true>(q, m, o, raw[h], hv[h], pfl, bil)
                AFMG_SIDE_SWITCH(side, AFMG_H2)
#undef AFMG_H2
                if (eps && hv[h] == -1) {
                    // physical side of the parent: the face cell's own coefficient
                    int L[3], X[3];
#define AFMG_H3(S)                                          \
    {                                                       \
        halo_cell<D, N, S>(m, o, L, X);                     \
        int f[3] = {L[0], L[1], L[2]};                      \
        f[SideOf<S>::d] = SideOf<S>::hi ? L[SideOf<S>::d] - 1 : 0; \
        qe[qpad<D, N>(L[0], L[1], L[2])] = qe[qpad<D, N>(f[0], f[1], f[2])]; \
    }
                    AFMG_SIDE_SWITCH(side, AFMG_H3)
#undef AFMG_H3
                }
            }
        }
    }
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int it = 0; it < NE; it++) {
        const int e = sl.t + it * G::TPB;
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int P[3] = {i >> 1, j >> 1, k >> 1};
        const int sg[3] = {(i & 1) ? 1 : -1, (j & 1) ? 1 : -1, (k & 1) ? 1 : -1};
        const T d0 = q[qpad<D, N>(P[0], P[1], P[2])], e0 = qe[qpad<D, N>(P[0], P[1], P[2])];
        T v;
        if (eps) {
            v = d0;
#pragma unroll
            for (int d = 0; d < D; d++) {
                int Q[3] = {P[0], P[1], P[2]};
                Q[d] += sg[d];
                const int qi = qpad<D, N>(Q[0], Q[1], Q[2]);
                const T ed = qe[qi];
                v += ed / (T(2) * (e0 + ed)) * (q[qi] - d0);
            }
        } else if (D == 2) {
            v = T(0.5) * d0 + T(0.25) * q[qpad<D, N>(P[0] + sg[0], P[1], 0)] +
                T(0.25) * q[qpad<D, N>(P[0], P[1] + sg[1], 0)];
        } else {
            v = T(0.25) * (((d0 + q[qpad<D, N>(P[0] + sg[0], P[1], P[2])]) + q[qpad<D, N>(P[0], P[1] + sg[1], P[2])]) +
                           q[qpad<D, N>(P[0], P[1], P[2] + sg[2])]);
        }
        a.u[bo + e] = uf[it] + v;
    }
}


// Coarse-grid correction with bi/trilinear prolongation (paper §2.5).  The
// whole parent box of delta = u - uold is staged with its side ghosts (the
// solve's schemes applied to deltas: the boundary values cancel), then its
// edge (3D) and corner ghosts (paper §2.4): the delta of the same-level box
// across that edge or corner, or else the linear extrapolation b + c - a
// (a 3D corner: its three edge ghosts minus its three side ghosts plus the
// inner cell).  A fine cell takes weights 3/4 and 1/4 per axis over the 2^D
// coarse cells nearest to it.
template <int D, int N, typename T>
__global__ __launch_bounds__((opw<D, N>())) void k_vprolong_lin(LevelArgs<T> a) {
    using G = Geo<D, N>;
    constexpr int NE = G::C / G::TPB;
    __shared__ T sm[opw<D, N>() / G::TPB * G::PC];
    const Slot<D, N> sl = slot_of<D, N, opw<D, N>()>(a.b0, a.nb, a.no_remap == 0);
    T *s = sm + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const bool act = sl.valid;
    const int t = sl.t;
    const size_t bo = (size_t)sl.b * G::C;
    const int64_t p = bi.parent;
    const BoxInfo pi = load_box<D, N>(a.info, p);
    const size_t po = (size_t)p * G::C;
    T uf[NE];
#pragma unroll
    for (int it = 0; it < NE; it++) uf[it] = a.u[bo + t + it * G::TPB];
    // the parent's rows of delta and the raw operands of its side ghosts
    Stager<D, N, T, true> st;
    st.bil = (a.opk & OPK_GHOST_BIL) ? 1 : 0;
    st.hg = 1;
    st.fl = pi.flags;
    st.hh = T(0);
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int m = 0; m < G::HN; m++) {
            const size_t e = po + c * G::HALF + t * G::HN + m;
            st.rowv[c][m] = a.u[e] - a.uold[e];
        }
#define AFMG_G1(S)                                                                           \
    {                                                                                        \
        const size_t off = (size_t)(ghost_ptr<D, N, S, T>(pi, t, a.u, nullptr, 1, st.v[S]) - a.u); \
        st.raw[S] = a.u[off] - a.uold[off];                                                  \
    }
    AFMG_G1(0) AFMG_G1(1) AFMG_G1(2) AFMG_G1(3)
    if (D == 3) {
        AFMG_G1(4) AFMG_G1(5)
    }
#undef AFMG_G1
    st.stage(s, t);
    __syncthreads();
    if (act) st.end(s, t);
    __syncthreads();
    // edges (2 axes outside the box), then corners (3 axes)
    for (int nout = 2; nout <= D; nout++) {
        const int count = nout == 2 ? (D == 3 ? 12 * N : 4) : 8;
        for (int w = t; act && w < count; w += G::TPB) {
            // the w-th direction with nout nonzero components, in the order
            // of the index (dx+1) + 3 (dy+1) + 9 (dz+1)
            const int dir_rank = nout == 2 && D == 3 ? w / N : w;
            const int along = nout == 2 && D == 3 ? w % N : 0;
            int o[3] = {0, 0, 0}, rank = 0, found = 0;
            for (int idx = 0; idx < 27 && !found; idx++) {
                const int dd[3] = {idx % 3 - 1, (idx / 3) % 3 - 1, idx / 9 - 1};
                if (D == 2 && dd[2] != 0) continue;
                if ((dd[0] != 0) + (dd[1] != 0) + (dd[2] != 0) != nout) continue;
                if (rank++ == dir_rank) {
                    o[0] = dd[0];
                    o[1] = dd[1];
                    o[2] = dd[2];
                    found = 1;
                }
            }
            int g[3];
            for (int d = 0; d < 3; d++) g[d] = o[d] == -1 ? -1 : o[d] == 1 ? N : along;
            const int didx = (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1);
            const int32_t v = a.dnbr[(size_t)p * 27 + didx];
            T val;
            if (v >= 0) {
                int q[3];
                for (int d = 0; d < 3; d++) q[d] = o[d] == -1 ? N - 1 : o[d] == 1 ? 0 : along;
                const size_t e = (size_t)v * G::C + cpos<D, N>(q[0], q[1], D == 3 ? q[2] : 0);
                val = a.u[e] - a.uold[e];
            } else {
                // inclusion-exclusion over the outside axes
                int ax[3], na = 0;
                for (int d = 0; d < D; d++)
                    if (o[d] != 0) ax[na++] = d;
                val = T(0);
                for (int sub = 1; sub < (1 << na); sub++) {
                    int q[3] = {g[0], g[1], D == 3 ? g[2] : 0}, cnt = 0;
                    for (int k = 0; k < na; k++)
                        if (sub & (1 << k)) {
                            q[ax[k]] += o[ax[k]] == -1 ? 1 : -1;
                            cnt++;
                        }
                    const T f = s[padi<D, N>(q[0], q[1], q[2])];
                    val += (cnt & 1) ? f : -f;
                }
            }
            s[padi<D, N>(g[0], g[1], D == 3 ? g[2] : 0)] = val;
        }
        __syncthreads();
    }
    if (!act) return;
    const int flags = bi.flags;
    const int o0 = obit(flags, 0) * G::H, o1 = obit(flags, 1) * G::H, o2 = D == 3 ? obit(flags, 2) * G::H : 0;
#pragma unroll
    for (int it = 0; it < NE; it++) {
        const int e = t + it * G::TPB;
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int X = o0 + (i >> 1), Y = o1 + (j >> 1), Z = o2 + (k >> 1);
        const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        T v;
        if (D == 2) {
            v = T(0.5625) * s[padi<D, N>(X, Y, 0)] + T(0.1875) * s[padi<D, N>(X + sx, Y, 0)] +
                T(0.1875) * s[padi<D, N>(X, Y + sy, 0)] + T(0.0625) * s[padi<D, N>(X + sx, Y + sy, 0)];
        } else {
            v = T(0.421875) * s[padi<D, N>(X, Y, Z)] +
                T(0.140625) * ((s[padi<D, N>(X + sx, Y, Z)] + s[padi<D, N>(X, Y + sy, Z)]) + s[padi<D, N>(X, Y, Z + sz)]) +
                T(0.046875) * ((s[padi<D, N>(X + sx, Y + sy, Z)] + s[padi<D, N>(X + sx, Y, Z + sz)]) +
                               s[padi<D, N>(X, Y + sy, Z + sz)]) +
                T(0.015625) * s[padi<D, N>(X + sx, Y + sy, Z + sz)];
        }
        a.u[bo + e] = uf[it] + v;
    }
}

// FMG / end of a solve: the parent's octant of field f receives the mean of
// the box's values, a volume mean in the cylindrical form
template <int D, int N, typename T>
__device__ __forceinline__ void restrict_octant_op(const T *s, T *__restrict__ dst, const BoxInfo &bi, int t,
                                                   bool cyl, T x0, T h) {
    using G = Geo<D, N>;
    const T w = D == 3 ? T(0.125) : T(0.25);
    const int flags = bi.flags;
    const int64_t p = bi.parent;
    for (int pc = t; pc < G::HC; pc += G::TPB) {
        const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
        T acc = T(0), vol = T(0);
#pragma unroll
        for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
#pragma unroll
            for (int dj = 0; dj < 2; dj++)
#pragma unroll
                for (int di = 0; di < 2; di++) {
                    const int i = 2 * I + di, j = 2 * J + dj, k = D == 3 ? 2 * K + dk : 0;
                    const T f = s[D == 3 ? i + N * (j + N * k) : i + N * j];
                    const T wq = vol_w<T>(cyl, x0, h, i);
                    acc += cyl ? wq * f : f;
                    vol += wq;
                }
        const int X = obit(flags, 0) * G::H + I, Y = obit(flags, 1) * G::H + J,
                  Z = D == 3 ? obit(flags, 2) * G::H + K : 0;
        dst[(size_t)p * G::C + cpos<D, N>(X, Y, Z)] = cyl ? acc / vol : w * acc;
    }
}

template <int D, int N, typename T>
__global__ __launch_bounds__(256) void k_vrestrict(const BoxInfo *__restrict__ info, T *f, int64_t b0, int nb,
                                                   int opk, const int32_t *__restrict__ bx, T h) {
    using G = Geo<D, N>;
    __shared__ T sm[G::BPW * G::C];
    const Slot<D, N> sl = slot_of<D, N>(b0, nb);
    T *s = sm + sl.slot * G::C;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    if (sl.valid) {
        for (int e = sl.t; e < G::C; e += G::TPB) {
            int i, j, k;
            cell_of<D, N>(e, i, j, k);
            s[D == 3 ? i + N * (j + N * k) : i + N * j] = f[bo + e];
        }
    }
    __syncthreads();
    const bool cyl = opk & OPK_CYL;
    if (sl.valid) restrict_octant_op<D, N, T>(s, f, bi, sl.t, cyl, cyl ? box_x0<N, T>(bx, sl.b, h) : T(0), h);
}

// *flag |= 1 for a leaf cell that is not positive and finite
template <int D, int N>
__global__ __launch_bounds__(256) void k_check_positive(const BoxInfo *__restrict__ info,
                                                        const double *__restrict__ f, int nb, int *flag) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb, false);
    if (!sl.valid) return;
    if (!(info[sl.b].flags & FLAG_LEAF)) return;
    int bad = 0;
    for (int e = sl.t; e < G::C; e += G::TPB) {
        const double x = f[(size_t)sl.b * G::C + e];
        bad |= !(x > 0.0 && x <= 1.7976931348623157e308);
    }
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// mesh adaptation (paper §2.3) and field transfer
// ---------------------------------------------------------------------------
// One word per box from the cell flags of a leaf box (int8, the caller's
// x-fastest order; > 0 refine, < 0 derefine): ADAPT_REFINE if some cell is
// flagged for refinement, ADAPT_REMOVE if every cell is flagged for
// derefinement, and the bit of each neighbour direction (dx, dy, dz) such
// that a refine-flagged cell lies within n_buf cells of that neighbour
// (along every axis where the direction is not 0, the cell is among the
// n_buf cells next to that side).  Parents get 0.  Thread t of a box scans
// row t; the words of a box's threads are combined across their lanes.
template <int D, int N>
__global__ __launch_bounds__(256) void k_box_flags(const BoxInfo *__restrict__ info, const int8_t *__restrict__ flags,
                                                   int nb, int n_buf, int32_t *__restrict__ words) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb, false);
    const bool leaf = sl.valid && (info[sl.b].flags & FLAG_LEAF);
    int w = 0, all_rm = 1;
    if (leaf) {
        int j, k;
        row_of<D, N>(sl.t, j, k);
        const int8_t *f = flags + (size_t)sl.b * G::C + (size_t)sl.t * N;
        for (int i = 0; i < N; i++) {
            const int v = f[i];
            all_rm &= v < 0 ? 1 : 0;
            if (v <= 0) continue;
            w |= ADAPT_REFINE;
            const bool lo[3] = {i < n_buf, j < n_buf, k < n_buf};
            const bool hi[3] = {i >= N - n_buf, j >= N - n_buf, k >= N - n_buf};
            for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        if (dx == 0 && dy == 0 && dz == 0) continue;
                        const int o[3] = {dx, dy, dz};
                        bool near = true;
                        for (int d = 0; d < D; d++)
                            if ((o[d] == -1 && !lo[d]) || (o[d] == 1 && !hi[d])) near = false;
                        if (near) w |= adapt_dir_bit(dx, dy, dz);
                    }
        }
    }
    constexpr int LW = G::TPB < 64 ? G::TPB : 64;
    for (int o = LW / 2; o > 0; o >>= 1) {
        w |= __shfl_xor(w, o);
        all_rm &= __shfl_xor(all_rm, o);
    }
    if constexpr (G::TPB > 64) {
        // a box of several waves: its waves through LDS
        __shared__ int red_w[4], red_a[4];
        const int wave = (int)threadIdx.x / 64;
        if ((threadIdx.x & 63) == 0) {
            red_w[wave] = w;
            red_a[wave] = all_rm;
        }
        __syncthreads();
        if (sl.t == 0)
            for (int q = 1; q < G::TPB / 64; q++) {
                w |= red_w[wave + q];
                all_rm &= red_a[wave + q];
            }
    }
    if (sl.valid && sl.t == 0) words[sl.b] = leaf ? (w | (all_rm ? ADAPT_REMOVE : 0)) : 0;
}

// whole boxes: to[dst[q]] = from[src[q]] (both colour-split)
template <int D, int N>
__global__ __launch_bounds__(256) void k_transfer_copy(const int32_t *__restrict__ dst, const int32_t *__restrict__ src,
                                                       int n, const double *__restrict__ from, double *__restrict__ to) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, n, false);
    if (!sl.valid) return;
    const size_t a = (size_t)src[sl.b] * G::C, b = (size_t)dst[sl.b] * G::C;
    for (int e = sl.t; e < G::C; e += G::TPB) to[b + e] = from[a + e];
}

// New boxes: to-box dst[q] receives the default prolongation (paper §2.5) of
// the from-tree's leaf src[q], its parent: the octant under the box plus a
// one-cell halo is staged, halo cells outside the parent box are the side
// ghosts of the solve (neighbour cells; 2 b - u1 or u1 + h q on physical
// sides with the boundary rows bc, zero values when homog; the default
// refinement-boundary scheme), and
//   2D: 1/2 u(P) + 1/4 u(P + sx ex) + 1/4 u(P + sy ey)
//   3D: 1/4 [u(P) + u(P + sx ex) + u(P + sy ey) + u(P + sz ez)].
template <int D, int N>
__global__ __launch_bounds__(256) void k_transfer_prolong(const BoxInfo *__restrict__ to_info,
                                                          const BoxInfo *__restrict__ from_info,
                                                          const int32_t *__restrict__ dst, const int32_t *__restrict__ src,
                                                          int n, const double *__restrict__ from,
                                                          const double *__restrict__ bc, int homog,
                                                          double *__restrict__ to) {
    using G = Geo<D, N>;
    constexpr int NH = (2 * D * G::HF + G::TPB - 1) / G::TPB;
    constexpr int NO = G::HC / G::TPB;
    constexpr int NE = G::C / G::TPB;
    __shared__ double qs[G::BPW * G::QC];
    const Slot<D, N> sl = slot_of<D, N>(0, n, false);
    double *q = qs + sl.slot * G::QC;
    const bool act = sl.valid;
    const int64_t b = act ? dst[sl.b] : 0, p = act ? src[sl.b] : 0;
    const BoxInfo bi = to_info[b];
    const BoxInfo pi = from_info[p];
    const int o[3] = {obit(bi.flags, 0) * G::H, obit(bi.flags, 1) * G::H, D == 3 ? obit(bi.flags, 2) * G::H : 0};
    const double hp = 1.0 / ((double)N * ldexp(1.0, pi.level - 1));
    double raw[NH];
    int hv[NH], hs[NH];
    if (act) {
        double od[NO];
#pragma unroll
        for (int it = 0; it < NO; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            od[it] = from[(size_t)p * G::C + cpos<D, N>(o[0] + I, o[1] + J, o[2] + K)];
        }
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int hc = sl.t + h * G::TPB;
            size_t ho = (size_t)p * G::C;
            hv[h] = 0;
            hs[h] = 0;
            if (hc < 2 * D * G::HF) {
                const int side = hc / G::HF, m = hc % G::HF;
#define AFMG_H1(S) ho = halo_addr<D, N, S>(m, o, pi, p, hv[h], hs[h])
                AFMG_SIDE_SWITCH(side, AFMG_H1)
#undef AFMG_H1
            }
            raw[h] = from[ho];
        }
#pragma unroll
        for (int it = 0; it < NO; it++) {
            const int pc = sl.t + it * G::TPB;
            const int I = pc % G::H, J = (pc / G::H) % G::H, K = D == 3 ? pc / (G::H * G::H) : 0;
            q[qpad<D, N>(I, J, K)] = od[it];
        }
#pragma unroll
        for (int h = 0; h < NH; h++)
            if (sl.t + h * G::TPB < 2 * D * G::HF && hv[h] >= 0) q[hs[h]] = raw[h];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int hc = sl.t + h * G::TPB;
            if (hc >= 2 * D * G::HF || hv[h] >= 0) continue;
            const int side = hc / G::HF, m = hc % G::HF;
            if (hv[h] <= -2) {
#define AFMG_H2(S) halo_phase2<D, N, S, double>(q, m, o, raw[h], hv[h], pi.flags)
                AFMG_SIDE_SWITCH(side, AFMG_H2)
#undef AFMG_H2
                continue;
            }
            // physical side of the parent: the ghost of the values
#define AFMG_H3(S)                                                                                    \
    {                                                                                                 \
        using SD = SideOf<S>;                                                                         \
        int L[3], X[3];                                                                               \
        halo_cell<D, N, S>(m, o, L, X);                                                               \
        int f[3] = {L[0], L[1], L[2]};                                                                \
        f[SD::d] = SD::hi ? L[SD::d] - 1 : 0;                                                         \
        const double d1 = q[qpad<D, N>(f[0], f[1], f[2])];                                            \
        const int mf = X[SD::t1] + (D == 3 ? N * X[SD::t2] : 0);                                      \
        const double bv = (homog || pi.bcoff[S] < 0) ? 0.0 : bc[(size_t)pi.bcoff[S] * G::F + mf];     \
        q[qpad<D, N>(L[0], L[1], L[2])] = phys_ghost<double>(neumann_side(pi.flags, S), bv, d1, hp);  \
    }
            AFMG_SIDE_SWITCH(side, AFMG_H3)
#undef AFMG_H3
        }
    }
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int it = 0; it < NE; it++) {
        const int e = sl.t + it * G::TPB;
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        double v;
        if (D == 2) {
            v = 0.5 * q[qpad<D, N>(I, J, 0)] + 0.25 * q[qpad<D, N>(I + sx, J, 0)] + 0.25 * q[qpad<D, N>(I, J + sy, 0)];
        } else {
            v = 0.25 * (((q[qpad<D, N>(I, J, K)] + q[qpad<D, N>(I + sx, J, K)]) + q[qpad<D, N>(I, J + sy, K)]) +
                        q[qpad<D, N>(I, J, K + sz)]);
        }
        to[(size_t)b * G::C + e] = v;
    }
}

#ifndef AFMG_INSTANTIATE_ONLY
// One workgroup of 1024 threads: out[0] = max of the partial maxima, out[1] =
// sqrt of the sum of the partial sums; the reduction order is fixed.
__global__ __launch_bounds__(1024) void k_reduce(const double *__restrict__ partial, int64_t n, double *out,
                                                 int root) {
    __shared__ double rm[1024], rsum[1024];
    double mx[4] = {0.0, 0.0, 0.0, 0.0}, ss[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = threadIdx.x;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            mx[q] = fmax(mx[q], partial[2 * (i + q * 1024)]);
            ss[q] += partial[2 * (i + q * 1024) + 1];
        }
    }
    for (; i < n; i += 1024) {
        mx[0] = fmax(mx[0], partial[2 * i]);
        ss[0] += partial[2 * i + 1];
    }
    rm[threadIdx.x] = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
    rsum[threadIdx.x] = (ss[0] + ss[1]) + (ss[2] + ss[3]);
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
            rsum[threadIdx.x] += rsum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // fmax drops NaN operands; the sum keeps them
        const double s = rsum[0];
        out[0] = (s == s) ? rm[0] : s;
        out[1] = root ? sqrt(s) : s;
        __threadfence_system();  // out may be host memory the host reads after the launch
    }
}

// One workgroup per tree of a forest: (max, sqrt of sum) of the per-box
// partials of the tree's leaf boxes, in a fixed order; trees whose mask entry
// is 0 are skipped.
__global__ __launch_bounds__(256) void k_reduce_trees(const double *__restrict__ partial,
                                                      const int64_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ boxes,
                                                      const int *__restrict__ active, double *out) {
    __shared__ double rm[256], rsum[256];
    const int tr = blockIdx.x;
    if (active && !active[tr]) return;
    double mx = 0.0, ss = 0.0;
    for (int64_t i = ptr[tr] + threadIdx.x; i < ptr[tr + 1]; i += 256) {
        const int64_t b = boxes[i];
        mx = fmax(mx, partial[2 * b]);
        ss += partial[2 * b + 1];
    }
    rm[threadIdx.x] = mx;
    rsum[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
            rsum[threadIdx.x] += rsum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = rsum[0];
        out[2 * tr + 0] = (s == s) ? rm[0] : s;
        out[2 * tr + 1] = sqrt(s);
        __threadfence_system();  // out may be host memory the host reads after the launch
    }
}

// Mask of the trees that take part in an FMG step at level l: out[t] =
// base[t] (1 when base is null) and the tree reaches level l.
__global__ __launch_bounds__(256) void k_level_mask(const int *__restrict__ base, const int32_t *__restrict__ tree_lmax,
                                                    int l, int *__restrict__ out, int n) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) out[t] = ((base ? base[t] : 1) != 0 && tree_lmax[t] >= l) ? 1 : 0;
}

// Compacted box lists of a forest: workgroup l-1 lists, for level l, the
// boxes of the trees whose mask entry is set, in box order, at act[lvl_off[l]
// ..] and their count at nact[l].  The boxes of one tree on one level are
// contiguous (box order: level, tree, Morton), ltoff[l][t] .. ltoff[l][t+1].
__global__ __launch_bounds__(256) void k_compact(const int *__restrict__ mask, const int64_t *__restrict__ ltoff,
                                                 const int64_t *__restrict__ lvl_off, int n_trees,
                                                 int32_t *__restrict__ act, int *__restrict__ nact) {
    const int l = (int)blockIdx.x + 1;
    const int64_t *to = ltoff + (size_t)l * (n_trees + 1);
    const int64_t base = lvl_off[l];
    int64_t pos = 0;  // every thread walks the trees in the same order
    for (int t = 0; t < n_trees; t++) {
        if (!mask[t]) continue;
        const int64_t b0 = to[t], cnt = to[t + 1] - b0;
        for (int64_t k = threadIdx.x; k < cnt; k += 256) act[base + pos + k] = (int32_t)(b0 + k);
        pos += cnt;
    }
    if (threadIdx.x == 0) nact[l] = (int)pos;
}

// The stop rule of every tree of a forest whose mask entry is set, after one
// cycle: the history entry, the cycle count, a non-finite norm, three
// growths in a row, convergence (max |r| <= tol max |r0|) or the last allowed
// cycle; a tree that stops leaves the mask, so later cycles skip it.
__global__ __launch_bounds__(256) void k_tree_stop(const double *__restrict__ norm, int *__restrict__ mask,
                                                   TreeStop *__restrict__ state, double *__restrict__ hist,
                                                   int n, double tol, int fixed, int nmax) {
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= n || !mask[t]) return;
    TreeStop s = state[t];
    const double rmax = norm[2 * t], rl2 = norm[2 * t + 1];
    s.rmax = rmax;
    s.rl2 = rl2;
    if (s.cycles < AFMG_HIST) {
        hist[((size_t)t * 2 + 0) * AFMG_HIST + s.cycles] = rmax;
        hist[((size_t)t * 2 + 1) * AFMG_HIST + s.cycles] = rl2;
    }
    s.cycles++;
    bool done = false;
    if (!isfinite(rmax)) {
        s.status = AFMG_ERR_NONFINITE;
        done = true;
    } else if (!fixed) {
        s.grow = rmax > s.prev ? s.grow + 1 : 0;
        if (s.grow >= 3) {
            s.status = AFMG_ERR_DIVERGED;
            done = true;
        } else if (rmax <= tol * s.r0) {
            s.conv = 1;
            done = true;
        }
    }
    if (!done) {
        s.prev = rmax;
        if (s.cycles >= nmax) done = true;
    }
    state[t] = s;
    if (done) mask[t] = 0;
}
#endif  // AFMG_INSTANTIATE_ONLY

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// FMG: the parent's octant of rho receives the mean of the box's rho.
template <int D, int N, typename T, bool F>
__global__ __launch_bounds__(256) void k_restrict_rho(LevelArgs<T> a) {
    using G = Geo<D, N>;
    __shared__ T sm[G::BPW * G::C];
    const Slot<D, N> sl = slot_lvl<D, N, 256, F>(a);
    T *s = sm + sl.slot * G::C;
    const BoxInfo bi = load_box<D, N>(a.info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    if (sl.valid) {
        for (int e = sl.t; e < G::C; e += G::TPB) {
            int i, j, k;
            cell_of<D, N>(e, i, j, k);
            s[D == 3 ? i + N * (j + N * k) : i + N * j] = a.rho[bo + e];
        }
    }
    __syncthreads();
    if (sl.valid) restrict_octant<D, N, T, false>(s, a.rho, bi, sl.t);
}

// In-place conversion of whole boxes between the caller's order (x fastest)
// and the colour-split storage.  to_split = 1: natural -> split.  Only boxes
// whose leaf flag matches `which` (0 all, 1 leaves) are converted.
template <int D, int N, typename T>
__global__ __launch_bounds__(256) void k_permute(const BoxInfo *__restrict__ info, T *f, int64_t b0, int nb,
                                                 int to_split, int which) {
    using G = Geo<D, N>;
    __shared__ T sm[G::BPW * G::C];
    const Slot<D, N> sl = slot_of<D, N>(b0, nb);
    T *s = sm + sl.slot * G::C;
    const bool go = sl.valid && (which == 0 || (info[sl.b].flags & FLAG_LEAF));
    T *fb = f + (size_t)sl.b * G::C;
    if (go)
        for (int e = sl.t; e < G::C; e += G::TPB) s[e] = fb[e];
    __syncthreads();
    if (!go) return;
    for (int e = sl.t; e < G::C; e += G::TPB) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int n = D == 3 ? i + N * (j + N * k) : i + N * j;
        if (to_split) fb[e] = s[n];
        else fb[n] = s[e];
    }
}

// Mixed-precision refinement: u += e on the leaf boxes (e in FP32), and e
// of those boxes back to zero, the initial guess of the next correction
// solve (its V-cycle writes every parent box's e by restriction before it
// reads it, so only leaves need the zero).
template <int D, int N>
__global__ __launch_bounds__(256) void k_ir_update(const BoxInfo *__restrict__ info, double *__restrict__ u,
                                                   float *__restrict__ e, int nb, const int *active) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    if (!sl.valid) return;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    if (!(bi.flags & FLAG_LEAF) || (active && !active[bi.tree])) return;
    const size_t bo = (size_t)sl.b * G::C;
    for (int c = sl.t; c < G::C; c += G::TPB) {
        const float ec = e[bo + c];
        u[bo + c] = u[bo + c] + (double)ec;
        e[bo + c] = 0.f;
    }
}

// Copy of the caller's boxes (natural order) into the colour-split working
// layout: box b receives the caller's box map[b] (b itself when map is null);
// leaves_only skips parent boxes.
template <int D, int N, typename T>
__global__ __launch_bounds__(256) void k_load_rho(const BoxInfo *__restrict__ info, const int32_t *__restrict__ map,
                                                  const T *__restrict__ src, T *__restrict__ dst, int nb,
                                                  int leaves_only) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    if (!sl.valid || (leaves_only && !(info[sl.b].flags & FLAG_LEAF))) return;
    const size_t bo = (size_t)sl.b * G::C;
    const size_t so = (size_t)(map ? map[sl.b] : sl.b) * G::C;
    for (int e = sl.t; e < G::C; e += G::TPB) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        dst[bo + e] = src[so + (D == 3 ? i + N * (j + N * k) : i + N * j)];
    }
}

// Inverse of k_load_rho for whole boxes: the caller's box map[b] (natural
// order) receives working box b (colour-split).
template <int D, int N, typename T>
__global__ __launch_bounds__(256) void k_store_boxes(const int32_t *__restrict__ map, const T *__restrict__ src,
                                                     T *__restrict__ dst, int nb) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    if (!sl.valid) return;
    const size_t bo = (size_t)sl.b * G::C;
    const size_t dof = (size_t)map[sl.b] * G::C;
    for (int e = sl.t; e < G::C; e += G::TPB) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        dst[dof + (D == 3 ? i + N * (j + N * k) : i + N * j)] = src[bo + e];
    }
}

#ifndef AFMG_INSTANTIATE_ONLY
// Rows of F values: dst row r receives src row map[r].
__global__ __launch_bounds__(256) void k_gather_rows(const int32_t *__restrict__ map, const double *__restrict__ src,
                                                     double *__restrict__ dst, int64_t n_rows, int F) {
    const int64_t n = n_rows * F;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[(int64_t)map[i / F] * F + i % F];
}
#endif  // AFMG_INSTANTIATE_ONLY

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T *__restrict__ src, T *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *__restrict__ dst, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = v;
}

// Boxes of level l (children): each physical side writes the covered part of
// its parent's Dirichlet row as means of 2^(D-1) child face values (the rows
// are in face order, tangential axes increasing, first fastest).
template <int D, int N>
__global__ __launch_bounds__(256) void k_bc_derive(const BoxInfo *__restrict__ info, int64_t b0, int nb,
                                                   double *bc) {
    using G = Geo<D, N>;
    const int64_t bl = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t work = (int64_t)nb * 2 * D * G::HF;
    if (bl >= work) return;
    const int64_t b = b0 + bl / (2 * D * G::HF);
    const int rem = (int)(bl % (2 * D * G::HF));
    const int side = rem / G::HF, m = rem % G::HF;
    const BoxInfo *bi = info + b;
    if (bi->nbr[side] != -1 || bi->parent < 0) return;
    const BoxInfo *pi = info + bi->parent;
    const int d = side >> 1;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int A = m % G::H, Cc = D == 3 ? m / G::H : 0;
    const double *cr = bc + (size_t)bi->bcoff[side] * G::F;
    double acc = 0.0;
    for (int dc = 0; dc < (D == 3 ? 2 : 1); dc++)
        for (int da = 0; da < 2; da++) acc += cr[(2 * A + da) + N * (2 * Cc + dc)];
    const int pa = obit(bi->flags, t1) * G::H + A;
    const int pc = D == 3 ? obit(bi->flags, t2) * G::H + Cc : 0;
    bc[(size_t)pi->bcoff[side] * G::F + pa + N * pc] = acc * (D == 3 ? 0.25 : 0.5);
}

// ---------------------------------------------------------------------------
// levels <= 2 of a tree in one workgroup: level 2 (below), the root box and
// the coarse grids below it
// ---------------------------------------------------------------------------
// The grids of N, N/2, ..., 2 cells per side (levels 1, 0, ..., lmin) are
// single boxes whose sides are all physical (Dirichlet).  They live in LDS
// without ghost layers, in FP64 for every precision of the caller's arrays.
// The grid index G (0: N cells per side) is a template parameter, so every
// index is a compile-time shift; the side ghosts 2 b - u1 (paper §2.4) are
// formed inline, with the same arithmetic a stored ghost layer would hold.
constexpr int COARSE_NT = 512;  // threads of the coarse kernel

template <int D, int N>
struct CoarseGeo {
    static constexpr int lg(int n) { return n <= 1 ? 0 : 1 + lg(n / 2); }
    static constexpr int NG = lg(N);  // grids of N, N/2, ..., 2 cells
    static constexpr int n(int g) { return N >> g; }
    static constexpr int cells(int g) { return D == 3 ? n(g) * n(g) * n(g) : n(g) * n(g); }
    static constexpr int off(int g) { return g == 0 ? 0 : off(g - 1) + cells(g - 1); }
    static constexpr int TOT = off(NG);
    static constexpr int fsz(int g) { return D == 3 ? n(g) * n(g) : n(g); }
    static constexpr int boff(int g) { return g == 0 ? 0 : boff(g - 1) + 2 * D * fsz(g - 1); }
    static constexpr int BTOT = boff(NG);
};

template <int D, int N>
struct CoarseState {
    using CG = CoarseGeo<D, N>;
    // rho of a coarser grid receives the restricted residual, and then (in
    // place) the FAS right-hand side: rbar + L u
    double *u, *rho, *uold, *bc;
    int n_down, n_up, n_base;

    template <int G>
    __device__ __forceinline__ static void ijk(int c, int &i, int &j, int &k) {
        constexpr int n = CG::n(G);
        i = c % n;
        j = (c / n) % n;
        k = D == 3 ? c / (n * n) : 0;
    }
    // Dirichlet value of side `side` next to cell (i, j, k) of grid G (the
    // tangential axes in increasing order, the first fastest)
    template <int G>
    __device__ __forceinline__ double bval(int side, int i, int j, int k) const {
        constexpr int n = CG::n(G), F = CG::fsz(G);
        const int d = side >> 1;
        const int m = d == 0 ? j + n * k : d == 1 ? i + n * k : i + n * j;
        return bc[CG::boff(G) + side * F + m];
    }
    // sum of the 2D neighbours of cell (i, j, k) of f on grid G.  Every
    // operand is fetched (a neighbour outside the grid at the cell's own
    // index, the boundary value of each side) before one is selected, so
    // that the LDS reads leave together instead of one branch at a time.
    template <int G>
    __device__ __forceinline__ double nbs(const double *f, int i, int j, int k) const {
        constexpr int n = CG::n(G);
        const double *g = f + CG::off(G);
        const int c = i + n * (j + n * k);
        const double uc = g[c];
        const double vxm = g[i > 0 ? c - 1 : c], vxp = g[i < n - 1 ? c + 1 : c];
        const double vym = g[j > 0 ? c - n : c], vyp = g[j < n - 1 ? c + n : c];
        const double bxm = bval<G>(0, i, j, k), bxp = bval<G>(1, i, j, k);
        const double bym = bval<G>(2, i, j, k), byp = bval<G>(3, i, j, k);
        const double xm = i > 0 ? vxm : 2.0 * bxm - uc;
        const double xp = i < n - 1 ? vxp : 2.0 * bxp - uc;
        const double ym = j > 0 ? vym : 2.0 * bym - uc;
        const double yp = j < n - 1 ? vyp : 2.0 * byp - uc;
        double s = (xm + xp) + (ym + yp);
        if (D == 3) {
            const double vzm = g[k > 0 ? c - n * n : c], vzp = g[k < n - 1 ? c + n * n : c];
            const double bzm = bval<G>(4, i, j, k), bzp = bval<G>(5, i, j, k);
            const double zm = k > 0 ? vzm : 2.0 * bzm - uc;
            const double zp = k < n - 1 ? vzp : 2.0 * bzp - uc;
            s = s + (zm + zp);
        }
        return s;
    }
    template <int G>
    __device__ static constexpr double hgrid() { return (double)(1 << G) / (double)N; }

    // Grid 0 (the root box) runs on the whole workgroup, the grids below it
    // (at most N^D / 2^D cells) on its first wave alone, where a phase ends
    // with a wave-scope fence instead of a workgroup barrier.  Every thread
    // computes all of its values before it stores the first.
    template <int G>
    static constexpr int nth() { return G == 0 ? COARSE_NT : 64; }
    template <int G>
    __device__ __forceinline__ static void sync() {
        if (G == 0) {
            __syncthreads();
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    template <int G, int X>
    static constexpr int rounds() { return (X + nth<G>() - 1) / nth<G>(); }

    // one colour of grid G
    template <int G>
    __device__ __forceinline__ void half(int colour) const {
        constexpr int n = CG::n(G), hn = n / 2, o = CG::off(G), NQ = CG::cells(G) / 2, IT = rounds<G, NQ>();
        constexpr double h = hgrid<G>(), h2 = h * h;
        double v[IT];
        int cc[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int q = (int)threadIdx.x + it * nth<G>();
            cc[it] = -1;
            if (q < NQ) {
                const int r = q / hn, j = r % n, k = D == 3 ? r / n : 0;
                const int i = 2 * (q % hn) + ((colour + j + k + D) & 1);
                cc[it] = i + n * (j + n * k);
                v[it] = (nbs<G>(u, i, j, k) - h2 * rho[o + cc[it]]) / double(2 * D);
            }
        }
#pragma unroll
        for (int it = 0; it < IT; it++)
            if (cc[it] >= 0) u[o + cc[it]] = v[it];
        sync<G>();
    }
    template <int G>
    __device__ __forceinline__ void gsrb(int nsweep) const {
        for (int q = 0; q < nsweep; q++) {
            half<G>(0);
            half<G>(1);
        }
    }
    // grid G+1 <- means of u and of the residual rho - L u of grid G
    template <int G>
    __device__ __forceinline__ void resid_restrict() const {
        constexpr int n = CG::n(G), nc = CG::n(G + 1), o = CG::off(G), oc = CG::off(G + 1);
        constexpr int NC = CG::cells(G + 1), IT = rounds<G, NC>();
        constexpr double h = hgrid<G>(), ih2 = 1.0 / (h * h);
        const double w = D == 3 ? 0.125 : 0.25;
        double mu[IT], mr[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int C = (int)threadIdx.x + it * nth<G>();
            if (C >= NC) continue;
            const int I = C % nc, J = (C / nc) % nc, K = D == 3 ? C / (nc * nc) : 0;
            double au = 0.0, ar = 0.0;
            for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
                for (int dj = 0; dj < 2; dj++)
                    for (int di = 0; di < 2; di++) {
                        const int i = 2 * I + di, j = 2 * J + dj, k = D == 3 ? 2 * K + dk : 0;
                        const int c = i + n * (j + n * k);
                        au += u[o + c];
                        ar += rho[o + c] - (nbs<G>(u, i, j, k) - double(2 * D) * u[o + c]) * ih2;
                    }
            mu[it] = w * au;
            mr[it] = w * ar;
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int C = (int)threadIdx.x + it * nth<G>();
            if (C >= NC) continue;
            u[oc + C] = mu[it];
            rho[oc + C] = mr[it];
        }
        sync<G>();
    }
    // rho of grid G (FMG) -> grid G+1
    template <int G>
    __device__ __forceinline__ void restrict_rho() const {
        constexpr int n = CG::n(G), nc = CG::n(G + 1), o = CG::off(G), oc = CG::off(G + 1);
        constexpr int NC = CG::cells(G + 1), IT = rounds<G, NC>();
        const double w = D == 3 ? 0.125 : 0.25;
        double m[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int C = (int)threadIdx.x + it * nth<G>();
            if (C >= NC) continue;
            const int I = C % nc, J = (C / nc) % nc, K = D == 3 ? C / (nc * nc) : 0;
            double acc = 0.0;
            for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
                for (int dj = 0; dj < 2; dj++)
                    for (int di = 0; di < 2; di++)
                        acc += rho[o + (2 * I + di) + n * ((2 * J + dj) + n * (D == 3 ? 2 * K + dk : 0))];
            m[it] = w * acc;
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int C = (int)threadIdx.x + it * nth<G>();
            if (C < NC) rho[oc + C] = m[it];
        }
        sync<G>();
    }
    // copy v' of grid G, and the FAS right-hand side rho <- rbar + L u (rho
    // holds the restricted residual rbar)
    template <int G>
    __device__ __forceinline__ void uold_crhs() const {
        constexpr int o = CG::off(G), NC = CG::cells(G), IT = rounds<G, NC>();
        constexpr double h = hgrid<G>(), ih2 = 1.0 / (h * h);
        double uc[IT], rc[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * nth<G>();
            if (c >= NC) continue;
            int i, j, k;
            ijk<G>(c, i, j, k);
            uc[it] = u[o + c];
            rc[it] = rho[o + c] + (nbs<G>(u, i, j, k) - double(2 * D) * u[o + c]) * ih2;
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * nth<G>();
            if (c >= NC) continue;
            uold[o + c] = uc[it];
            rho[o + c] = rc[it];
        }
        sync<G>();
    }
    // u - v' on grid G at (I, J, K) + s e_axis; outside the grid the ghost of
    // u minus the ghost of v' (the Dirichlet value cancels up to rounding)
    // (the operands are fetched before the selection, as in nbs)
    template <int G>
    __device__ __forceinline__ double delta(int axis, int I, int J, int K, int s) const {
        constexpr int n = CG::n(G), o = CG::off(G);
        int a[3] = {I, J, K};
        a[axis] += s;
        const bool in = a[axis] >= 0 && a[axis] < n;
        const int c = in ? a[0] + n * (a[1] + n * a[2]) : I + n * (J + n * K);
        const double uu = u[o + c], uo = uold[o + c];
        const double b = bval<G>(2 * axis + (s > 0 ? 1 : 0), I, J, K);
        return in ? uu - uo : (2.0 * b - uu) - (2.0 * b - uo);
    }
    // u of grid G += P211(u - v' of grid G+1); with store_old, v' of grid G
    // first receives u (FMG)
    template <int G>
    __device__ __forceinline__ void prolong(bool store_old) const {
        constexpr int o = CG::off(G), NC = CG::cells(G), IT = rounds<G, NC>();
        double uc[IT], nv[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * nth<G>();
            if (c >= NC) continue;
            int i, j, k;
            ijk<G>(c, i, j, k);
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
            double v;
            if (D == 2)
                v = 0.5 * delta<G + 1>(0, I, J, K, 0) + 0.25 * delta<G + 1>(0, I, J, K, sx) +
                    0.25 * delta<G + 1>(1, I, J, K, sy);
            else
                v = 0.25 * (((delta<G + 1>(0, I, J, K, 0) + delta<G + 1>(0, I, J, K, sx)) +
                             delta<G + 1>(1, I, J, K, sy)) +
                            delta<G + 1>(2, I, J, K, sz));
            uc[it] = u[o + c];
            nv[it] = uc[it] + v;
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * nth<G>();
            if (c >= NC) continue;
            if (store_old) uold[o + c] = uc[it];
            u[o + c] = nv[it];
        }
        sync<G>();
    }
    // FAS V-cycle from grid G (paper §3.2)
    template <int G>
    __device__ __forceinline__ void vcycle() const {
        if constexpr (G == CG::NG - 1) {
            gsrb<G>(n_base);
        } else {
            gsrb<G>(n_down);
            resid_restrict<G>();
            if (G > 0 || threadIdx.x < nth<G + 1>()) {
                uold_crhs<G + 1>();
                vcycle<G + 1>();
            }
            if (G == 0) __syncthreads();
            prolong<G>(false);
            gsrb<G>(n_up);
        }
    }
    // FMG from a zero guess on grids G .. NG-1, then the V-cycle from G:
    // rho restricted down, per grid store v', correct from the coarser grid
    template <int G>
    __device__ __forceinline__ void fmg() const {
        if constexpr (G < CG::NG - 1) {
            restrict_rho<G>();
            if (G > 0 || threadIdx.x < nth<G + 1>()) fmg<G + 1>();
            if (G == 0) __syncthreads();
            prolong<G>(true);
        } else {
            for (int c = threadIdx.x; c < CG::cells(G); c += nth<G>()) uold[CG::off(G) + c] = u[CG::off(G) + c];
            sync<G>();
        }
        vcycle<G>();
    }
};

// Level 2 of a tree inside the coarse kernel: the 2^D boxes under the root
// form one (2N)^D grid in LDS (natural order, x fastest, with a ghost layer
// that holds the Dirichlet ghosts of the current values) in the precision T
// of the level kernels.  Every step uses the formulas and summation orders of
// the box kernels (k_gsrb, k_resid_restrict, k_coarse_rhs, k_prolong): level 2
// is complete (all children of the root exist), so its ghosts are grid cells
// or Dirichlet ghosts 2 b - u1 (b = 0 when homogeneous), and the deltas of
// the root seen from level 2 have the ghost -delta(face cell) outside the
// domain (paper §2.4, §2.5, §3.1, §3.2).
template <int D, int N, typename T>
struct Level2 {
    static constexpr int M = 2 * N;                          // cells per axis
    static constexpr int CELLS = D == 3 ? M * M * M : M * M;
    static constexpr int F = D == 3 ? M * M : M;             // cells per side
    static constexpr int P = M + 2;                          // padded axis
    static constexpr int PCELLS = D == 3 ? P * P * P : P * P;
    T *u;          // grid values with a ghost layer (padded, natural order)
    T *rho;        // right-hand side (unpadded)
    const T *bc;   // [2D][F] Dirichlet values (zero when homogeneous)
    T h2, ih2;
    int parents;   // bit o: the box of octant o is a parent

    __device__ __forceinline__ static int at(int i, int j, int k) { return D == 3 ? i + M * (j + M * k) : i + M * j; }
    __device__ __forceinline__ static int pad(int i, int j, int k) {
        return D == 3 ? (i + 1) + P * ((j + 1) + P * (k + 1)) : (i + 1) + P * (j + 1);
    }
    __device__ __forceinline__ static int octant(int i, int j, int k) {
        return (i >= N ? 1 : 0) | (j >= N ? 2 : 0) | (D == 3 && k >= N ? 4 : 0);
    }
    // cell of grid position c
    __device__ __forceinline__ static void ijk(int c, int &i, int &j, int &k) {
        i = c % M;
        j = (c / M) % M;
        k = D == 3 ? c / (M * M) : 0;
    }
    // Dirichlet value of side s next to cell (i, j, k) (tangential axes
    // increasing, the first fastest)
    __device__ __forceinline__ T bval(int s, int i, int j, int k) const {
        const int d = s >> 1;
        const int m = d == 0 ? j + M * k : d == 1 ? i + M * k : i + M * j;
        return bc[s * F + m];
    }
    // cell (i, j, k) takes the value v; on the domain boundary its ghosts
    // 2 b - v follow (each ghost slot belongs to one cell, so the slots hold
    // the ghost of the cell's current value)
    __device__ __forceinline__ void set(int i, int j, int k, T v) const {
        u[pad(i, j, k)] = v;
        if (i == 0) u[pad(-1, j, k)] = T(2) * bval(0, i, j, k) - v;
        if (i == M - 1) u[pad(M, j, k)] = T(2) * bval(1, i, j, k) - v;
        if (j == 0) u[pad(i, -1, k)] = T(2) * bval(2, i, j, k) - v;
        if (j == M - 1) u[pad(i, M, k)] = T(2) * bval(3, i, j, k) - v;
        if (D == 3 && k == 0) u[pad(i, j, -1)] = T(2) * bval(4, i, j, k) - v;
        if (D == 3 && k == M - 1) u[pad(i, j, M)] = T(2) * bval(5, i, j, k) - v;
    }
    __device__ __forceinline__ T val(int i, int j, int k) const { return u[pad(i, j, k)]; }
    // every ghost slot from the current values (after staging)
    __device__ __forceinline__ void ghosts() const {
        for (int g = threadIdx.x; g < 2 * D * F; g += blockDim.x) {
            const int side = g / F, m = g % F, d = side >> 1, hi = side & 1;
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            int x[3];
            x[t1] = m % M;
            x[t2] = D == 3 ? m / M : 0;
            x[d] = hi ? M - 1 : 0;
            int y[3] = {x[0], x[1], x[2]};
            y[d] = hi ? M : -1;
            u[pad(y[0], y[1], y[2])] = T(2) * bc[g] - u[pad(x[0], x[1], x[2])];
        }
        __syncthreads();
    }
    // neighbour sum of the stencil, ghosts included
    __device__ __forceinline__ T nb_sum(int i, int j, int k) const {
        const int c = pad(i, j, k);
        T sum = (u[c - 1] + u[c + 1]) + (u[c - P] + u[c + P]);
        if (D == 3) sum = sum + (u[c - P * P] + u[c + P * P]);
        return sum;
    }
    // one red (0) or black (1) half sweep; every new value of the thread is
    // computed before the first is stored, so that the LDS reads of all its
    // cells are in flight together
    __device__ __forceinline__ void half(int colour) const {
        constexpr int hm = M / 2, NQ = CELLS / 2, IT = (NQ + COARSE_NT - 1) / COARSE_NT;
        T res[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int q = (int)threadIdx.x + it * COARSE_NT;
            if (q < NQ) {
                const int r = q / hm, j = r % M, k = D == 3 ? r / M : 0;
                const int i = 2 * (q % hm) + ((colour + j + k + D) & 1);
                res[it] = (nb_sum(i, j, k) - h2 * rho[at(i, j, k)]) / T(2 * D);
            }
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int q = (int)threadIdx.x + it * COARSE_NT;
            if (q < NQ) {
                const int r = q / hm, j = r % M, k = D == 3 ? r / M : 0;
                const int i = 2 * (q % hm) + ((colour + j + k + D) & 1);
                set(i, j, k, res[it]);
            }
        }
        __syncthreads();
    }
    __device__ __forceinline__ void gsrb(int n) const {
        for (int q = 0; q < n; q++) {
            half(0);
            half(1);
        }
    }
    // FAS right-hand side on the parent boxes: rho (= rbar) += L u
    __device__ __forceinline__ void crhs() const {
        constexpr int IT = (CELLS + COARSE_NT - 1) / COARSE_NT;
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * COARSE_NT;
            if (c < CELLS) {
                int i, j, k;
                ijk(c, i, j, k);
                if ((parents >> octant(i, j, k)) & 1) rho[c] = rho[c] + (nb_sum(i, j, k) - T(2 * D) * val(i, j, k)) * ih2;
            }
        }
        __syncthreads();
    }
    // level-1 cell P (natural order of the root box): means of u and of the
    // residual over its 2^D block
    __device__ __forceinline__ void resid_restrict(int P, T &mu, T &mr) const {
        constexpr int NB = D == 3 ? 8 : 4;
        const T w = D == 3 ? T(0.125) : T(0.25);
        const int I = P % N, J = (P / N) % N, K = D == 3 ? P / (N * N) : 0;
        T su = T(0), sr = T(0);
#pragma unroll
        for (int q = 0; q < NB; q++) {
            const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = D == 3 ? 2 * K + (q >> 2) : 0;
            const T uc = val(i, j, k);
            su += uc;
            sr += rho[at(i, j, k)] - (nb_sum(i, j, k) - T(2 * D) * uc) * ih2;
        }
        mu = w * su;
        mr = w * sr;
    }
    // u += P(delta) with delta = u - v' of the root (level 1, FP64 in LDS,
    // rounded to T as the box path stores it)
    __device__ __forceinline__ static T delta(const double *fu, const double *fo, int I, int J, int K) {
        const int c = I + N * (J + N * K);
        return (T)fu[c] - (T)fo[c];
    }
    __device__ __forceinline__ void prolong(const double *fu, const double *fo) const {
        constexpr int IT = (CELLS + COARSE_NT - 1) / COARSE_NT;
        T res[IT];
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * COARSE_NT;
            if (c >= CELLS) continue;
            int i, j, k;
            ijk(c, i, j, k);
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
            // neighbours outside the root at the cell's own index, fetched
            // before the selection (the reads leave together)
            const bool ix = I + sx >= 0 && I + sx < N, iy = J + sy >= 0 && J + sy < N;
            const T dP = delta(fu, fo, I, J, K);
            const T ex = delta(fu, fo, ix ? I + sx : I, J, K), ey = delta(fu, fo, I, iy ? J + sy : J, K);
            const T dx = ix ? ex : -dP;
            const T dy = iy ? ey : -dP;
            T v;
            if (D == 2) {
                v = T(0.5) * dP + T(0.25) * dx + T(0.25) * dy;
            } else {
                const bool iz = K + sz >= 0 && K + sz < N;
                const T ez = delta(fu, fo, I, J, iz ? K + sz : K);
                const T dz = iz ? ez : -dP;
                v = T(0.25) * (((dP + dx) + dy) + dz);
            }
            res[it] = val(i, j, k) + v;
        }
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int c = (int)threadIdx.x + it * COARSE_NT;
            if (c < CELLS) {
                int i, j, k;
                ijk(c, i, j, k);
                set(i, j, k, res[it]);
            }
        }
        __syncthreads();
    }
};

// LDS of k_coarse: the FP64 chain (u, rho, v', Dirichlet rows) and the
// padded level-2 grid with its rho and Dirichlet rows in T (FP64 counted)
template <int D, int N>
constexpr size_t coarse_lds_bytes(bool with_l2) {
    using CG = CoarseGeo<D, N>;
    using L2 = Level2<D, N, double>;
    return sizeof(double) * (3 * (size_t)CG::TOT + CG::BTOT) +
           (with_l2 ? sizeof(double) * ((size_t)L2::PCELLS + L2::CELLS + 2 * D * L2::F) : 0);
}
constexpr size_t LDS_PER_WORKGROUP = 160 * 1024;
template <int D, int N>
constexpr bool coarse_l2_fits() {
    return coarse_lds_bytes<D, N>(true) <= LDS_PER_WORKGROUP;
}
static_assert(coarse_lds_bytes<3, 16>(false) <= LDS_PER_WORKGROUP, "levels <= 1 of 16^3 boxes fit");

template <int D, int N, typename T>
__global__ __launch_bounds__(COARSE_NT) void k_coarse(CoarseArgs<T> a) {
    using CG = CoarseGeo<D, N>;
    using G = Geo<D, N>;
    using L2 = Level2<D, N, T>;
    // level 2 in LDS where it fits (boxes of 8^D cells, 16^2); otherwise
    // the scheduler runs level 2 box by box and asks for levels <= 1 only
    constexpr bool HAS_L2 = coarse_l2_fits<D, N>();
    __shared__ double f_u[CG::TOT], f_rho[CG::TOT], f_uold[CG::TOT], f_bc[CG::BTOT];
    __shared__ T l2_u[HAS_L2 ? L2::PCELLS : 1], l2_rho[HAS_L2 ? L2::CELLS : 1], l2_bc[HAS_L2 ? 2 * D * L2::F : 1];
    CoarseState<D, N> st{f_u, f_rho, f_uold, f_bc, a.n_down, a.n_up, a.n_base};
    // one workgroup per tree; the roots are boxes 0 .. n_trees-1
    const int64_t root = blockIdx.x;
    const BoxInfo *ri = a.info + root;
    if (a.active && !a.active[ri->tree]) return;
    // the mode that fits the tree: a tree that is its root box alone starts
    // at level 1; with level 2 but no level 3, a V-cycle starts at level 2
    int mode = a.mode;
    const bool root_leaf = ri->flags & FLAG_LEAF;
    int parents = 0;
    if (mode == COARSE_V2_FROM_3 || mode == COARSE_V2_TOP) {
        if (root_leaf) {
            mode = COARSE_V_TOP1;
        } else {
            for (int o = 0; o < (1 << D); o++)
                if (!(a.info[a.child[root * 8 + o]].flags & FLAG_LEAF)) parents |= 1 << o;
            if (mode == COARSE_V2_FROM_3 && parents == 0) mode = COARSE_V2_TOP;
        }
    } else if (mode == COARSE_V_FROM_2 && root_leaf) {
        mode = COARSE_V_TOP1;
    }
    const bool two = HAS_L2 && (mode == COARSE_V2_FROM_3 || mode == COARSE_V2_TOP);
    T *gu = a.u + root * G::C;
    T *grho = a.rho + root * G::C;
    T *guold = a.uold ? a.uold + root * G::C : nullptr;
    // the root box (colour-split in global memory) and its Dirichlet rows;
    // the coarser grids start at zero.  Compile-time strides keep all loads
    // of a thread in flight together.
    constexpr int NT = COARSE_NT;
    constexpr int NE = (G::C + NT - 1) / NT, NBC = (2 * D * G::F + NT - 1) / NT;
    double lu[NE], lr[NE], lb[NBC];
    if (!two) {
#pragma unroll
        for (int q = 0; q < NE; q++) {
            const int e = (int)threadIdx.x + q * NT;
            lu[q] = (e < G::C && mode != COARSE_FMG) ? (double)gu[e] : 0.0;
            lr[q] = e < G::C ? (double)grho[e] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < NBC; q++) {
        const int g = (int)threadIdx.x + q * NT;
        lb[q] = (g < 2 * D * G::F && !a.homog) ? a.bc[(size_t)ri->bcoff[g / G::F] * G::F + g % G::F] : 0.0;
    }
    const L2 lv2{l2_u, l2_rho, l2_bc, a.h2_2, a.ih2_2, parents};
    if constexpr (HAS_L2) if (two) {
        // level 2: the children of the root into one grid, their Dirichlet
        // rows on the domain sides
        constexpr int C2 = (1 << D) * G::C, NE2 = (C2 + NT - 1) / NT;
        T v2u[NE2], v2r[NE2];
#pragma unroll
        for (int q = 0; q < NE2; q++) {
            const int e = (int)threadIdx.x + q * NT, o = (e < C2 ? e : 0) / G::C;
            const size_t bx = (size_t)a.child[root * 8 + o];
            v2u[q] = e < C2 ? a.u[bx * G::C + e % G::C] : T(0);
            v2r[q] = e < C2 ? a.rho[bx * G::C + e % G::C] : T(0);
        }
        for (int g = threadIdx.x; g < 2 * D * L2::F; g += NT) {
            // side s, grid face cell m: tangential coordinates (t1, t2)
            const int side = g / L2::F, m = g % L2::F, d = side >> 1;
            const int x1 = m % L2::M, x2 = D == 3 ? m / L2::M : 0;
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            const int o = ((side & 1) << d) | ((x1 >= N ? 1 : 0) << t1) | (D == 3 && x2 >= N ? 1 << t2 : 0);
            const BoxInfo &bi = a.info[a.child[root * 8 + o]];
            const int mb = (x1 % N) + (D == 3 ? N * (x2 % N) : 0);
            l2_bc[g] = a.homog ? T(0) : (T)a.bc[(size_t)bi.bcoff[side] * G::F + mb];
        }
#pragma unroll
        for (int q = 0; q < NE2; q++) {
            const int e = (int)threadIdx.x + q * NT, o = e / G::C;
            if (e >= C2) continue;
            int i, j, k;
            cell_of<D, N>(e % G::C, i, j, k);
            const int gi = i + (o & 1) * N, gj = j + ((o >> 1) & 1) * N, gk = D == 3 ? k + ((o >> 2) & 1) * N : 0;
            l2_u[L2::pad(gi, gj, gk)] = v2u[q];
            l2_rho[L2::at(gi, gj, gk)] = v2r[q];
            // after a restriction from level 3: the copy v' of level 2
            if (mode == COARSE_V2_FROM_3) a.uold[(size_t)a.child[root * 8 + o] * G::C + e % G::C] = v2u[q];
        }
        __syncthreads();
        lv2.ghosts();
        if (mode == COARSE_V2_FROM_3) lv2.crhs();
        lv2.gsrb(a.n_down);
        // residual and u restricted into the root: level 1 then starts as
        // after a restriction from level 2
        for (int e = threadIdx.x; e < G::C; e += NT) {
            int i, j, k;
            cell_of<D, N>(e, i, j, k);
            const int c = i + N * (j + N * k);
            T mu, mr;
            lv2.resid_restrict(c, mu, mr);
            grho[e] = mr;
            f_u[c] = (double)mu;
            f_rho[c] = (double)mr;
            f_uold[c] = 0.0;
        }
    }
    if (!two) {
#pragma unroll
        for (int q = 0; q < NE; q++) {
            const int e = (int)threadIdx.x + q * NT;
            if (e < G::C) {
                int i, j, k;
                cell_of<D, N>(e, i, j, k);
                const int c = i + N * (j + N * k);
                // the right-hand side, or after a restriction from level 2
                // the restricted residual
                f_u[c] = lu[q];
                f_rho[c] = lr[q];
                f_uold[c] = 0.0;
            }
        }
    }
    for (int p = G::C + (int)threadIdx.x; p < CG::TOT; p += NT) {
        f_u[p] = 0.0;
        f_rho[p] = 0.0;
        f_uold[p] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < NBC; q++) {
        const int g = (int)threadIdx.x + q * NT;
        if (g < 2 * D * G::F) f_bc[g] = lb[q];
    }
    __syncthreads();
    // Dirichlet values of the coarser grids: means of the covered values
    for (int li = 1; li < CG::NG; li++) {
        const int n = N >> li, F = D == 3 ? n * n : n, Ff = D == 3 ? 4 * n * n : 2 * n, nf = 2 * n;
        int bo = 0, bof = 0;
        for (int q = 0; q < li; q++) {
            bof = bo;
            bo += 2 * D * (D == 3 ? (N >> q) * (N >> q) : (N >> q));
        }
        for (int g = threadIdx.x; g < 2 * D * F; g += blockDim.x) {
            const int side = g / F, m = g % F;
            const int A = m % n, Cc = D == 3 ? m / n : 0;
            double acc = 0.0;
            for (int dc = 0; dc < (D == 3 ? 2 : 1); dc++)
                for (int da = 0; da < 2; da++) acc += f_bc[bof + side * Ff + (2 * A + da) + nf * (2 * Cc + dc)];
            f_bc[bo + side * F + m] = acc * (D == 3 ? 0.25 : 0.5);
        }
        __syncthreads();
    }
    if (mode == COARSE_V_FROM_2 || two) {
        // level 1 right after restriction from level 2: copy v', FAS
        // right-hand side, then the V-cycle from level 1
        st.template uold_crhs<0>();
        st.template vcycle<0>();
    } else if (mode == COARSE_V_TOP1) {
        st.template vcycle<0>();
    } else {
        st.template fmg<0>();
    }
    for (int e = threadIdx.x; e < G::C; e += blockDim.x) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int c = i + N * (j + N * k);
        gu[e] = (T)f_u[c];
        if (guold && mode != COARSE_V_TOP1) guold[e] = (T)f_uold[c];
    }
    if constexpr (HAS_L2) {
        if (!two) return;
        // back to level 2: correction from the root, smoothing, store
        lv2.prolong(f_u, f_uold);
        lv2.gsrb(a.n_up);
#pragma unroll 4
        for (int e = threadIdx.x; e < (1 << D) * G::C; e += NT) {
            const int o = e / G::C;
            int i, j, k;
            cell_of<D, N>(e % G::C, i, j, k);
            const int c = L2::pad(i + (o & 1) * N, j + ((o >> 1) & 1) * N, D == 3 ? k + ((o >> 2) & 1) * N : 0);
            a.u[(size_t)a.child[root * 8 + o] * G::C + e % G::C] = l2_u[c];
        }
    }
}

// ---------------------------------------------------------------------------
// levels <= 1 of a tree on a general domain: a coarse grid of several
// level-1 boxes and Neumann or periodic sides (paper §2.2, §3, §3.2)
// ---------------------------------------------------------------------------
// Grid g = 0 is level 1 (N cells per side), grids g = 1 .. NG-1 the extra
// coarse grids of N/2, ..., 2 cells below it.  Every level-1 box (root r, box
// id r: level 1 comes first in the box order) has one box on every grid,
// linked to the boxes of its neighbouring roots as the roots are (a periodic
// side names its wrapped neighbour, a side without a neighbour is physical),
// so a non-square coarse grid has several 2^D-cell boxes at the bottom.  One
// workgroup keeps all grids in FP64 in a global scratch area (some KB per
// root, cache resident), natural order x fastest, and runs the FAS cycle
// (paper §3.2) on them: the smoothing, residual, restriction, FAS right-hand
// side and 2-1-1 prolongation of the box kernels, with side ghosts from the
// neighbouring root's box or the boundary values.  Phases end with workgroup
// barriers; within a phase the arrays read and written are distinct, except
// the in-place red-black update, which reads only the other colour and the
// cell's own old value.
template <int D, int N>
struct GenGeo {
    static constexpr int lg(int n) { return n <= 1 ? 0 : 1 + lg(n / 2); }
    static constexpr int NG = lg(N);  // grids of N, N/2, ..., 2 cells
    static constexpr int n(int g) { return N >> g; }
    static constexpr int cells(int g) { return D == 3 ? n(g) * n(g) * n(g) : n(g) * n(g); }
    static constexpr int off(int g) { return g == 0 ? 0 : off(g - 1) + cells(g - 1); }
    static constexpr int TOT = off(NG);
    static constexpr int fsz(int g) { return D == 3 ? n(g) * n(g) : n(g); }
    static constexpr int boff(int g) { return g == 0 ? 0 : boff(g - 1) + 2 * D * fsz(g - 1); }
    static constexpr int BTOT = boff(NG);
};

template <int D, int N>
struct GenState {
    using GG = GenGeo<D, N>;
    const BoxInfo *info;
    double *U, *RHO, *UOLD, *RES, *BC;  // [root][TOT] each, BC [root][BTOT]
    int R, homog, n_down, n_up, n_base;
    double *E;             // coefficients [root][TOT] (OPK_EPS)
    const int32_t *bx;     // x index of the boxes (roots first)
    int opk;               // operator (OPK_* bits)
    const int32_t *dnbr;   // OPK_PROLONG_LIN: roots' same-level boxes across edges and corners
    double *WT;            // with an operator: the 2D side weights of every cell and their
                           // sum, [2D + 1][root][TOT] (prep_weights)

    __device__ static double hgrid(int g) { return (double)(1 << g) / (double)N; }
    __device__ double *at(double *f, int r, int g) const { return f + (size_t)r * GG::TOT + GG::off(g); }
    __device__ static int cidx(int n, int i, int j, int k) { return i + n * (j + n * k); }
    // boundary value of side s next to cell (i, j, k) of root r on grid g
    // (tangential axes in increasing order, the first fastest)
    __device__ double bval(int r, int g, int s, int i, int j, int k) const {
        if (homog) return 0.0;
        const int n = GG::n(g), d = s >> 1;
        const int m = d == 0 ? j + n * k : d == 1 ? i + n * k : i + n * j;
        return BC[(size_t)r * GG::BTOT + GG::boff(g) + s * GG::fsz(g) + m];
    }
    // value across side s of cell (i, j, k) of root r on grid g: a cell of
    // the box, of the neighbouring root's box, or the physical ghost
    __device__ double across(const double *f0, int r, int g, int s, int i, int j, int k) const {
        const int n = GG::n(g), d = s >> 1, hi = s & 1;
        int x[3] = {i, j, k};
        x[d] += hi ? 1 : -1;
        const double *f = f0 + GG::off(g);
        if (x[d] >= 0 && x[d] < n) return f[(size_t)r * GG::TOT + cidx(n, x[0], x[1], x[2])];
        const int v = info[r].nbr[s];
        if (v >= 0) {
            x[d] = hi ? 0 : n - 1;
            return f[(size_t)v * GG::TOT + cidx(n, x[0], x[1], x[2])];
        }
        const double uc = f[(size_t)r * GG::TOT + cidx(n, i, j, k)];
        return phys_ghost<double>(neumann_side(info[r].flags, s), bval(r, g, s, i, j, k), uc, hgrid(g));
    }
    __device__ double nbs(const double *f, int r, int g, int i, int j, int k) const {
        double sum = (across(f, r, g, 0, i, j, k) + across(f, r, g, 1, i, j, k)) +
                     (across(f, r, g, 2, i, j, k) + across(f, r, g, 3, i, j, k));
        if (D == 3) sum = sum + (across(f, r, g, 4, i, j, k) + across(f, r, g, 5, i, j, k));
        return sum;
    }
    // coefficient across side s of cell (i, j, k): the cell there, or the
    // cell's own on a physical side
    __device__ double eacross(int r, int g, int s, int i, int j, int k) const {
        const int n = GG::n(g), d = s >> 1, hi = s & 1;
        int x[3] = {i, j, k};
        x[d] += hi ? 1 : -1;
        const double *f = E + GG::off(g);
        if (x[d] >= 0 && x[d] < n) return f[(size_t)r * GG::TOT + cidx(n, x[0], x[1], x[2])];
        const int v = info[r].nbr[s];
        if (v >= 0) {
            x[d] = hi ? 0 : n - 1;
            return f[(size_t)v * GG::TOT + cidx(n, x[0], x[1], x[2])];
        }
        return f[(size_t)r * GG::TOT + cidx(n, i, j, k)];
    }
    // left edge (x = r) of root r's box on grid g (its grids cover one unit)
    __device__ double x0(int r, int g) const { return (double)(bx[r] - 1) * (double)GG::n(g) * hgrid(g); }
    __device__ double *wt(int q, int r, int g) const { return WT + ((size_t)q * R + r) * GG::TOT + GG::off(g); }
    // The side weights of the operator at every cell of every grid, and their
    // sum, formed once per call (the coefficients do not change during it):
    // w_s = 2 ec en / (ec + en) with eps, times (x of the face) / (x of the
    // centre) on the x sides in the cylindrical form
    __device__ void prep_weights() const {
        for (int g = 0; g < GG::NG; g++) {
            const int n = GG::n(g), NC = GG::cells(g);
            const double h = hgrid(g);
            const bool eps = opk & OPK_EPS, cyl = opk & OPK_CYL;
            for (int e = threadIdx.x; e < R * NC; e += blockDim.x) {
                const int r = e / NC, c = e % NC;
                int i, j, k;
                ijk(n, c, i, j, k);
                const double ec = eps ? at(E, r, g)[c] : 1.0;
                const double xl = cyl ? x0(r, g) : 0.0;
                const double rc = xl + (i + 0.5) * h;
                double d = 0.0;
                for (int s = 0; s < 2 * D; s++) {
                    double w = 1.0;
                    if (eps) {
                        const double en = eacross(r, g, s, i, j, k);
                        w = 2.0 * ec * en / (ec + en);
                    }
                    if (cyl && s < 2) w *= (xl + (i + s) * h) / rc;
                    wt(s, r, g)[c] = w;
                    d += w;
                }
                wt(2 * D, r, g)[c] = d;
            }
        }
        __syncthreads();
    }
    // with the operator: sum over the sides of w_s f_s, dg = sum of w_s
    __device__ double osum(const double *f, int r, int g, int i, int j, int k, double &dg) const {
        const int c = cidx(GG::n(g), i, j, k);
        double sum = 0.0;
        for (int s = 0; s < 2 * D; s++) sum += wt(s, r, g)[c] * across(f, r, g, s, i, j, k);
        dg = wt(2 * D, r, g)[c];
        return sum;
    }
    // h^2 (L f) at cell (i, j, k) of grid g
    __device__ double oph2(const double *f, int r, int g, int i, int j, int k) const {
        const double uc = at(const_cast<double *>(f), r, g)[cidx(GG::n(g), i, j, k)];
        if (!opk) return nbs(f, r, g, i, j, k) - double(2 * D) * uc;
        double dg;
        const double sm = osum(f, r, g, i, j, k, dg);
        return sm - dg * uc;
    }
    // restriction weight of column i of grid g (volume in the cylindrical form)
    __device__ double rw(int r, int g, int i) const {
        return (opk & OPK_CYL) ? x0(r, g) + (i + 0.5) * hgrid(g) : 1.0;
    }
    // mean of the 2^D block under coarse cell (I, J, K) of grid g+1 for field f
    __device__ double block_mean(const double *f, int r, int g, int I, int J, int K) const {
        const int n = GG::n(g);
        const bool cyl = opk & OPK_CYL;
        double acc = 0.0, vol = 0.0;
        for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
            for (int dj = 0; dj < 2; dj++)
                for (int di = 0; di < 2; di++) {
                    const int i = 2 * I + di;
                    const double v = at(const_cast<double *>(f), r, g)[cidx(n, i, 2 * J + dj, D == 3 ? 2 * K + dk : 0)];
                    const double wq = rw(r, g, i);
                    acc += cyl ? wq * v : v;
                    vol += wq;
                }
        return cyl ? acc / vol : (D == 3 ? 0.125 : 0.25) * acc;
    }
    __device__ static void ijk(int n, int c, int &i, int &j, int &k) {
        i = c % n;
        j = (c / n) % n;
        k = D == 3 ? c / (n * n) : 0;
    }
    // one red (0) or black (1) half sweep of grid g, every root
    __device__ void half(int g, int colour) const {
        const int n = GG::n(g), hn = n / 2, nq = GG::cells(g) / 2;
        const double h = hgrid(g), h2 = h * h;
        for (int e = threadIdx.x; e < R * nq; e += blockDim.x) {
            const int r = e / nq, q = e % nq;
            const int row = q / hn, j = row % n, k = D == 3 ? row / n : 0;
            const int i = 2 * (q % hn) + ((colour + j + k + D) & 1);
            const int c = cidx(n, i, j, k);
            double v;
            if (opk) {
                double dg;
                const double sm = osum(U, r, g, i, j, k, dg);
                v = (sm - h2 * at(RHO, r, g)[c]) / dg;
            } else {
                v = (nbs(U, r, g, i, j, k) - h2 * at(RHO, r, g)[c]) / double(2 * D);
            }
            at(U, r, g)[c] = v;
        }
        __syncthreads();
    }
    __device__ void gsrb(int g, int nsweep) const {
        for (int q = 0; q < nsweep; q++) {
            half(g, 0);
            half(g, 1);
        }
    }
    // grid g+1 <- means of u and of the residual rho - L u of grid g
    __device__ void resid_restrict(int g) const {
        const int n = GG::n(g), nc = GG::n(g + 1), NC = GG::cells(g + 1);
        const double h = hgrid(g), ih2 = 1.0 / (h * h);
        const double w = D == 3 ? 0.125 : 0.25;
        for (int e = threadIdx.x; e < R * NC; e += blockDim.x) {
            const int r = e / NC, C = e % NC;
            int I, J, K;
            ijk(nc, C, I, J, K);
            double au = 0.0, ar = 0.0, vol = 0.0;
            const bool cyl = opk & OPK_CYL;
            for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
                for (int dj = 0; dj < 2; dj++)
                    for (int di = 0; di < 2; di++) {
                        const int i = 2 * I + di, j = 2 * J + dj, k = D == 3 ? 2 * K + dk : 0;
                        const int c = cidx(n, i, j, k);
                        const double uc = at(U, r, g)[c];
                        const double res = at(RHO, r, g)[c] - oph2(U, r, g, i, j, k) * ih2;
                        const double wq = rw(r, g, i);
                        au += cyl ? wq * uc : uc;
                        ar += cyl ? wq * res : res;
                        vol += wq;
                    }
            at(U, r, g + 1)[C] = cyl ? au / vol : w * au;
            at(RES, r, g + 1)[C] = cyl ? ar / vol : w * ar;
        }
        __syncthreads();
    }
    // rho of grid g -> grid g+1 (FMG)
    __device__ void restrict_rho(int g) const {
        const int n = GG::n(g), nc = GG::n(g + 1), NC = GG::cells(g + 1);
        const double w = D == 3 ? 0.125 : 0.25;
        for (int e = threadIdx.x; e < R * NC; e += blockDim.x) {
            const int r = e / NC, C = e % NC;
            int I, J, K;
            ijk(nc, C, I, J, K);
            if (opk & OPK_CYL) {
                at(RHO, r, g + 1)[C] = block_mean(RHO, r, g, I, J, K);
                continue;
            }
            double acc = 0.0;
            for (int dk = 0; dk < (D == 3 ? 2 : 1); dk++)
                for (int dj = 0; dj < 2; dj++)
                    for (int di = 0; di < 2; di++)
                        acc += at(RHO, r, g)[cidx(n, 2 * I + di, 2 * J + dj, D == 3 ? 2 * K + dk : 0)];
            at(RHO, r, g + 1)[C] = w * acc;
        }
        __syncthreads();
    }
    // the copy v' of grid g and, on the roots marked in `parents` (every
    // root below level 1), the FAS right-hand side rho <- rbar + L u
    __device__ void uold_crhs(int g, bool all_parents) const {
        const int n = GG::n(g), NC = GG::cells(g);
        const double h = hgrid(g), ih2 = 1.0 / (h * h);
        for (int e = threadIdx.x; e < R * NC; e += blockDim.x) {
            const int r = e / NC, c = e % NC;
            int i, j, k;
            ijk(n, c, i, j, k);
            const double uc = at(U, r, g)[c];
            at(UOLD, r, g)[c] = uc;
            if (all_parents || !(info[r].flags & FLAG_LEAF))
                at(RHO, r, g)[c] = at(RES, r, g)[c] + oph2(U, r, g, i, j, k) * ih2;
        }
        __syncthreads();
    }
    // u - v' on grid g at the cell (I, J, K) + one step along `axis` (sgn), or
    // at the cell itself (sgn = 0); across a box side the difference of the
    // ghosts of u and of v'
    __device__ double delta(int r, int g, int axis, int sgn, int I, int J, int K) const {
        const int n = GG::n(g);
        if (sgn == 0) {
            const int c = cidx(n, I, J, K);
            return at(U, r, g)[c] - at(UOLD, r, g)[c];
        }
        int x[3] = {I, J, K};
        x[axis] += sgn;
        if (x[axis] >= 0 && x[axis] < n) {
            const int c = cidx(n, x[0], x[1], x[2]);
            return at(U, r, g)[c] - at(UOLD, r, g)[c];
        }
        const int s = 2 * axis + (sgn > 0 ? 1 : 0);
        return across(U, r, g, s, I, J, K) - across(UOLD, r, g, s, I, J, K);
    }
    // u - v' of grid g at cell c0 with every axis at most one cell outside
    // the root's box: inside, across one side (delta), or across an edge or
    // corner: the same-level root there, else the linear extrapolation of
    // the edge and corner ghosts (k_vprolong_lin).  `outs` limits the axes
    // outside (callers go from corners to edges to sides, no recursion).
    __device__ double dval_side(int r, int g, const int c0[3]) const {
        const int n = GG::n(g);
        for (int d = 0; d < D; d++) {
            const int o = c0[d] < 0 ? -1 : c0[d] >= n ? 1 : 0;
            if (o) {
                int in[3] = {c0[0], c0[1], c0[2]};
                in[d] -= o;
                return delta(r, g, d, o, in[0], in[1], in[2]);
            }
        }
        const int c = cidx(n, c0[0], c0[1], c0[2]);
        return at(U, r, g)[c] - at(UOLD, r, g)[c];
    }
    // across an edge or corner (2 or 3 axes outside): the root there, or
    // -1 when there is none
    __device__ double dval_diag(int r, int g, const int c0[3], const int o[3], bool &found) const {
        const int n = GG::n(g);
        const int v = dnbr[(size_t)r * 27 + (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
        found = v >= 0;
        if (!found) return 0.0;
        int q[3] = {c0[0], c0[1], c0[2]};
        for (int d = 0; d < D; d++)
            if (o[d]) q[d] = o[d] < 0 ? n - 1 : 0;
        const int c = cidx(n, q[0], q[1], q[2]);
        return at(U, v, g)[c] - at(UOLD, v, g)[c];
    }
    __device__ double dval_edge(int r, int g, const int c0[3], const int o[3]) const {
        bool found;
        const double dv = dval_diag(r, g, c0, o, found);
        if (found) return dv;
        int ax[2], na = 0;
        for (int d = 0; d < D; d++)
            if (o[d]) ax[na++] = d;
        int b[3] = {c0[0], c0[1], c0[2]}, c[3] = {c0[0], c0[1], c0[2]}, in[3] = {c0[0], c0[1], c0[2]};
        b[ax[0]] -= o[ax[0]];
        c[ax[1]] -= o[ax[1]];
        in[ax[0]] -= o[ax[0]];
        in[ax[1]] -= o[ax[1]];
        return dval_side(r, g, b) + dval_side(r, g, c) - dval_side(r, g, in);
    }
    __device__ double dval(int r, int g, const int c0[3]) const {
        const int n = GG::n(g);
        int o[3] = {0, 0, 0}, na = 0;
        for (int d = 0; d < D; d++) {
            o[d] = c0[d] < 0 ? -1 : c0[d] >= n ? 1 : 0;
            na += o[d] != 0;
        }
        if (na <= 1) return dval_side(r, g, c0);
        if (na == 2) return dval_edge(r, g, c0, o);
        bool found;
        const double dv = dval_diag(r, g, c0, o, found);
        if (found) return dv;
        // a corner: its three edge ghosts minus its three side ghosts plus
        // the inner cell
        double val = 0.0;
        for (int d = 0; d < 3; d++) {
            int e[3] = {c0[0], c0[1], c0[2]}, oe[3] = {o[0], o[1], o[2]};
            e[d] -= o[d];
            oe[d] = 0;
            val += dval_edge(r, g, e, oe);
        }
        for (int d = 0; d < 3; d++) {
            int sd[3] = {c0[0] - o[0], c0[1] - o[1], c0[2] - o[2]};
            sd[d] += o[d];
            val -= dval_side(r, g, sd);
        }
        const int in[3] = {c0[0] - o[0], c0[1] - o[1], c0[2] - o[2]};
        return val + dval_side(r, g, in);
    }
    // u of grid g += P211(u - v' of grid g+1); with store_old, v' of grid g
    // first receives u (FMG)
    __device__ void prolong(int g, bool store_old) const {
        const int n = GG::n(g), NC = GG::cells(g);
        for (int e = threadIdx.x; e < R * NC; e += blockDim.x) {
            const int r = e / NC, c = e % NC;
            int i, j, k;
            ijk(n, c, i, j, k);
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
            double v;
            if (opk & OPK_PROLONG_LIN) {
                // bi/trilinear (see k_vprolong_lin)
                const int P[3] = {I, J, K};
                const int sg[3] = {sx, sy, sz};
                auto dv = [&](int a, int b, int c) {
                    const int q[3] = {P[0] + a * sg[0], P[1] + b * sg[1], D == 3 ? P[2] + c * sg[2] : 0};
                    return dval(r, g + 1, q);
                };
                if (D == 2)
                    v = 0.5625 * dv(0, 0, 0) + 0.1875 * dv(1, 0, 0) + 0.1875 * dv(0, 1, 0) + 0.0625 * dv(1, 1, 0);
                else
                    v = 0.421875 * dv(0, 0, 0) + 0.140625 * ((dv(1, 0, 0) + dv(0, 1, 0)) + dv(0, 0, 1)) +
                        0.046875 * ((dv(1, 1, 0) + dv(1, 0, 1)) + dv(0, 1, 1)) + 0.015625 * dv(1, 1, 1);
            } else if (opk & OPK_PROLONG_EPS) {
                // eps-weighted (see k_vprolong)
                const int nc = GG::n(g + 1);
                const int sg[3] = {sx, sy, sz};
                const double d0 = delta(r, g + 1, 0, 0, I, J, K);
                const double e0 = at(E, r, g + 1)[cidx(nc, I, J, K)];
                v = d0;
                for (int d = 0; d < D; d++) {
                    int Q[3] = {I, J, K};
                    Q[d] += sg[d];
                    const double ed = (Q[d] >= 0 && Q[d] < nc) ? at(E, r, g + 1)[cidx(nc, Q[0], Q[1], Q[2])]
                                                              : eacross(r, g + 1, 2 * d + (sg[d] > 0 ? 1 : 0), I, J, K);
                    v += ed / (2.0 * (e0 + ed)) * (delta(r, g + 1, d, sg[d], I, J, K) - d0);
                }
            } else if (D == 2)
                v = 0.5 * delta(r, g + 1, 0, 0, I, J, K) + 0.25 * delta(r, g + 1, 0, sx, I, J, K) +
                    0.25 * delta(r, g + 1, 1, sy, I, J, K);
            else
                v = 0.25 * (((delta(r, g + 1, 0, 0, I, J, K) + delta(r, g + 1, 0, sx, I, J, K)) +
                             delta(r, g + 1, 1, sy, I, J, K)) +
                            delta(r, g + 1, 2, sz, I, J, K));
            const double uc = at(U, r, g)[c];
            if (store_old) at(UOLD, r, g)[c] = uc;
            at(U, r, g)[c] = uc + v;
        }
        __syncthreads();
    }
    // FAS V-cycle from grid g0 (paper §3.2)
    __device__ void vcycle(int g0) const {
        for (int g = g0; g < GG::NG - 1; g++) {
            gsrb(g, n_down);
            resid_restrict(g);
            uold_crhs(g + 1, true);
        }
        gsrb(GG::NG - 1, n_base);
        for (int g = GG::NG - 2; g >= g0; g--) {
            prolong(g, false);
            gsrb(g, n_up);
        }
    }
    // FMG from a zero guess on grids 0 .. NG-1, then the V-cycle from grid 0
    __device__ void fmg() const {
        for (int g = 0; g < GG::NG - 1; g++) restrict_rho(g);
        const int last = GG::NG - 1, nl = GG::cells(last);
        for (int e = threadIdx.x; e < R * nl; e += blockDim.x) {
            const int r = e / nl, c = e % nl;
            at(UOLD, r, last)[c] = at(U, r, last)[c];
        }
        __syncthreads();
        gsrb(last, n_base);
        for (int g = last - 1; g >= 0; g--) {
            prolong(g, true);
            vcycle(g);
        }
    }
};

template <int D, int N, typename T>
__global__ __launch_bounds__(COARSE_NT) void k_coarse_gen(CoarseGenArgs<T> a) {
    using GG = GenGeo<D, N>;
    using G = Geo<D, N>;
    const int R = a.n_roots;
    // the grids in LDS where they fit (the kernel fills them from the boxes
    // and writes its results back, so the scratch holds nothing between
    // calls), else in the caller's scratch
    extern __shared__ double gen_lds[];
    double *ws = a.in_lds ? gen_lds : a.ws;
    // with the grids in LDS, the roots' box records and x indices follow
    // them there (every cell's neighbour lookup reads them)
    const BoxInfo *info = a.info;
    const int32_t *bx = a.bx;
    // grids, then (with an operator) the side weights: the layout of
    // coarse_gen_doubles
    const size_t ngrid = (size_t)R * (5 * GG::TOT + GG::BTOT);
    const size_t nwt = a.opk ? (size_t)(2 * D + 1) * R * GG::TOT : 0;
    if (a.in_lds) {
        BoxInfo *li = reinterpret_cast<BoxInfo *>(gen_lds + ngrid + nwt);
        int32_t *lx = reinterpret_cast<int32_t *>(li + R);
        for (int e = threadIdx.x; e < R; e += blockDim.x) {
            li[e] = a.info[e];
            if (a.bx) lx[e] = a.bx[e];
        }
        info = li;
        if (a.bx) bx = lx;
        __syncthreads();
    }
    GenState<D, N> st{info, ws, ws + (size_t)R * GG::TOT, ws + (size_t)2 * R * GG::TOT,
                      ws + (size_t)3 * R * GG::TOT, ws + (size_t)4 * R * GG::TOT, R, a.homog,
                      a.n_down, a.n_up, a.n_base,
                      ws + (size_t)4 * R * GG::TOT + (size_t)R * GG::BTOT, bx, a.opk, a.dnbr, ws + ngrid};
    const int mode = a.mode;
    // level 1 from the roots' boxes (colour-split in the tree's arrays), the
    // coarser grids start at zero
    for (int e = threadIdx.x; e < R * GG::TOT; e += blockDim.x) {
        const int r = e / GG::TOT, p = e % GG::TOT;
        double u = 0.0, rho = 0.0, res = 0.0;
        if (p < G::C) {
            const int i = p % N, j = (p / N) % N, k = D == 3 ? p / (N * N) : 0;
            const size_t gi = (size_t)r * G::C + cpos<D, N>(i, j, k);
            const bool leaf = a.info[r].flags & FLAG_LEAF;
            u = mode == COARSE_FMG ? 0.0 : (double)a.u[gi];
            const double rg = (double)a.rho[gi];
            // after the restriction from level 2 the rho of a refined root
            // is the restricted residual; its FAS right-hand side follows
            if (mode == COARSE_V_FROM_2 && !leaf) res = rg;
            else rho = rg;
        }
        st.U[e] = u;
        st.RHO[e] = rho;
        st.RES[e] = res;
        st.UOLD[e] = 0.0;
        if (a.opk & OPK_EPS) {
            if (p < G::C) {
                const int i = p % N, j = (p / N) % N, k = D == 3 ? p / (N * N) : 0;
                st.E[e] = a.eps[(size_t)r * G::C + cpos<D, N>(i, j, k)];
            }
        }
    }
    // the coefficients of the coarser grids: means of the finer ones
    if (a.opk & OPK_EPS) {
        __syncthreads();
        for (int g = 0; g + 1 < GG::NG; g++) {
            const int NC = GG::cells(g + 1), nc = GG::n(g + 1);
            for (int e = threadIdx.x; e < R * NC; e += blockDim.x) {
                const int r = e / NC, C = e % NC;
                const int I = C % nc, J = (C / nc) % nc, K = D == 3 ? C / (nc * nc) : 0;
                st.at(st.E, r, g + 1)[C] = st.block_mean(st.E, r, g, I, J, K);
            }
            __syncthreads();
        }
    }
    // boundary values: the roots' rows on grid 0, means of the covered
    // values below
    for (int e = threadIdx.x; e < R * 2 * D * G::F; e += blockDim.x) {
        const int r = e / (2 * D * G::F), g = e % (2 * D * G::F), s = g / G::F;
        const int32_t row = a.info[r].bcoff[s];
        st.BC[(size_t)r * GG::BTOT + g] = (row >= 0 && !a.homog) ? a.bc[(size_t)row * G::F + g % G::F] : 0.0;
    }
    __syncthreads();
    for (int gl = 1; gl < GG::NG; gl++) {
        const int n = GG::n(gl), F = GG::fsz(gl), Ff = GG::fsz(gl - 1), nf = 2 * n;
        for (int e = threadIdx.x; e < R * 2 * D * F; e += blockDim.x) {
            const int r = e / (2 * D * F), g = e % (2 * D * F), s = g / F, m = g % F;
            const int A = m % n, Cc = D == 3 ? m / n : 0;
            const double *src = st.BC + (size_t)r * GG::BTOT + GG::boff(gl - 1) + s * Ff;
            double acc = 0.0;
            for (int dc = 0; dc < (D == 3 ? 2 : 1); dc++)
                for (int da = 0; da < 2; da++) acc += src[(2 * A + da) + nf * (2 * Cc + dc)];
            st.BC[(size_t)r * GG::BTOT + GG::boff(gl) + s * F + m] = acc * (D == 3 ? 0.25 : 0.5);
        }
        __syncthreads();
    }
    if (a.opk) st.prep_weights();
    if (mode == COARSE_V_FROM_2) {
        st.uold_crhs(0, false);
        st.vcycle(0);
    } else if (mode == COARSE_FMG) {
        st.fmg();
    } else {
        st.vcycle(0);
    }
    for (int e = threadIdx.x; e < R * G::C; e += blockDim.x) {
        const int r = e / G::C, p = e % G::C;
        const int i = p % N, j = (p / N) % N, k = D == 3 ? p / (N * N) : 0;
        const size_t gi = (size_t)r * G::C + cpos<D, N>(i, j, k);
        a.u[gi] = (T)st.U[(size_t)r * GG::TOT + p];
        if (a.uold && mode != COARSE_V_TOP1) a.uold[gi] = (T)st.UOLD[(size_t)r * GG::TOT + p];
    }
}

// ---------------------------------------------------------------------------
// the composite operator and its transpose on leaf cells (adjoint)
// ---------------------------------------------------------------------------
// With homogeneous Dirichlet values the composite operator L is a sparse
// matrix on the leaf cells; its rows are the stencil with the ghost formulas
// written out (paper §2.4, §3.3).  On adaptive grids L is not symmetric: the
// refinement-boundary ghost couples a fine face cell to the coarse cell
// (1/2 uH / h^2) while the coarse cell sees the fine cells through the mean of
// their parent (1/2^D / H^2), and the fine ghost also involves the partner and
// the next inner cell.  k_apply_lt gathers, for every leaf cell c, the entries
// L_rc y_r of all rows r that reference c:
//   - in-box and same-level leaf neighbours: y_r / h^2, and -2D y_c / h^2;
//   - a refined same-level neighbour: the 2^(D-1) fine face cells next to c
//     reference c as their uH: 1/2 / (h/2)^2 = 2 / h^2 each;
//   - a physical side: -y_c / h^2 (ghost -u_c);
//   - a refinement side, c on the face layer: k1 y_c / h^2 (k1 = 1 in 2D, 5/4
//     in 3D), -1/4 y / h^2 for each tangential partner (their ghosts use c),
//     and the coarse cell R next to c's parent cell: y_R / (2^D (2h)^2);
//   - a refinement side, c on the second layer: -1/4 y_f / h^2 for the face
//     cell f in front (its ghost uses c as the inner cell) and y_R / (2^D (2h)^2).

__device__ __forceinline__ double level_ih2(int N, int level) {
    const double h = 1.0 / ((double)N * ldexp(1.0, level - 1));
    return 1.0 / (h * h);
}

template <int D, int N, int S>
__device__ __forceinline__ void coarse_cell(int flags, const int c[3], int q[3]) {
    using SD = SideOf<S>;
    q[SD::d] = SD::hi ? 0 : N - 1;
    q[SD::t1] = obit(flags, SD::t1) * (N / 2) + (c[SD::t1] >> 1);
    q[SD::t2] = D == 3 ? obit(flags, SD::t2) * (N / 2) + (c[SD::t2] >> 1) : 0;
}

// contribution to (L^T y)_c across side S, c on the face layer of S
template <int D, int N, int S>
__device__ double lt_face(const BoxInfo &bi, const int c[3], const double *s, const double *__restrict__ y,
                          const int *__restrict__ child, double ih2) {
    using SD = SideOf<S>;
    using G = Geo<D, N>;
    const int v = bi.nbr[S];
    const double yc = s[padi<D, N>(c[0], c[1], c[2])];
    if (v == -1) return neumann_side(bi.flags, S) ? ih2 * yc : -ih2 * yc;
    if (v >= 0) {
        if (!(bi.flags & (FLAG_NBR_REFINED << S))) {
            int o[3] = {c[0], c[1], c[2]};
            o[SD::d] = SD::hi ? 0 : N - 1;
            return ih2 * y[(size_t)v * G::C + cpos<D, N>(o[0], o[1], o[2])];
        }
        double acc = 0.0;
        for (int sub = 0; sub < (D == 3 ? 4 : 2); sub++) {
            int f[3], bit[3];
            const int g1 = 2 * c[SD::t1] + (sub & 1);
            bit[SD::t1] = g1 / N;
            f[SD::t1] = g1 % N;
            if (D == 3) {
                const int g2 = 2 * c[SD::t2] + (sub >> 1);
                bit[SD::t2] = g2 / N;
                f[SD::t2] = g2 % N;
            } else {
                bit[SD::t2] = 0;
                f[SD::t2] = 0;
            }
            bit[SD::d] = SD::hi ? 0 : 1;
            f[SD::d] = SD::hi ? 0 : N - 1;
            const int oc = bit[0] | (bit[1] << 1) | (D == 3 ? bit[2] << 2 : 0);
            const int ch = child[(size_t)v * 8 + oc];
            acc += y[(size_t)ch * G::C + cpos<D, N>(f[0], f[1], f[2])];
        }
        return 2.0 * ih2 * acc;
    }
    int q[3];
    coarse_cell<D, N, S>(bi.flags, c, q);
    const double yR = y[(size_t)(-v - 2) * G::C + cpos<D, N>(q[0], q[1], q[2])];
    int p1[3] = {c[0], c[1], c[2]};
    p1[SD::t1] ^= 1;
    double part = s[padi<D, N>(p1[0], p1[1], p1[2])];
    if (D == 3) {
        int p2[3] = {c[0], c[1], c[2]};
        p2[SD::t2] ^= 1;
        part += s[padi<D, N>(p2[0], p2[1], p2[2])];
    }
    const double k1 = D == 3 ? 1.25 : 1.0;
    return k1 * ih2 * yc - 0.25 * ih2 * part + ih2 / (4.0 * (1 << D)) * yR;
}

// contribution across side S for c on the second layer of a refinement side
template <int D, int N, int S>
__device__ double lt_layer1(const BoxInfo &bi, const int c[3], const double *s, const double *__restrict__ y,
                            double ih2) {
    using SD = SideOf<S>;
    using G = Geo<D, N>;
    const int v = bi.nbr[S];
    if (v > -2) return 0.0;
    int f[3] = {c[0], c[1], c[2]};
    f[SD::d] = SD::hi ? N - 1 : 0;
    int q[3];
    coarse_cell<D, N, S>(bi.flags, c, q);
    const double yR = y[(size_t)(-v - 2) * G::C + cpos<D, N>(q[0], q[1], q[2])];
    return -0.25 * ih2 * s[padi<D, N>(f[0], f[1], f[2])] + ih2 / (4.0 * (1 << D)) * yR;
}

// out = L^T y on leaf boxes (zero on parents); one launch for all boxes
template <int D, int N>
__global__ __launch_bounds__(256) void k_apply_lt(const BoxInfo *__restrict__ info, const int *__restrict__ child,
                                                  const double *__restrict__ y, double *__restrict__ out, int nb) {
    using G = Geo<D, N>;
    __shared__ double sm[G::BPW * G::PC];
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    double *s = sm + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    const bool leaf = bi.flags & FLAG_LEAF;
    const size_t bo = (size_t)sl.b * G::C;
    Stager<D, N, double> st;
    if (sl.valid && leaf) st.begin(s, bi, y + bo, y, nullptr, 1, sl.t, false);
    __syncthreads();
    if (!sl.valid) return;
    int j, k;
    row_of<D, N>(sl.t, j, k);
    if (!leaf) {
        for (int i = 0; i < N; i++) out[bo + cpos<D, N>(i, j, k)] = 0.0;
        return;
    }
    const double ih2 = level_ih2(N, bi.level);
    for (int i = 0; i < N; i++) {
        const int c[3] = {i, j, k};
        const double yc = s[padi<D, N>(i, j, k)];
        double nbs = 0.0;
        if (i > 0) nbs += s[padi<D, N>(i - 1, j, k)];
        if (i < N - 1) nbs += s[padi<D, N>(i + 1, j, k)];
        if (j > 0) nbs += s[padi<D, N>(i, j - 1, k)];
        if (j < N - 1) nbs += s[padi<D, N>(i, j + 1, k)];
        if (D == 3) {
            if (k > 0) nbs += s[padi<D, N>(i, j, k - 1)];
            if (k < N - 1) nbs += s[padi<D, N>(i, j, k + 1)];
        }
        double acc = ih2 * (nbs - 2.0 * D * yc);
        if (i == 0) acc += lt_face<D, N, 0>(bi, c, s, y, child, ih2);
        if (i == N - 1) acc += lt_face<D, N, 1>(bi, c, s, y, child, ih2);
        if (i == 1) acc += lt_layer1<D, N, 0>(bi, c, s, y, ih2);
        if (i == N - 2) acc += lt_layer1<D, N, 1>(bi, c, s, y, ih2);
        if (j == 0) acc += lt_face<D, N, 2>(bi, c, s, y, child, ih2);
        if (j == N - 1) acc += lt_face<D, N, 3>(bi, c, s, y, child, ih2);
        if (j == 1) acc += lt_layer1<D, N, 2>(bi, c, s, y, ih2);
        if (j == N - 2) acc += lt_layer1<D, N, 3>(bi, c, s, y, ih2);
        if (D == 3) {
            if (k == 0) acc += lt_face<D, N, 4>(bi, c, s, y, child, ih2);
            if (k == N - 1) acc += lt_face<D, N, 5>(bi, c, s, y, child, ih2);
            if (k == 1) acc += lt_layer1<D, N, 4>(bi, c, s, y, ih2);
            if (k == N - 2) acc += lt_layer1<D, N, 5>(bi, c, s, y, ih2);
        }
        out[bo + cpos<D, N>(i, j, k)] = acc;
    }
}

// out = L x on leaf boxes (zero on parents), homogeneous Dirichlet values; x
// must hold the restriction of its leaf values on parent boxes
template <int D, int N>
__global__ __launch_bounds__(256) void k_apply_l(const BoxInfo *__restrict__ info, const double *__restrict__ x,
                                                 double *__restrict__ out, int nb) {
    using G = Geo<D, N>;
    __shared__ double sm[G::BPW * G::PC];
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    double *s = sm + sl.slot * G::PC;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    const bool leaf = bi.flags & FLAG_LEAF;
    const size_t bo = (size_t)sl.b * G::C;
    Stager<D, N, double> st;
    if (sl.valid && leaf) st.begin(s, bi, x + bo, x, nullptr, 1, sl.t, true, 0.0);
    __syncthreads();
    if (sl.valid && leaf) st.end(s, sl.t);
    __syncthreads();
    if (!sl.valid) return;
    const double ih2 = level_ih2(N, bi.level);
    for (int e = sl.t; e < G::C; e += G::TPB) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        out[bo + e] = leaf ? (nb_sum<D, N, double>(s, i, j, k) - 2.0 * D * s[padi<D, N>(i, j, k)]) * ih2 : 0.0;
    }
}

// restriction of field f into the parents of the boxes of one level
template <int D, int N>
__global__ __launch_bounds__(256) void k_restrict_field(const BoxInfo *__restrict__ info, double *f, int64_t b0,
                                                        int nb) {
    using G = Geo<D, N>;
    __shared__ double sm[G::BPW * G::C];
    const Slot<D, N> sl = slot_of<D, N>(b0, nb);
    double *s = sm + sl.slot * G::C;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    const size_t bo = (size_t)sl.b * G::C;
    if (sl.valid) {
        for (int e = sl.t; e < G::C; e += G::TPB) {
            int i, j, k;
            cell_of<D, N>(e, i, j, k);
            s[D == 3 ? i + N * (j + N * k) : i + N * j] = f[bo + e];
        }
    }
    __syncthreads();
    if (sl.valid) restrict_octant<D, N, double, false>(s, f, bi, sl.t);
}

// transpose of the restriction for the boxes of one level: each cell adds
// 1/2^D of its parent cell (run from coarse to fine, so that values on parent
// boxes reach the leaves)
template <int D, int N>
__global__ __launch_bounds__(256) void k_push_down(const BoxInfo *__restrict__ info, double *f, int64_t b0,
                                                   int nb) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(b0, nb);
    if (!sl.valid) return;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    if (bi.parent < 0) return;
    const size_t bo = (size_t)sl.b * G::C, po = (size_t)bi.parent * G::C;
    const double w = D == 3 ? 0.125 : 0.25;
    for (int e = sl.t; e < G::C; e += G::TPB) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        const int X = obit(bi.flags, 0) * G::H + (i >> 1), Y = obit(bi.flags, 1) * G::H + (j >> 1),
                  Z = D == 3 ? obit(bi.flags, 2) * G::H + (k >> 1) : 0;
        f[bo + e] += w * f[po + cpos<D, N>(X, Y, Z)];
    }
}

#ifndef AFMG_INSTANTIATE_ONLY
// per-workgroup (max |a|, sum a b) over n elements with a fixed grid, in a
// fixed order; reduced by k_reduce
__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a, const double *__restrict__ b,
                                             int64_t n, double *__restrict__ partial) {
    __shared__ double rm[256], rs[256];
    double mx = 0.0, ss = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        mx = fmax(mx, fabs(a[i]));
        ss += a[i] * b[i];
    }
    rm[threadIdx.x] = mx;
    rs[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
            rs[threadIdx.x] += rs[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rm[0];
        partial[2 * blockIdx.x + 1] = rs[0];
    }
}

// out = a x + b y + c z (y, z may be null)
__global__ __launch_bounds__(256) void k_lc3(double *out, double a, const double *x, double b, const double *y,
                                             double c, const double *z, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double v = a * x[i];
        if (y) v += b * y[i];
        if (z) v += c * z[i];
        out[i] = v;
    }
}
#endif  // AFMG_INSTANTIATE_ONLY

// dst = (h^D)^pw src on leaf boxes (pw in {-1, 0, 1}), 0 on parent boxes
template <int D, int N>
__global__ __launch_bounds__(256) void k_scale_leaves(const BoxInfo *__restrict__ info, double *dst,
                                                      const double *src, int pw, int nb) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    if (!sl.valid) return;
    const BoxInfo bi = load_box<D, N>(info, sl.b);
    const bool leaf = bi.flags & FLAG_LEAF;
    const double h = 1.0 / ((double)N * ldexp(1.0, bi.level - 1));
    const double hD = D == 3 ? h * h * h : h * h;
    const double f = pw > 0 ? hD : (pw < 0 ? 1.0 / hD : 1.0);
    const size_t bo = (size_t)sl.b * G::C;
    for (int e = sl.t; e < G::C; e += G::TPB) dst[bo + e] = leaf ? f * src[bo + e] : 0.0;
}

// natural-order copy of the leaf boxes of src (colour-split) into dst; parent
// boxes of dst are zeroed
template <int D, int N>
__global__ __launch_bounds__(256) void k_store_leaves(const BoxInfo *__restrict__ info,
                                                      const double *__restrict__ src, double *__restrict__ dst,
                                                      int nb) {
    using G = Geo<D, N>;
    const Slot<D, N> sl = slot_of<D, N>(0, nb);
    if (!sl.valid) return;
    const bool leaf = load_box<D, N>(info, sl.b).flags & FLAG_LEAF;
    const size_t bo = (size_t)sl.b * G::C;
    for (int e = sl.t; e < G::C; e += G::TPB) {
        int i, j, k;
        cell_of<D, N>(e, i, j, k);
        dst[bo + (D == 3 ? i + N * (j + N * k) : i + N * j)] = leaf ? src[bo + e] : 0.0;
    }
}

// gradient with respect to the boundary rows of the leaves:
// d loss / d b_f = -2 lambda_c(f) / h^2 for a Dirichlet side (the boundary
// part of the rhs is 2 b / h^2 per Dirichlet side of a cell) and
// -lambda_c(f) / h for a Neumann side (q / h per Neumann side)
template <int D, int N>
__global__ __launch_bounds__(256) void k_bc_grad(const BoxInfo *__restrict__ info, const double *__restrict__ lam,
                                                 double *__restrict__ bc_bar, int nb) {
    using G = Geo<D, N>;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)nb * 2 * D * G::F) return;
    const int64_t b = g / (2 * D * G::F);
    const int rem = (int)(g % (2 * D * G::F));
    const int side = rem / G::F, m = rem % G::F;
    const BoxInfo *bi = info + b;
    if (!(bi->flags & FLAG_LEAF) || bi->nbr[side] != -1) return;
    const int d = side >> 1, hi = side & 1;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    int x[3];
    x[t1] = m % N;
    x[t2] = D == 3 ? m / N : 0;
    x[d] = hi ? N - 1 : 0;
    const double ih2 = level_ih2(N, bi->level);
    const double lc = lam[(size_t)b * G::C + cpos<D, N>(x[0], x[1], x[2])];
    bc_bar[(size_t)bi->bcoff[side] * G::F + m] = neumann_side(bi->flags, side) ? -sqrt(ih2) * lc : -2.0 * ih2 * lc;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int D, int N, int W = 256>
static inline int wg_count(int64_t nb) {
    constexpr int BPW = W / Geo<D, N>::TPB;
    return (int)((nb + BPW - 1) / BPW);
}

#define AFMG_LAUNCH(kernel, grid, stream, ...)                                                      \
    do {                                                                                            \
        if ((grid) > 0) hipLaunchKernelGGL(kernel, dim3(grid), dim3(256), 0, stream, __VA_ARGS__); \
    } while (0)
#define AFMG_LAUNCH_W(kernel, grid, W, stream, ...)                                               \
    do {                                                                                          \
        if ((grid) > 0) hipLaunchKernelGGL(kernel, dim3(grid), dim3(W), 0, stream, __VA_ARGS__); \
    } while (0)

constexpr int64_t CUBE_MAX_THREADS = int64_t(1) << 19;  // 8192 boxes of 8^3 cells

template <int D, int N, typename T, int W, bool F>
static void launch_level_wf(Op op, const LevelArgs<T> &a, int colour, hipStream_t st) {
    const int g = wg_count<D, N, W>(a.nb);
    switch (op) {
    case Op::GSRB:
        // the complete-level variant pays off where the level fits the GPU in
        // about one round of waves (latency-bound), and on every level in
        // FP32 (3D), where a box's loads are half as long; on larger FP64
        // levels it is no faster (measured on 256^3: levels of 512 and 4096
        // boxes 4-10% faster; 32768 boxes 1-2% slower in FP64, 15% faster in
        // FP32)
        // (the modes of a correction: the caller checked that the level is
        // complete and holds every leaf of the one tree)
        if (a.add_to)
            AFMG_LAUNCH_W((k_gsrb_cube<D, N, T, W, CUBE_ADD>), g, W, st, a, colour);
        else if (a.own_zero)
            AFMG_LAUNCH_W((k_gsrb_cube<D, N, T, W, CUBE_OWN_ZERO>), g, W, st, a, colour);
        else if (!F && a.xmask &&
                 ((D == 3 && sizeof(T) == 4) || (int64_t)a.nb * Geo<D, N>::TPB <= CUBE_MAX_THREADS))
            AFMG_LAUNCH_W((k_gsrb_cube<D, N, T, W, CUBE_PLAIN>), g, W, st, a, colour);
        else
            AFMG_LAUNCH_W((k_gsrb<D, N, T, W, F>), g, W, st, a, colour);
        break;
    case Op::RESID_RESTRICT: AFMG_LAUNCH_W((k_resid_restrict<D, N, T, W, F>), g, W, st, a); break;
    case Op::COARSE_RHS: AFMG_LAUNCH_W((k_coarse_rhs<D, N, T, W, F>), g, W, st, a); break;
    case Op::PROLONG: AFMG_LAUNCH_W((k_prolong<D, N, T, W, F>), g, W, st, a); break;
    case Op::RESTRICT_RHO: AFMG_LAUNCH((k_restrict_rho<D, N, T, F>), (wg_count<D, N, 256>(a.nb)), st, a); break;
    }
}
template <int D, int N, typename T, int W>
static void launch_level_w(Op op, const LevelArgs<T> &a, int colour, hipStream_t st) {
    if (a.active) launch_level_wf<D, N, T, W, true>(op, a, colour, st);
    else launch_level_wf<D, N, T, W, false>(op, a, colour, st);
}

// trees with an operator: one tree, 256-thread workgroups (FP64 only; the
// FP32 instantiation launches nothing, the scheduler never asks for it)
template <int D, int N, typename T>
static void launch_level_op(Op op, const LevelArgs<T> &a, int colour, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        const int g = wg_count<D, N, 256>(a.nb);
        constexpr int OW = opw<D, N>();
        const int go = wg_count<D, N, OW>(a.nb);
        switch (op) {
        case Op::GSRB:
            // the row form on large 3D levels; small levels are
            // latency-bound, and there the staged box is faster (its LDS
            // reads do not wait behind the ghost selection): 3D levels of 8
            // to 512 boxes 5.6-6.0 against 7.3-7.6 us per launch, paper case
            // 2 (2D) 6.07-6.13 against 6.53-6.63 ms
            if constexpr (D == 3) {
                if (!(a.opk & OPK_GHOST_BIL) && a.nb > 1024) {
                    AFMG_LAUNCH((k_vgsrb_row<D, N, T, 256>), g, st, a, colour);
                    break;
                }
            }
            AFMG_LAUNCH_W((k_vgsrb<D, N, T>), go, OW, st, a, colour);
            break;
        case Op::RESID_RESTRICT: AFMG_LAUNCH_W((k_vresid_restrict<D, N, T>), go, OW, st, a); break;
        case Op::COARSE_RHS: AFMG_LAUNCH_W((k_vcoarse_rhs<D, N, T>), go, OW, st, a); break;
        case Op::PROLONG:
            if (a.opk & OPK_PROLONG_LIN) AFMG_LAUNCH_W((k_vprolong_lin<D, N, T>), go, OW, st, a);
            else if (a.opk & (OPK_PROLONG_EPS | OPK_GHOST_BIL)) AFMG_LAUNCH_W((k_vprolong<D, N, T>), go, OW, st, a);
            else AFMG_LAUNCH((k_prolong<D, N, T, 256, false>), g, st, a);
            break;
        case Op::RESTRICT_RHO:
            AFMG_LAUNCH((k_vrestrict<D, N, T>), g, st, a.info, a.rho, a.b0, a.nb, a.opk, a.bx, a.h);
            break;
        }
    }
}

template <int D, int N, typename T>
void launch_level(Op op, const LevelArgs<T> &a, int colour, int wg, hipStream_t st) {
    if (a.opk) {
        launch_level_op<D, N, T>(op, a, colour, st);
        return;
    }
    // workgroups of 64 or 128 threads where they hold whole boxes
    constexpr int TPB = Geo<D, N>::TPB;
    if constexpr (TPB <= 64)
        if (wg == 64) return launch_level_w<D, N, T, 64>(op, a, colour, st);
    if constexpr (TPB <= 128)
        if (wg == 128) return launch_level_w<D, N, T, 128>(op, a, colour, st);
    launch_level_w<D, N, T, 256>(op, a, colour, st);
}

template <int D, int N, typename T, int W>
static void launch_final_w(const LevelArgs<T> &a, double *partial, int64_t part0, double hD, float *rout,
                           hipStream_t st) {
    const int g = wg_count<D, N, W>(a.nb);
    if (a.active) AFMG_LAUNCH_W((k_final<D, N, T, W, true>), g, W, st, a, partial, part0, hD, rout);
    else AFMG_LAUNCH_W((k_final<D, N, T, W, false>), g, W, st, a, partial, part0, hD, rout);
}

template <int D, int N, typename T>
void launch_final(const LevelArgs<T> &a, double *partial, int64_t part0, double hD, float *rout, int wg,
                  hipStream_t st) {
    if (a.opk) {
        constexpr int OW = opw<D, N>();
        if constexpr (sizeof(T) == 8)
            AFMG_LAUNCH_W((k_vfinal<D, N, T>), (wg_count<D, N, OW>(a.nb)), OW, st, a, partial, part0, hD);
        return;
    }
    constexpr int TPB = Geo<D, N>::TPB;
    if constexpr (TPB <= 64)
        if (wg == 64) return launch_final_w<D, N, T, 64>(a, partial, part0, hD, rout, st);
    if constexpr (TPB <= 128)
        if (wg == 128) return launch_final_w<D, N, T, 128>(a, partial, part0, hD, rout, st);
    launch_final_w<D, N, T, 256>(a, partial, part0, hD, rout, st);
}

template <int D, int N>
void launch_ir_update(const BoxInfo *info, double *u, float *e, int64_t nb, const int *active,
                      hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_ir_update<D, N>), g, st, info, u, e, (int)nb, active);
}

template <int D, int N>
int final_wgs(int64_t nb, int wg) {
    constexpr int TPB = Geo<D, N>::TPB;
    if constexpr (TPB <= 64)
        if (wg == 64) return wg_count<D, N, 64>(nb);
    if constexpr (TPB <= 128)
        if (wg == 128) return wg_count<D, N, 128>(nb);
    return wg_count<D, N, 256>(nb);
}

#ifndef AFMG_INSTANTIATE_ONLY
void launch_reduce(const double *partial, int64_t n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partial, n, out, 1);
}

void launch_reduce_trees(const double *partial, const int64_t *ptr, const int32_t *boxes, const int *active,
                         double *out, int n_trees, hipStream_t st) {
    AFMG_LAUNCH(k_reduce_trees, n_trees, st, partial, ptr, boxes, active, out);
}

void launch_compact(const int *mask, const int64_t *ltoff, const int64_t *lvl_off, int n_trees, int lmax,
                    int32_t *act, int *nact, hipStream_t st) {
    AFMG_LAUNCH(k_compact, lmax, st, mask, ltoff, lvl_off, n_trees, act, nact);
}

void launch_tree_stop(const double *norm, int *mask, TreeStop *state, double *hist, int n_trees, double tol,
                      int fixed, int nmax, hipStream_t st) {
    const int g = (n_trees + 255) / 256;
    AFMG_LAUNCH(k_tree_stop, g, st, norm, mask, state, hist, n_trees, tol, fixed, nmax);
}

void launch_level_mask(const int *base, const int32_t *tree_lmax, int l, int *out, int n_trees, hipStream_t st) {
    const int g = (n_trees + 255) / 256;
    AFMG_LAUNCH(k_level_mask, g, st, base, tree_lmax, l, out, n_trees);
}
#endif  // AFMG_INSTANTIATE_ONLY

template <int D, int N, typename T>
void launch_coarse(const CoarseArgs<T> &a, int n_trees, hipStream_t st) {
    if (n_trees > 0) hipLaunchKernelGGL((k_coarse<D, N, T>), dim3(n_trees), dim3(COARSE_NT), 0, st, a);
}

template <int D, int N, typename T>
void launch_coarse_gen(const CoarseGenArgs<T> &a, hipStream_t st) {
    // up to 64 KB of dynamic LDS (a level-1 box with its chain: 27 KB in 3D
    // with 8^3 cells, 3.8 KB in 2D); on the 3D eps-jump solve 162 against
    // 192 us per call with the grids in global memory
    constexpr size_t LDS_GEN_MAX = 64 * 1024;
    const size_t bytes = sizeof(double) * coarse_gen_doubles<D, N>(a.n_roots, a.opk) +
                         (sizeof(BoxInfo) + sizeof(int32_t)) * (size_t)a.n_roots;
    CoarseGenArgs<T> b = a;
    b.in_lds = bytes <= LDS_GEN_MAX ? 1 : 0;
    hipLaunchKernelGGL((k_coarse_gen<D, N, T>), dim3(1), dim3(COARSE_NT), b.in_lds ? bytes : 0, st, b);
}
template <int D, int N>
void launch_restrict_field_op(const BoxInfo *info, double *f, int64_t b0, int64_t nb, int opk, const int32_t *bx,
                              double h, hipStream_t st) {
    AFMG_LAUNCH((k_vrestrict<D, N, double>), (wg_count<D, N>(nb)), st, info, f, b0, (int)nb, opk, bx, h);
}
template <int D, int N>
void launch_check_positive(const BoxInfo *info, const double *f, int64_t nb, int *flag, hipStream_t st) {
    AFMG_LAUNCH((k_check_positive<D, N>), (wg_count<D, N>(nb)), st, info, f, (int)nb, flag);
}

template <int D, int N>
void launch_box_flags(const BoxInfo *info, const int8_t *flags, int64_t nb, int n_buf, int32_t *words,
                      hipStream_t st) {
    AFMG_LAUNCH((k_box_flags<D, N>), (wg_count<D, N>(nb)), st, info, flags, (int)nb, n_buf, words);
}
template <int D, int N>
void launch_transfer(const BoxInfo *to_info, const BoxInfo *from_info, const int32_t *copy_dst,
                     const int32_t *copy_src, int64_t n_copy, const int32_t *pro_dst, const int32_t *pro_src,
                     int64_t n_pro, const double *from, const double *bc, int homog, double *to, hipStream_t st) {
    AFMG_LAUNCH((k_transfer_copy<D, N>), (wg_count<D, N>(n_copy)), st, copy_dst, copy_src, (int)n_copy, from, to);
    AFMG_LAUNCH((k_transfer_prolong<D, N>), (wg_count<D, N>(n_pro)), st, to_info, from_info, pro_dst, pro_src,
                (int)n_pro, from, bc, homog, to);
}

template <int D, int N>
size_t coarse_gen_doubles(int n_roots, int opk) {
    using GG = GenGeo<D, N>;
    return (size_t)n_roots * (5 * GG::TOT + GG::BTOT) + (opk ? (size_t)(2 * D + 1) * n_roots * GG::TOT : 0);
}

template <int D, int N, typename T>
void launch_permute(const BoxInfo *info, T *f, int64_t b0, int64_t nb, int to_split, int leaves_only,
                    hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_permute<D, N, T>), g, st, info, f, b0, (int)nb, to_split, leaves_only);
}

template <int D, int N, typename T>
void launch_load_rho(const BoxInfo *info, const int32_t *map, const T *src, T *dst, int64_t nb, int leaves_only,
                     hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_load_rho<D, N, T>), g, st, info, map, src, dst, (int)nb, leaves_only);
}

template <int D, int N, typename T>
void launch_store_boxes(const int32_t *map, const T *src, T *dst, int64_t nb, hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_store_boxes<D, N, T>), g, st, map, src, dst, (int)nb);
}

#ifndef AFMG_INSTANTIATE_ONLY
void launch_gather_rows(const int32_t *map, const double *src, double *dst, int64_t n_rows, int F,
                        hipStream_t st) {
    int64_t g = (n_rows * F + 255) / 256;
    if (g > 65536) g = 65536;
    AFMG_LAUNCH(k_gather_rows, (int)g, st, map, src, dst, n_rows, F);
}
#endif  // AFMG_INSTANTIATE_ONLY

template <int D, int N>
void launch_bc_derive(const BoxInfo *info, int64_t b0, int64_t nb, double *bc, hipStream_t st) {
    using G = Geo<D, N>;
    const int64_t work = nb * 2 * D * G::HF;
    const int g = (int)((work + 255) / 256);
    AFMG_LAUNCH((k_bc_derive<D, N>), g, st, info, b0, (int)nb, bc);
}

template <typename T>
void launch_copy(const T *src, T *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)g), dim3(256), 0, st, src, dst, n);
}
template <typename T>
void launch_fill(T *dst, int64_t n, T v, hipStream_t st) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)g), dim3(256), 0, st, dst, n, v);
}

template <int D, int N>
void launch_apply_lt(const BoxInfo *info, const int *child, const double *y, double *out, int64_t nb,
                     hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_apply_lt<D, N>), g, st, info, child, y, out, (int)nb);
}
template <int D, int N>
void launch_apply_l(const BoxInfo *info, const double *x, double *out, int64_t nb, hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_apply_l<D, N>), g, st, info, x, out, (int)nb);
}
template <int D, int N>
void launch_restrict_field(const BoxInfo *info, double *f, int64_t b0, int64_t nb, hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_restrict_field<D, N>), g, st, info, f, b0, (int)nb);
}
template <int D, int N>
void launch_push_down(const BoxInfo *info, double *f, int64_t b0, int64_t nb, hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_push_down<D, N>), g, st, info, f, b0, (int)nb);
}
template <int D, int N>
void launch_scale_leaves(const BoxInfo *info, double *dst, const double *src, int pw, int64_t nb, hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_scale_leaves<D, N>), g, st, info, dst, src, pw, (int)nb);
}
template <int D, int N>
void launch_store_leaves(const BoxInfo *info, const double *src, double *dst, int64_t nb, hipStream_t st) {
    const int g = wg_count<D, N>(nb);
    AFMG_LAUNCH((k_store_leaves<D, N>), g, st, info, src, dst, (int)nb);
}
template <int D, int N>
void launch_bc_grad(const BoxInfo *info, const double *lam, double *bc_bar, int64_t nb, hipStream_t st) {
    using G = Geo<D, N>;
    const int64_t work = nb * 2 * D * G::F;
    const int g = (int)((work + 255) / 256);
    AFMG_LAUNCH((k_bc_grad<D, N>), g, st, info, lam, bc_bar, (int)nb);
}
#ifndef AFMG_INSTANTIATE_ONLY
void launch_dot(const double *a, const double *b, int64_t n, double *partial, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot, dim3(DOT_WGS), dim3(256), 0, st, a, b, n, partial);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partial, (int64_t)DOT_WGS, out, 0);
}
void launch_lc3(double *out, double a, const double *x, double b, const double *y, double c, const double *z,
                int64_t n, hipStream_t st) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_lc3, dim3((unsigned)g), dim3(256), 0, st, out, a, x, b, y, c, z, n);
}
#endif  // AFMG_INSTANTIATE_ONLY

#define AFMG_ADJ_INST(D, N)                                                                          \
    template void launch_apply_lt<D, N>(const BoxInfo *, const int *, const double *, double *, int64_t, \
                                        hipStream_t);                                                \
    template void launch_apply_l<D, N>(const BoxInfo *, const double *, double *, int64_t, hipStream_t); \
    template void launch_restrict_field<D, N>(const BoxInfo *, double *, int64_t, int64_t, hipStream_t);   \
    template void launch_push_down<D, N>(const BoxInfo *, double *, int64_t, int64_t, hipStream_t);        \
    template void launch_scale_leaves<D, N>(const BoxInfo *, double *, const double *, int, int64_t,       \
                                            hipStream_t);                                             \
    template void launch_store_leaves<D, N>(const BoxInfo *, const double *, double *, int64_t,            \
                                            hipStream_t);                                             \
    template void launch_bc_grad<D, N>(const BoxInfo *, const double *, double *, int64_t, hipStream_t);

#define AFMG_INST(D, N, T)                                                                              \
    template void launch_level<D, N, T>(Op, const LevelArgs<T> &, int, int, hipStream_t);                \
    template void launch_final<D, N, T>(const LevelArgs<T> &, double *, int64_t, double, float *, int, \
                                        hipStream_t);                                                 \
    template void launch_coarse<D, N, T>(const CoarseArgs<T> &, int, hipStream_t);                      \
    template void launch_coarse_gen<D, N, T>(const CoarseGenArgs<T> &, hipStream_t);                     \
    template void launch_permute<D, N, T>(const BoxInfo *, T *, int64_t, int64_t, int, int, hipStream_t); \
    template void launch_load_rho<D, N, T>(const BoxInfo *, const int32_t *, const T *, T *, int64_t, int, \
                                           hipStream_t);                                              \
    template void launch_store_boxes<D, N, T>(const int32_t *, const T *, T *, int64_t, hipStream_t);

// every template the scheduler calls, for boxes of N^D cells
#define AFMG_BOX_INST(D, N)                                                                                   \
    AFMG_ADJ_INST(D, N)                                                                                       \
    AFMG_INST(D, N, double)                                                                                   \
    AFMG_INST(D, N, float)                                                                                    \
    template void launch_ir_update<D, N>(const BoxInfo *, double *, float *, int64_t, const int *, hipStream_t); \
    template size_t coarse_gen_doubles<D, N>(int, int);                                                             \
    template void launch_restrict_field_op<D, N>(const BoxInfo *, double *, int64_t, int64_t, int,             \
                                                 const int32_t *, double, hipStream_t);                        \
    template void launch_check_positive<D, N>(const BoxInfo *, const double *, int64_t, int *, hipStream_t);  \
    template void launch_box_flags<D, N>(const BoxInfo *, const int8_t *, int64_t, int, int32_t *, hipStream_t); \
    template void launch_transfer<D, N>(const BoxInfo *, const BoxInfo *, const int32_t *, const int32_t *,    \
                                        int64_t, const int32_t *, const int32_t *, int64_t, const double *,    \
                                        const double *, int, double *, hipStream_t);                           \
    template int final_wgs<D, N>(int64_t, int);                                                               \
    template void launch_bc_derive<D, N>(const BoxInfo *, int64_t, int64_t, double *, hipStream_t);

// Boxes of 8^D cells here; the boxes of 16^D cells are instantiated in a
// translation unit of their own (afmg_kernels_n16.hip), which includes this
// file with AFMG_INSTANTIATE_ONLY set.
#ifndef AFMG_INSTANTIATE_ONLY
AFMG_BOX_INST(2, 8)
AFMG_BOX_INST(3, 8)
template void launch_copy<float>(const float *, float *, int64_t, hipStream_t);
template void launch_fill<float>(float *, int64_t, float, hipStream_t);
template void launch_copy<double>(const double *, double *, int64_t, hipStream_t);
template void launch_fill<double>(double *, int64_t, double, hipStream_t);
template void launch_fill<int>(int *, int64_t, int, hipStream_t);

bool coarse_kernel_level2(int dim, int box_n) {
    if (dim == 3) return box_n == 8 ? coarse_l2_fits<3, 8>() : box_n == 16 ? coarse_l2_fits<3, 16>() : false;
    return box_n == 8 ? coarse_l2_fits<2, 8>() : box_n == 16 ? coarse_l2_fits<2, 16>() : false;
}
#endif  // AFMG_INSTANTIATE_ONLY

}  // namespace afmg
