/*
 * FP64 CPU oracle for the FAS multigrid Poisson solve on quadtree/octree box
 * grids (Teunissen & Ebert, "Afivo", §2-§3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  It shares no code with the GPU library,
 * and only tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.
 *
 * Data model (paper §2.1): every box holds n^D cells plus one stored ghost
 * layer, so each field of a box is an (n+2)^D array indexed 1..n in the
 * interior and 0 / n+1 in the ghost layer (1-based, as the paper numbers
 * cells).  Boxes of the tree have n = N.  The coarse grid (paper §2.2) is
 * one or more level-1 boxes on an integer lattice; below each of them extra
 * coarse grids of N/2, N/4, ..., 2 cells per side are added (paper §3.2,
 * V-cycle), linked like their level-1 boxes.  Each side orientation of the
 * domain is Dirichlet, Neumann or periodic (paper §3).
 *
 * Steps, each following the paper:
 *   fill_gc      side ghost cells: same-level copy, Dirichlet, or the default
 *                refinement-boundary scheme (paper §2.4 and §3.3)
 *   half_sweep   Gauss-Seidel red-black on one colour (paper §3.1)
 *   vcycle       the FAS V-cycle (paper §3.2, eqs. residual, coarse-rhs,
 *                coarse-corr)
 *   fmg          the FMG cycle without an initial guess (paper §3.2)
 *   restriction  averaging over the 2^D children (paper §2.5); in the
 *                cylindrical form the mean over the parent cell's volume
 *   prolongation 2-1-1 interpolation (paper §2.5)
 *   schemes      the refinement-boundary ghost of paper §3.3 (the default,
 *                from the two closest fine values) or its bilinear
 *                extrapolation variant; 2-1-1 or bi/trilinear prolongation
 *                (paper §2.5), the latter with edge and corner ghosts
 *                copied from a diagonal neighbour or extrapolated as
 *                b + c - a (paper §2.4)
 *   operators    the Laplacian, or div(eps grad u) with eps per cell and the
 *                harmonic mean of the two cells' eps on each face (paper
 *                §3.4), or the cylindrical (r, z) form of either (paper §3.5,
 *                §4.1 case 2); an eps-weighted prolongation (paper §3.5)
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - red cells are those whose 1-based global index sum is even;
 *   - side ghosts are refreshed before every half sweep;
 *   - a Dirichlet ghost is 2 b - u1 (linear through the face value b), a
 *     Neumann ghost u1 + h q (q the outward normal derivative at the face);
 *   - boundary values (Dirichlet or Neumann) of non-leaf boxes are the means
 *     of their children's face values;
 *   - the copy v'_H includes side ghosts filled right after restriction;
 *   - the stop test uses the max-norm of the composite leaf residual relative
 *     to that of the zero initial guess.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXLEV 40

typedef struct {
    int dim, N;
    int lmin, lmax;
    int nbox;
    int *lev, *ix, *iy, *iz, *n, *parent, *leaf;
    int *child;  /* [nbox*8], octant bits x | y<<1 | z<<2, -1 if none */
    int *nbr;    /* [nbox*6]: >=0 same-level box, -1 physical, -2 refinement boundary */
    int64_t *off;   /* offset of each box's padded array */
    int64_t *bcoff; /* [nbox*6] offset into bc store, -1 if side not physical */
    int64_t ntot, nbc;
    double *u, *rho, *uold, *res, *bc;
    int nleaf_in;
    int *leaf_box; /* box id of input leaf i */
    /* per level lists, level l stored at index l - lmin */
    int *lvl_first[OR_MAXLEV];
    int lvl_cnt[OR_MAXLEV];
    int *lvl_store;
    int bctype[6];  /* side type per orientation (OR_DIRICHLET, OR_NEUMANN, OR_PERIODIC) */
    int ext[3];     /* extent of the coarse-grid lattice (level-1 boxes) per axis */
    int nroot;      /* level-1 boxes */
    int opk;        /* operator: OR_OP_* bits, 0 for the Laplacian */
    double *eps;    /* eps per cell with ghosts (OR_OP_EPS), else NULL */
    int ghost_bil;  /* 1: bilinear-extrapolation refinement ghosts */
    int prolong_lin;/* 1: bi/trilinear prolongation (edge and corner ghosts filled) */
    int *dnbr;      /* [nbox*27]: same-level box across direction (dx,dy,dz), index
                       (dx+1) + 3 (dy+1) + 9 (dz+1), -1 if none */
} otree;

/* ------------------------------------------------------------------------ */
/* hash map (level, i, j, k) -> box id                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t *key;
    int *val;
    int64_t cap;
} ohash;

static uint64_t okey(int l, int i, int j, int k) {
    return ((uint64_t)(l + 8) << 57) | ((uint64_t)i << 38) | ((uint64_t)j << 19) | (uint64_t)k;
}
static uint64_t omix(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}
static int oh_init(ohash *h, int64_t n) {
    h->cap = 16;
    while (h->cap < 2 * n + 16) h->cap *= 2;
    h->key = (uint64_t *)malloc(sizeof(uint64_t) * h->cap);
    h->val = (int *)malloc(sizeof(int) * h->cap);
    if (!h->key || !h->val) return -1;
    for (int64_t i = 0; i < h->cap; i++) h->key[i] = 0;
    return 0;
}
static int oh_get(const ohash *h, uint64_t k) {
    int64_t p = (int64_t)(omix(k) & (uint64_t)(h->cap - 1));
    while (h->key[p]) {
        if (h->key[p] == k) return h->val[p];
        p = (p + 1) & (h->cap - 1);
    }
    return -1;
}
static int oh_put(ohash *h, uint64_t k, int v) { /* returns existing value or -1 when inserted */
    int64_t p = (int64_t)(omix(k) & (uint64_t)(h->cap - 1));
    while (h->key[p]) {
        if (h->key[p] == k) return h->val[p];
        p = (p + 1) & (h->cap - 1);
    }
    h->key[p] = k;
    h->val[p] = v;
    return -1;
}
static void oh_free(ohash *h) { free(h->key); free(h->val); }

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int or_np(const otree *t, int b) { return t->n[b] + 2; }
/* padded index, 1-based interior */
static int64_t PI(const otree *t, int b, int i, int j, int k) {
    int m = t->n[b] + 2;
    return t->off[b] + i + (int64_t)m * (j + (int64_t)m * k);
}
static double level_h(const otree *t, int l) { return 1.0 / ((double)t->N * ldexp(1.0, l - 1)); }
static int lvl_count(const otree *t, int l) { return t->lvl_cnt[l - t->lmin]; }
static int lvl_box(const otree *t, int l, int m) { return t->lvl_first[l - t->lmin][m]; }

/* offset (0-based, in parent cells) of box b inside its parent along axis d */
static int child_offset(const otree *t, int b, int d) {
    if (t->lev[b] <= 1) return 0; /* root and coarse grids cover their parent fully */
    int id = d == 0 ? t->ix[b] : (d == 1 ? t->iy[b] : t->iz[b]);
    return ((id - 1) & 1) * (t->n[b] / 2);
}

static char or_errbuf[512];
static void seterr(char *err, int errlen, const char *msg) {
    snprintf(or_errbuf, sizeof(or_errbuf), "%s", msg);
    if (err && errlen > 0) snprintf(err, (size_t)errlen, "%s", msg);
}

/* ------------------------------------------------------------------------ */
/* tree construction from a leaf list                                        */
/* ------------------------------------------------------------------------ */
void or_tree_free(void *p);

/* Side types of the domain boundary (paper §3: Dirichlet, Neumann or
   periodic, or a mix), one per side orientation -x, +x, -y, +y, -z, +z. */
#define OR_DIRICHLET 0
#define OR_NEUMANN 1
#define OR_PERIODIC 2

/* The coarse grid (paper §2.2) is the set of level-1 boxes that contain
   leaves: boxes of unit size at 1-based lattice positions 1..ext[d] along
   each axis, which may leave out positions (an L-shaped domain).  Each root
   box gets its own chain of extra coarse grids of N/2, ..., 2 cells per side
   below level 1 (paper §3.2), linked to the chains of its neighbouring roots,
   so a domain of several roots has several 2^D-cell boxes on its coarsest
   level.  A periodic axis wraps the neighbour search around the lattice and
   needs a rectangular coarse grid. */
void *or_tree_new_bc(int dim, int N, const int32_t *bctype, int64_t n_leaves, const int32_t *level,
                     const int32_t *idx, char *err, int errlen) {
    if (dim != 2 && dim != 3) { seterr(err, errlen, "dim must be 2 or 3"); return NULL; }
    if (N < 2 || (N & (N - 1))) { seterr(err, errlen, "N must be a power of two >= 2"); return NULL; }
    if (n_leaves <= 0) { seterr(err, errlen, "no leaves"); return NULL; }
    int bct[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < 2 * dim; s++) {
        bct[s] = bctype ? bctype[s] : OR_DIRICHLET;
        if (bct[s] < OR_DIRICHLET || bct[s] > OR_PERIODIC) { seterr(err, errlen, "bad side type"); return NULL; }
    }
    for (int d = 0; d < dim; d++)
        if ((bct[2 * d] == OR_PERIODIC) != (bct[2 * d + 1] == OR_PERIODIC)) {
            seterr(err, errlen, "periodic sides come in pairs"); return NULL;
        }
    int lg = 0;
    while ((2 << lg) < N) lg++; /* N = 2^(lg+1) */
    otree *t = (otree *)calloc(1, sizeof(otree));
    t->dim = dim;
    t->N = N;
    t->lmin = 1 - lg;
    t->lmax = 1;
    for (int s = 0; s < 6; s++) t->bctype[s] = bct[s];
    t->ext[0] = t->ext[1] = t->ext[2] = 1;
    for (int64_t q = 0; q < n_leaves; q++) {
        int l = level[q], c[3] = {idx[3 * q], idx[3 * q + 1], dim == 3 ? idx[3 * q + 2] : 1};
        if (l < 1 || l > 18) { seterr(err, errlen, "leaf level out of range [1,18]"); free(t); return NULL; }
        for (int d = 0; d < 3; d++) {
            if (c[d] < 1 || c[d] >= (1 << 19) || (d == 2 && dim == 2 && c[d] != 1)) {
                seterr(err, errlen, "leaf spatial index out of range"); free(t); return NULL;
            }
            int r = ((c[d] - 1) >> (l - 1)) + 1;
            if (r > t->ext[d]) t->ext[d] = r;
        }
    }
    if ((int64_t)t->ext[0] * t->ext[1] * t->ext[2] > 4096) {
        seterr(err, errlen, "coarse grid larger than 4096 boxes"); free(t); return NULL;
    }
    ohash h;
    int64_t cap = n_leaves * 2 + 64;
    if (oh_init(&h, cap) != 0) { free(t); seterr(err, errlen, "out of memory"); return NULL; }
    /* provisional arrays */
    int *L = (int *)malloc(sizeof(int) * cap), *I = (int *)malloc(sizeof(int) * cap),
        *J = (int *)malloc(sizeof(int) * cap), *K = (int *)malloc(sizeof(int) * cap),
        *isleaf = (int *)malloc(sizeof(int) * cap);
    int nb = 0;
    for (int64_t q = 0; q < n_leaves; q++) {
        int l = level[q], i = idx[3 * q], j = idx[3 * q + 1], k = dim == 3 ? idx[3 * q + 2] : 1;
        if (oh_put(&h, okey(l, i, j, k), nb) >= 0) { seterr(err, errlen, "duplicate leaf"); goto fail; }
        L[nb] = l; I[nb] = i; J[nb] = j; K[nb] = k; isleaf[nb] = 1;
        nb++;
        if (l > t->lmax) t->lmax = l;
    }
    /* ancestors */
    for (int q = 0; q < (int)n_leaves; q++) {
        int l = L[q], i = I[q], j = J[q], k = K[q];
        while (l > 1) {
            l--; i = (i + 1) / 2; j = (j + 1) / 2; k = dim == 3 ? (k + 1) / 2 : 1;
            if (nb >= cap) {
                cap *= 2;
                L = realloc(L, sizeof(int) * cap); I = realloc(I, sizeof(int) * cap);
                J = realloc(J, sizeof(int) * cap); K = realloc(K, sizeof(int) * cap);
                isleaf = realloc(isleaf, sizeof(int) * cap);
                ohash h2; oh_init(&h2, cap);
                for (int64_t p = 0; p < h.cap; p++) if (h.key[p]) oh_put(&h2, h.key[p], h.val[p]);
                oh_free(&h); h = h2;
            }
            int ex = oh_put(&h, okey(l, i, j, k), nb);
            if (ex >= 0) {
                if (isleaf[ex]) { seterr(err, errlen, "a leaf overlaps a finer leaf"); goto fail; }
                break;
            }
            L[nb] = l; I[nb] = i; J[nb] = j; K[nb] = k; isleaf[nb] = 0;
            nb++;
        }
    }
    /* the roots: level-1 boxes, in provisional order */
    int nroot = 0;
    for (int q = 0; q < nb; q++) if (L[q] == 1) nroot++;
    t->nroot = nroot;
    int periodic_any = 0;
    for (int d = 0; d < dim; d++) periodic_any |= bct[2 * d] == OR_PERIODIC;
    if (periodic_any && nroot != t->ext[0] * t->ext[1] * (dim == 3 ? t->ext[2] : 1)) {
        seterr(err, errlen, "periodic sides need a rectangular coarse grid"); goto fail;
    }
    /* final numbering: coarse grids first (levels lmin..0, nroot boxes each,
       box (l, r) at (l - lmin) * nroot + r), then the tree boxes level by
       level in provisional order, so root r is box ncoarse + r */
    int ncoarse = (1 - t->lmin) * nroot;
    t->nbox = nb + ncoarse;
    int B = t->nbox;
    t->lev = malloc(sizeof(int) * B); t->ix = malloc(sizeof(int) * B); t->iy = malloc(sizeof(int) * B);
    t->iz = malloc(sizeof(int) * B); t->n = malloc(sizeof(int) * B); t->parent = malloc(sizeof(int) * B);
    t->leaf = malloc(sizeof(int) * B); t->child = malloc(sizeof(int) * B * 8);
    t->nbr = malloc(sizeof(int) * B * 6); t->off = malloc(sizeof(int64_t) * B);
    t->dnbr = malloc(sizeof(int) * B * 27);
    t->bcoff = malloc(sizeof(int64_t) * B * 6);
    int *newid = malloc(sizeof(int) * nb);
    int pos = ncoarse;
    for (int l = 1; l <= t->lmax; l++)
        for (int q = 0; q < nb; q++)
            if (L[q] == l) {
                newid[q] = pos;
                t->lev[pos] = l; t->ix[pos] = I[q]; t->iy[pos] = J[q]; t->iz[pos] = K[q];
                t->n[pos] = N; t->leaf[pos] = isleaf[q];
                pos++;
            }
    for (int l = t->lmin; l <= 0; l++)
        for (int r = 0; r < nroot; r++) {
            int b = (l - t->lmin) * nroot + r, R = ncoarse + r;
            t->lev[b] = l; t->ix[b] = t->ix[R]; t->iy[b] = t->iy[R]; t->iz[b] = t->iz[R];
            t->n[b] = N >> (1 - l); t->leaf[b] = 0;
        }
    for (int64_t p = 0; p < h.cap; p++) if (h.key[p]) h.val[p] = newid[h.val[p]];
    t->nleaf_in = (int)n_leaves;
    t->leaf_box = malloc(sizeof(int) * n_leaves);
    for (int q = 0; q < (int)n_leaves; q++) t->leaf_box[q] = newid[q];
    free(newid);
    /* parents / children */
    int nch = 1 << dim;
    for (int b = 0; b < B; b++) {
        for (int c = 0; c < 8; c++) t->child[8 * b + c] = -1;
        t->parent[b] = -1;
    }
    for (int b = 0; b < B; b++) {
        int l = t->lev[b];
        if (l <= 1) {
            /* chain of root r: (l - 1, r) is the parent of (l, r), and the
               coarse box covers its only child completely */
            int r = l == 1 ? b - ncoarse : b % nroot;
            t->parent[b] = l > t->lmin ? (l - 1 - t->lmin) * nroot + r : -1;
            if (t->parent[b] >= 0) t->child[8 * t->parent[b]] = b;
            continue;
        }
        int pi = (t->ix[b] + 1) / 2, pj = (t->iy[b] + 1) / 2, pk = dim == 3 ? (t->iz[b] + 1) / 2 : 1;
        int p = oh_get(&h, okey(l - 1, pi, pj, pk));
        t->parent[b] = p;
        int oc = ((t->ix[b] - 1) & 1) | (((t->iy[b] - 1) & 1) << 1) | (dim == 3 ? (((t->iz[b] - 1) & 1) << 2) : 0);
        t->child[8 * p + oc] = b;
    }
    for (int b = 0; b < B; b++) {
        if (t->lev[b] < 1 || t->leaf[b]) continue;
        for (int c = 0; c < nch; c++)
            if (t->child[8 * b + c] < 0) { seterr(err, errlen, "leaves do not tile the domain (missing child)"); goto fail2; }
    }
    /* neighbours of the tree boxes: same-level box, physical side (-1:
       outside the lattice on a non-periodic axis, or a lattice position
       without a root), or refinement boundary (-2) */
    for (int b = ncoarse; b < B; b++) {
        int l = t->lev[b];
        for (int s = 0; s < 6; s++) t->nbr[6 * b + s] = -1;
        for (int s = 0; s < 2 * dim; s++) {
            int d = s / 2, dir = (s % 2) ? 1 : -1;
            int q[3] = {t->ix[b], t->iy[b], t->iz[b]};
            int n1 = t->ext[d] << (l - 1);
            q[d] += dir;
            if (q[d] < 1 || q[d] > n1) {
                if (bct[s] != OR_PERIODIC) continue;
                q[d] = q[d] < 1 ? n1 : 1;
            }
            int nb2 = oh_get(&h, okey(l, q[0], q[1], q[2]));
            if (nb2 >= 0) { t->nbr[6 * b + s] = nb2; continue; }
            int rq[3] = {((q[0] - 1) >> (l - 1)) + 1, ((q[1] - 1) >> (l - 1)) + 1,
                         dim == 3 ? ((q[2] - 1) >> (l - 1)) + 1 : 1};
            if (oh_get(&h, okey(1, rq[0], rq[1], rq[2])) < 0) continue; /* a hole in the coarse grid */
            t->nbr[6 * b + s] = -2;
            /* 2:1 balance: the parent's neighbour must exist */
            int p = t->parent[b];
            int pq[3] = {t->ix[p], t->iy[p], t->iz[p]};
            int n0 = t->ext[d] << (l - 2);
            pq[d] += dir;
            if (pq[d] < 1 || pq[d] > n0) pq[d] = pq[d] < 1 ? n0 : 1; /* periodic here */
            if (oh_get(&h, okey(l - 1, pq[0], pq[1], pq[2])) < 0) {
                seterr(err, errlen, "grid violates 2:1 balance across a box side"); goto fail2;
            }
        }
    }
    /* same-level boxes across every direction (sides, edges, corners;
       periodic axes wrapped), for edge and corner ghosts */
    for (int b = ncoarse; b < B; b++) {
        int l = t->lev[b];
        for (int o = 0; o < 27; o++) {
            int dd[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
            t->dnbr[27 * b + o] = -1;
            if (dim == 2 && dd[2] != 0) continue;
            int q[3] = {t->ix[b] + dd[0], t->iy[b] + dd[1], t->iz[b] + dd[2]}, inside = 1;
            for (int d = 0; d < dim; d++) {
                int n1 = t->ext[d] << (l - 1);
                if (q[d] < 1 || q[d] > n1) {
                    if (bct[2 * d] != OR_PERIODIC) inside = 0;
                    else q[d] = q[d] < 1 ? n1 : 1;
                }
            }
            if (inside) t->dnbr[27 * b + o] = oh_get(&h, okey(l, q[0], q[1], q[2]));
        }
    }
    /* neighbours on the coarse grids below level 1 mirror those of the roots */
    for (int b = 0; b < ncoarse; b++) {
        int r = b % nroot, l = t->lev[b];
        for (int s = 0; s < 6; s++) {
            int v = t->nbr[6 * (ncoarse + r) + s];
            t->nbr[6 * b + s] = v >= 0 ? (l - t->lmin) * nroot + (v - ncoarse) : -1;
        }
        for (int o = 0; o < 27; o++) {
            int v = t->dnbr[27 * (ncoarse + r) + o];
            t->dnbr[27 * b + o] = v >= 0 ? (l - t->lmin) * nroot + (v - ncoarse) : -1;
        }
    }
    /* level lists */
    t->lvl_store = malloc(sizeof(int) * B);
    pos = 0;
    for (int l = t->lmin; l <= t->lmax; l++) {
        t->lvl_first[l - t->lmin] = t->lvl_store + pos;
        int c = 0;
        for (int b = 0; b < B; b++) if (t->lev[b] == l) t->lvl_store[pos + c++] = b;
        t->lvl_cnt[l - t->lmin] = c;
        pos += c;
    }
    /* storage */
    int64_t o = 0;
    for (int b = 0; b < B; b++) {
        t->off[b] = o;
        int64_t m = t->n[b] + 2;
        o += dim == 3 ? m * m * m : m * m;
    }
    t->ntot = o;
    int64_t ob = 0;
    for (int b = 0; b < B; b++)
        for (int s = 0; s < 6; s++) {
            t->bcoff[6 * b + s] = -1;
            if (s < 2 * dim && t->nbr[6 * b + s] == -1) {
                t->bcoff[6 * b + s] = ob;
                ob += dim == 3 ? (int64_t)t->n[b] * t->n[b] : t->n[b];
            }
        }
    t->nbc = ob;
    t->u = calloc(o, sizeof(double)); t->rho = calloc(o, sizeof(double));
    t->uold = calloc(o, sizeof(double)); t->res = calloc(o, sizeof(double));
    t->bc = calloc(ob > 0 ? ob : 1, sizeof(double));
    free(L); free(I); free(J); free(K); free(isleaf); oh_free(&h);
    return t;
fail2:
    free(L); free(I); free(J); free(K); free(isleaf); oh_free(&h);
    or_tree_free(t);
    return NULL;
fail:
    free(L); free(I); free(J); free(K); free(isleaf); oh_free(&h); free(t);
    return NULL;
}

/* one root box on [0,1]^D with Dirichlet sides */
void *or_tree_new(int dim, int N, int64_t n_leaves, const int32_t *level, const int32_t *idx,
                  char *err, int errlen) {
    for (int64_t q = 0; q < n_leaves; q++) {
        int l = level[q], n1 = (l >= 1 && l <= 18) ? 1 << (l - 1) : 0;
        for (int d = 0; d < dim; d++)
            if (idx[3 * q + d] > n1) { seterr(err, errlen, "leaf spatial index out of range"); return NULL; }
    }
    return or_tree_new_bc(dim, N, NULL, n_leaves, level, idx, err, errlen);
}

void or_tree_free(void *p) {
    otree *t = (otree *)p;
    if (!t) return;
    free(t->lev); free(t->ix); free(t->iy); free(t->iz); free(t->n); free(t->parent);
    free(t->leaf); free(t->child); free(t->nbr); free(t->off); free(t->bcoff); free(t->dnbr);
    free(t->leaf_box); free(t->lvl_store);
    free(t->u); free(t->rho); free(t->uold); free(t->res); free(t->bc); free(t->eps);
    free(t);
}

const char *or_last_error(void) { return or_errbuf; }

/* info: [nbox, lmin, lmax, n_leaf_in, dim, N, nroot, ext0, ext1, ext2] */
void or_tree_info(void *p, int64_t *out) {
    otree *t = (otree *)p;
    out[0] = t->nbox; out[1] = t->lmin; out[2] = t->lmax; out[3] = t->nleaf_in;
    out[4] = t->dim; out[5] = t->N; out[6] = t->nroot;
    out[7] = t->ext[0]; out[8] = t->ext[1]; out[9] = t->ext[2];
}

/* per box: [level, ix, iy, iz, n, parent, leaf, nbr0..nbr5] */
void or_box_info(void *p, int b, int32_t *out) {
    otree *t = (otree *)p;
    out[0] = t->lev[b]; out[1] = t->ix[b]; out[2] = t->iy[b]; out[3] = t->iz[b];
    out[4] = t->n[b]; out[5] = t->parent[b]; out[6] = t->leaf[b];
    for (int s = 0; s < 6; s++) out[7 + s] = t->nbr[6 * b + s];
}

void or_leaf_boxes(void *p, int32_t *out) {
    otree *t = (otree *)p;
    for (int q = 0; q < t->nleaf_in; q++) out[q] = t->leaf_box[q];
}

/* ------------------------------------------------------------------------ */
/* field access helpers                                                      */
/* ------------------------------------------------------------------------ */
static double *fld(otree *t, int which) {
    switch (which) {
    case 0: return t->u;
    case 1: return t->rho;
    case 2: return t->uold;
    case 4: return t->eps;
    default: return t->res;
    }
}

/* Loop over the interior cells of box b, 1-based (i, j, k); k == 1 in 2D. */
#define FOR_CELLS(t, b, i, j, k)                                  \
    for (int k = 1; k <= ((t)->dim == 3 ? (t)->n[b] : 1); k++)      \
        for (int j = 1; j <= (t)->n[b]; j++)                        \
            for (int i = 1; i <= (t)->n[b]; i++)
/* padded index allowing k = 1 in 2D */
static int64_t PX(const otree *t, int b, int i, int j, int k) {
    return t->dim == 3 ? PI(t, b, i, j, k) : PI(t, b, i, j, 0);
}

/* copy interior of leaf-ordered input array into field */
static void load_leaf_field(otree *t, double *f, const double *src) {
    int N = t->N, D = t->dim;
    int64_t nc = D == 3 ? (int64_t)N * N * N : (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int q = 0; q < t->nleaf_in; q++) {
        int b = t->leaf_box[q];
        const double *s = src + nc * q;
        int64_t m = 0;
        FOR_CELLS(t, b, i, j, k) f[PX(t, b, i, j, k)] = s[m++];
    }
}
static void store_leaf_field(otree *t, const double *f, double *dst) {
    int N = t->N, D = t->dim;
    int64_t nc = D == 3 ? (int64_t)N * N * N : (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int q = 0; q < t->nleaf_in; q++) {
        int b = t->leaf_box[q];
        double *s = dst + nc * q;
        int64_t m = 0;
        FOR_CELLS(t, b, i, j, k) s[m++] = f[PX(t, b, i, j, k)];
    }
}

/* ------------------------------------------------------------------------ */
/* boundary values                                                           */
/* ------------------------------------------------------------------------ */
/* bc layout of the input: [n_leaves][2D][N^(D-1)], tangential axes in
   increasing order, first fastest.  Values of non-leaf boxes are the means
   of the 2^(D-1) child face values that cover each coarse face. */
static void set_bc(otree *t, const double *bc_leaf) {
    int N = t->N, D = t->dim;
    int64_t nf = D == 3 ? (int64_t)N * N : N;
    for (int64_t i = 0; i < t->nbc; i++) t->bc[i] = 0.0;
    for (int q = 0; q < t->nleaf_in; q++) {
        int b = t->leaf_box[q];
        for (int s = 0; s < 2 * D; s++) {
            int64_t o = t->bcoff[6 * b + s];
            if (o < 0) continue;
            for (int64_t m = 0; m < nf; m++) t->bc[o + m] = bc_leaf[(q * 2 * D + s) * nf + m];
        }
    }
    /* from fine to coarse */
    for (int l = t->lmax - 1; l >= t->lmin; l--) {
        for (int m = 0; m < lvl_count(t, l); m++) {
            int b = lvl_box(t, l, m);
            if (t->leaf[b]) continue;
            int n = t->n[b];
            for (int s = 0; s < 2 * D; s++) {
                int64_t o = t->bcoff[6 * b + s];
                if (o < 0) continue;
                int d = s / 2, hi = s % 2;
                int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2; /* tangential axes */
                int na = n, nc2 = D == 3 ? n : 1;
                for (int c = 0; c < nc2; c++)
                    for (int a = 0; a < na; a++) {
                        /* find the child box covering coarse face cell (a, c) */
                        double sum = 0.0;
                        int cnt = 0;
                        for (int oc = 0; oc < 8; oc++) {
                            int ch = t->child[8 * b + oc];
                            if (ch < 0) continue;
                            int bits[3] = {oc & 1, (oc >> 1) & 1, (oc >> 2) & 1};
                            if (t->lev[ch] >= 2 && bits[d] != hi) continue;
                            int nc_ = t->n[ch];
                            int offa = child_offset(t, ch, t1), offc = D == 3 ? child_offset(t, ch, t2) : 0;
                            if (a < offa || a >= offa + nc_ / 2) continue;
                            if (D == 3 && (c < offc || c >= offc + nc_ / 2)) continue;
                            int64_t oc_ = t->bcoff[6 * ch + s];
                            int fa = 2 * (a - offa), fc = 2 * (c - offc);
                            int nc3 = D == 3 ? 2 : 1;
                            for (int dc = 0; dc < nc3; dc++)
                                for (int da = 0; da < 2; da++) {
                                    sum += t->bc[oc_ + (fa + da) + (int64_t)nc_ * (fc + dc)];
                                    cnt++;
                                }
                        }
                        t->bc[o + a + (int64_t)n * c] = sum / cnt;
                    }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* ghost cells (paper §2.4, §3.3)                                            */
/* ------------------------------------------------------------------------ */
/* Edge (3D) and corner ghosts of every box at level l (paper §2.4): copied
   from the same-level box across that edge or corner when there is one,
   otherwise extrapolated linearly from the box's own side ghosts and cells:
   an edge or 2D corner ghost is b + c - a (b, c: the two values that share
   it with the inner cell a), a 3D corner ghost is the sum of its three
   edge ghosts minus its three side ghosts plus the inner cell (the same
   linear extrapolation applied along all three axes).  Side ghosts must be
   filled; edges are filled before corners. */
static void fill_gc_corners(otree *t, int l, double *f) {
    int D = t->dim;
    for (int pass = 2; pass <= D; pass++) /* edges (2 axes outside), then corners */
        for (int m = 0; m < lvl_count(t, l); m++) {
            int b = lvl_box(t, l, m), n = t->n[b];
            for (int o = 0; o < 27; o++) {
                int dd[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
                if (D == 2 && dd[2] != 0) continue;
                int nout = (dd[0] != 0) + (dd[1] != 0) + (dd[2] != 0);
                if (nout != pass) continue;
                int v = t->dnbr[27 * b + o];
                int lo[3], hi[3];
                for (int d = 0; d < 3; d++) {
                    if (d >= D) { lo[d] = hi[d] = 1; continue; }
                    lo[d] = dd[d] == -1 ? 0 : dd[d] == 1 ? n + 1 : 1;
                    hi[d] = dd[d] == -1 ? 0 : dd[d] == 1 ? n + 1 : n;
                }
                for (int k = lo[2]; k <= hi[2]; k++)
                    for (int j = lo[1]; j <= hi[1]; j++)
                        for (int i = lo[0]; i <= hi[0]; i++) {
                            int g[3] = {i, j, k};
                            double val;
                            if (v >= 0) {
                                int q[3] = {i, j, k};
                                for (int d = 0; d < D; d++)
                                    if (dd[d] != 0) q[d] = dd[d] == -1 ? n : 1;
                                val = f[PX(t, v, q[0], q[1], q[2])];
                            } else {
                                /* inclusion-exclusion over the outside axes:
                                   each value with a subset of them moved one
                                   cell inward, sign (-1)^(size of subset + 1) */
                                val = 0.0;
                                int ax[3], na = 0;
                                for (int d = 0; d < D; d++)
                                    if (dd[d] != 0) ax[na++] = d;
                                for (int sub = 1; sub < (1 << na); sub++) {
                                    int q[3] = {g[0], g[1], g[2]}, cnt = 0;
                                    for (int a = 0; a < na; a++)
                                        if (sub & (1 << a)) {
                                            q[ax[a]] += dd[ax[a]] == -1 ? 1 : -1;
                                            cnt++;
                                        }
                                    double w = (cnt % 2) ? 1.0 : -1.0;
                                    val += w * f[PX(t, b, q[0], q[1], q[2])];
                                }
                            }
                            f[PX(t, b, g[0], g[1], g[2])] = val;
                        }
            }
        }
}

/* Fill the side ghosts of every box at level l for field f.  homog != 0
   uses zero Dirichlet values. */
static void fill_gc(otree *t, int l, double *f, int homog) {
    int D = t->dim;
#pragma omp parallel for schedule(dynamic, 16)
    for (int m = 0; m < lvl_count(t, l); m++) {
        int b = lvl_box(t, l, m);
        int n = t->n[b];
        for (int s = 0; s < 2 * D; s++) {
            int d = s / 2, hi = s % 2;
            int nb = t->nbr[6 * b + s];
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            int nc2 = D == 3 ? n : 1;
            for (int c = 1; c <= nc2; c++)
                for (int a = 1; a <= n; a++) {
                    /* ghost position g, face cell c1, inner cell c2 (1-based) */
                    int g[3], c1[3], c2[3];
                    g[t1] = c1[t1] = c2[t1] = a;
                    g[t2] = c1[t2] = c2[t2] = (D == 3 ? c : 1);
                    g[d] = hi ? n + 1 : 0;
                    c1[d] = hi ? n : 1;
                    c2[d] = hi ? n - 1 : 2;
                    int64_t ig = PX(t, b, g[0], g[1], g[2]);
                    double u1 = f[PX(t, b, c1[0], c1[1], c1[2])];
                    if (nb >= 0) {
                        int q[3] = {c1[0], c1[1], c1[2]};
                        q[d] = hi ? 1 : n;
                        f[ig] = f[PX(t, nb, q[0], q[1], q[2])];
                    } else if (nb == -1) {
                        double bv = homog ? 0.0 : t->bc[t->bcoff[6 * b + s] + (a - 1) + (int64_t)n * ((D == 3 ? c : 1) - 1)];
                        if (t->bctype[s] == OR_NEUMANN)
                            f[ig] = u1 + level_h(t, t->lev[b]) * bv; /* outward derivative bv across the face */
                        else
                            f[ig] = 2.0 * bv - u1;                  /* value bv at the face */
                    } else {
                        /* refinement boundary: coarse value from the parent's neighbour */
                        int p = t->parent[b];
                        int cb = t->nbr[6 * p + s];
                        int qc[3];
                        qc[d] = hi ? 1 : n;
                        qc[t1] = child_offset(t, b, t1) + (a + 1) / 2;
                        qc[t2] = D == 3 ? child_offset(t, b, t2) + (c + 1) / 2 : 1;
                        double uH = f[PX(t, cb, qc[0], qc[1], qc[2])];
                        double u2 = f[PX(t, b, c2[0], c2[1], c2[2])];
                        int p1[3] = {c1[0], c1[1], c1[2]};
                        p1[t1] = (a % 2) ? a + 1 : a - 1; /* partner inside the same coarse cell */
                        double u1p = f[PX(t, b, p1[0], p1[1], p1[2])];
                        int q1[3] = {c2[0], c2[1], c2[2]};
                        q1[t1] = p1[t1];
                        double u2p = f[PX(t, b, q1[0], q1[1], q1[2])]; /* partner of u2 */
                        if (D == 2) {
                            if (t->ghost_bil) /* bilinear extrapolation (paper §3.3) */
                                f[ig] = 0.5 * uH + 1.125 * u1 - 0.375 * (u1p + u2) + 0.125 * u2p;
                            else
                                f[ig] = 0.5 * uH + u1 - 0.25 * (u1p + u2);
                        } else {
                            int p2[3] = {c1[0], c1[1], c1[2]};
                            p2[t2] = (c % 2) ? c + 1 : c - 1;
                            double u1pp = f[PX(t, b, p2[0], p2[1], p2[2])];
                            if (t->ghost_bil) {
                                /* trilinear extrapolation: the 2D scheme's
                                   construction with one more tangential axis */
                                int p3[3] = {p1[0], p1[1], p1[2]};
                                p3[t2] = p2[t2];
                                int q2[3] = {c2[0], c2[1], c2[2]}, q3[3] = {c2[0], c2[1], c2[2]};
                                q2[t2] = p2[t2];
                                q3[t1] = p1[t1];
                                q3[t2] = p2[t2];
                                double u1ppp = f[PX(t, b, p3[0], p3[1], p3[2])];
                                double u2pp = f[PX(t, b, q2[0], q2[1], q2[2])];
                                double u2ppp = f[PX(t, b, q3[0], q3[1], q3[2])];
                                f[ig] = 0.5 * uH + (27.0 / 16.0) * u1 - (9.0 / 16.0) * (u2 + u1p + u1pp) +
                                        (3.0 / 16.0) * (u2p + u2pp + u1ppp) - (1.0 / 16.0) * u2ppp;
                            } else {
                                f[ig] = 0.5 * uH + 1.25 * u1 - 0.25 * (u2 + u1p + u1pp);
                            }
                        }
                    }
                }
        }
    }
    if (t->prolong_lin) fill_gc_corners(t, l, f);
}

/* sum of the 2D side neighbours of cell (i,j,k) (ghosts included) */
static double nb_sum(const otree *t, const double *f, int b, int i, int j, int k) {
    if (t->dim == 2)
        return (f[PX(t, b, i - 1, j, k)] + f[PX(t, b, i + 1, j, k)]) +
               (f[PX(t, b, i, j - 1, k)] + f[PX(t, b, i, j + 1, k)]);
    return (f[PI(t, b, i - 1, j, k)] + f[PI(t, b, i + 1, j, k)]) +
           (f[PI(t, b, i, j - 1, k)] + f[PI(t, b, i, j + 1, k)]) +
           (f[PI(t, b, i, j, k - 1)] + f[PI(t, b, i, j, k + 1)]);
}

/* ------------------------------------------------------------------------ */
/* operators (paper §3.4, §3.5)                                              */
/* ------------------------------------------------------------------------ */
/* With an operator set, the equation of a cell is
     (1/h^2) sum over its 2D sides of w_s (u_s - u_c) = rho_c
   where u_s is the value across side s (neighbour or ghost, as for the
   Laplacian) and w_s the face coefficient:
     OR_OP_EPS: 2 eps_c eps_s / (eps_c + eps_s), eps_s the eps of the cell
                across the side (a ghost of eps, see fill_eps_gc);
     OR_OP_CYL: the radial sides (x is r) also carry r_face / r_c, from the
                finite-volume form of (1/r) d/dr (r eps du/dr); the face on
                the axis (r = 0) has w = 0.
   With every w_s = 1 this is the Laplacian. */
#define OR_OP_EPS 1
#define OR_OP_CYL 2
#define OR_OP_PROLONG_EPS 4

static double face_coef(const otree *t, int b, int i, int j, int k, int s) {
    double w = 1.0;
    if (t->opk & OR_OP_EPS) {
        int d = s / 2, hi = s % 2;
        int q[3] = {i, j, k};
        q[d] += hi ? 1 : -1;
        double ec = t->eps[PX(t, b, i, j, k)], en = t->eps[PX(t, b, q[0], q[1], q[2])];
        w = 2.0 * ec * en / (ec + en);
    }
    if ((t->opk & OR_OP_CYL) && s < 2) {
        double h = level_h(t, t->lev[b]);
        double x0 = (double)(t->ix[b] - 1) * t->n[b] * h; /* left edge of the box */
        double rc = x0 + (i - 0.5) * h;
        double rf = x0 + (s == 1 ? i : i - 1) * h;
        w *= rf / rc;
    }
    return w;
}

/* sum over the 2D sides of w_s f_s, and in *diag the sum of the w_s */
static double op_sum(const otree *t, const double *f, int b, int i, int j, int k, double *diag) {
    double sum = 0.0, dg = 0.0;
    for (int s = 0; s < 2 * t->dim; s++) {
        int d = s / 2, hi = s % 2;
        int q[3] = {i, j, k};
        q[d] += hi ? 1 : -1;
        double w = face_coef(t, b, i, j, k, s);
        sum += w * f[PX(t, b, q[0], q[1], q[2])];
        dg += w;
    }
    *diag = dg;
    return sum;
}

/* (L f)_c * h^2 on cell (i, j, k) of box b (ghosts filled) */
static double op_h2(const otree *t, const double *f, int b, int i, int j, int k) {
    if (!t->opk) return nb_sum(t, f, b, i, j, k) - 2.0 * t->dim * f[PX(t, b, i, j, k)];
    double dg, sm = op_sum(t, f, b, i, j, k, &dg);
    return sm - dg * f[PX(t, b, i, j, k)];
}

/* Side ghosts of eps on every box of level l: the eps of the cell across
   the side; on a physical side the face cell's own eps; on a refinement
   boundary the eps of the coarse cell that contains the ghost centre (the
   jumps lie on coarse-grid faces, paper §3.4, so this is the eps there). */
static void fill_eps_gc(otree *t, int l) {
    int D = t->dim;
    double *f = t->eps;
    for (int m = 0; m < lvl_count(t, l); m++) {
        int b = lvl_box(t, l, m);
        int n = t->n[b];
        for (int s = 0; s < 2 * D; s++) {
            int d = s / 2, hi = s % 2;
            int nb = t->nbr[6 * b + s];
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int c = 1; c <= (D == 3 ? n : 1); c++)
                for (int a = 1; a <= n; a++) {
                    int g[3], c1[3];
                    g[t1] = c1[t1] = a;
                    g[t2] = c1[t2] = D == 3 ? c : 1;
                    g[d] = hi ? n + 1 : 0;
                    c1[d] = hi ? n : 1;
                    double v;
                    if (nb >= 0) {
                        int q[3] = {c1[0], c1[1], c1[2]};
                        q[d] = hi ? 1 : n;
                        v = f[PX(t, nb, q[0], q[1], q[2])];
                    } else if (nb == -1) {
                        v = f[PX(t, b, c1[0], c1[1], c1[2])];
                    } else {
                        int cb = t->nbr[6 * t->parent[b] + s];
                        int qc[3];
                        qc[d] = hi ? 1 : n;
                        qc[t1] = child_offset(t, b, t1) + (a + 1) / 2;
                        qc[t2] = D == 3 ? child_offset(t, b, t2) + (c + 1) / 2 : 1;
                        v = f[PX(t, cb, qc[0], qc[1], qc[2])];
                    }
                    f[PX(t, b, g[0], g[1], g[2])] = v;
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* smoother (paper §3.1)                                                     */
/* ------------------------------------------------------------------------ */
/* colour 0 = red: 1-based index sum even (within a box this equals the
   parity of the global index sum because box offsets are even) */
static void half_sweep(otree *t, int l, int colour, int homog) {
    fill_gc(t, l, t->u, homog);
    double h = level_h(t, l), h2 = h * h;
    double twoD = 2.0 * t->dim;
#pragma omp parallel for schedule(dynamic, 16)
    for (int m = 0; m < lvl_count(t, l); m++) {
        int b = lvl_box(t, l, m);
        FOR_CELLS(t, b, i, j, k) {
            int par = (i + j + (t->dim == 3 ? k : 0)) & 1;
            if (par != colour) continue;
            int64_t c = PX(t, b, i, j, k);
            if (t->opk) {
                /* the cell's own equation solved with the neighbours fixed */
                double dg, sm = op_sum(t, t->u, b, i, j, k, &dg);
                t->u[c] = (sm - h2 * t->rho[c]) / dg;
            } else {
                t->u[c] = (nb_sum(t, t->u, b, i, j, k) - h2 * t->rho[c]) / twoD;
            }
        }
    }
}
static void gsrb(otree *t, int l, int nsweep, int homog) {
    for (int s = 0; s < nsweep; s++) {
        half_sweep(t, l, 0, homog);
        half_sweep(t, l, 1, homog);
    }
}

/* r = rho - L u on the given box (ghosts must be filled) */
static void box_residual(otree *t, int b, double *out) {
    double h = level_h(t, t->lev[b]), ih2 = 1.0 / (h * h);
    FOR_CELLS(t, b, i, j, k) {
        int64_t c = PX(t, b, i, j, k);
        out[c] = t->rho[c] - op_h2(t, t->u, b, i, j, k) * ih2;
    }
}

/* ------------------------------------------------------------------------ */
/* restriction / prolongation (paper §2.5)                                   */
/* ------------------------------------------------------------------------ */
/* parent cells covered by box b <- mean of its 2^D cells, for field src -> dst
   (in the cylindrical form the mean over the parent cell's volume, each
   child weighted by its volume, which is proportional to its radius) */
static void restrict_box(otree *t, int b, const double *src, double *dst) {
    int p = t->parent[b], D = t->dim, n = t->n[b];
    int o0 = child_offset(t, b, 0), o1 = child_offset(t, b, 1), o2 = D == 3 ? child_offset(t, b, 2) : 0;
    int nk = D == 3 ? n / 2 : 1;
    double w = D == 3 ? 0.125 : 0.25;
    if (t->opk & OR_OP_CYL) {
        /* volume mean: the children's volumes are proportional to their
           radius r (x); the parent cell's volume is their sum */
        double h = level_h(t, t->lev[b]);
        double x0 = (double)(t->ix[b] - 1) * n * h;
        for (int J = 1; J <= n / 2; J++)
            for (int I = 1; I <= n / 2; I++) {
                double s = 0.0, v = 0.0;
                for (int dj = 0; dj < 2; dj++)
                    for (int di = 0; di < 2; di++) {
                        int i = 2 * I - 1 + di;
                        double r = x0 + (i - 0.5) * h;
                        s += r * src[PX(t, b, i, 2 * J - 1 + dj, 1)];
                        v += r;
                    }
                dst[PX(t, p, o0 + I, o1 + J, 1)] = s / v;
            }
        return;
    }
    for (int K = 1; K <= nk; K++)
        for (int J = 1; J <= n / 2; J++)
            for (int I = 1; I <= n / 2; I++) {
                double s = 0.0;
                int nkk = D == 3 ? 2 : 1;
                for (int dk = 0; dk < nkk; dk++)
                    for (int dj = 0; dj < 2; dj++)
                        for (int di = 0; di < 2; di++)
                            s += src[PX(t, b, 2 * I - 1 + di, 2 * J - 1 + dj, D == 3 ? 2 * K - 1 + dk : 1)];
                dst[PX(t, p, o0 + I, o1 + J, D == 3 ? o2 + K : 1)] = w * s;
            }
}

/* u_b += P211(delta) where delta = u - uold of the parent, ghosts included.
   With OR_OP_PROLONG_EPS the weights come from the parent's eps: along each
   axis d the fine cell sits a quarter coarse cell from its coarse cell P
   towards the neighbour P + s_d e_d, and the piecewise-linear profile with
   continuous value and continuous flux eps du/dx at the face between them
   (the local reconstruction of paper §3.4) puts it at
     delta(P) + eps_d / (2 (eps_P + eps_d)) (delta(P + s_d e_d) - delta(P));
   the corrections of the axes add up.  With equal eps every weight is 1/4,
   which is the default interpolation in 2D and 3D. */
static void prolong_correct_box(otree *t, int b) {
    int p = t->parent[b], D = t->dim;
    int o0 = child_offset(t, b, 0), o1 = child_offset(t, b, 1), o2 = D == 3 ? child_offset(t, b, 2) : 0;
    FOR_CELLS(t, b, i, j, k) {
        int P[3] = {o0 + (i + 1) / 2, o1 + (j + 1) / 2, D == 3 ? o2 + (k + 1) / 2 : 1};
        int s[3] = {(i & 1) ? -1 : 1, (j & 1) ? -1 : 1, (k & 1) ? -1 : 1};
#define DEL(a, bb, cc) (t->u[PX(t, p, a, bb, cc)] - t->uold[PX(t, p, a, bb, cc)])
        double v;
        if (t->prolong_lin) {
            /* bi/trilinear: weights 3/4 and 1/4 per axis over the 2^D
               nearest coarse cells (edge and corner ghosts included) */
            if (D == 2) {
                v = 0.5625 * DEL(P[0], P[1], 1) + 0.1875 * DEL(P[0] + s[0], P[1], 1) +
                    0.1875 * DEL(P[0], P[1] + s[1], 1) + 0.0625 * DEL(P[0] + s[0], P[1] + s[1], 1);
            } else {
                v = 0.421875 * DEL(P[0], P[1], P[2]) +
                    0.140625 * (DEL(P[0] + s[0], P[1], P[2]) + DEL(P[0], P[1] + s[1], P[2]) +
                                DEL(P[0], P[1], P[2] + s[2])) +
                    0.046875 * (DEL(P[0] + s[0], P[1] + s[1], P[2]) + DEL(P[0] + s[0], P[1], P[2] + s[2]) +
                                DEL(P[0], P[1] + s[1], P[2] + s[2])) +
                    0.015625 * DEL(P[0] + s[0], P[1] + s[1], P[2] + s[2]);
            }
        } else if (t->opk & OR_OP_PROLONG_EPS) {
            double d0 = DEL(P[0], P[1], P[2]), e0 = t->eps[PX(t, p, P[0], P[1], P[2])];
            v = d0;
            for (int d = 0; d < D; d++) {
                int Q[3] = {P[0], P[1], P[2]};
                Q[d] += s[d];
                double ed = t->eps[PX(t, p, Q[0], Q[1], Q[2])];
                v += ed / (2.0 * (e0 + ed)) * (DEL(Q[0], Q[1], Q[2]) - d0);
            }
        } else if (D == 2) {
            v = 0.5 * DEL(P[0], P[1], 1) + 0.25 * DEL(P[0] + s[0], P[1], 1) + 0.25 * DEL(P[0], P[1] + s[1], 1);
        } else {
            v = 0.25 * (DEL(P[0], P[1], P[2]) + DEL(P[0] + s[0], P[1], P[2]) +
                        DEL(P[0], P[1] + s[1], P[2]) + DEL(P[0], P[1], P[2] + s[2]));
        }
#undef DEL
        t->u[PX(t, b, i, j, k)] += v;
    }
}

static void copy_box_padded(otree *t, int b, const double *src, double *dst) {
    int64_t m = or_np(t, b), sz = t->dim == 3 ? m * m * m : m * m;
    memcpy(dst + t->off[b], src + t->off[b], sizeof(double) * sz);
}

/* ------------------------------------------------------------------------ */
/* cycles (paper §3.2)                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int cycle;      /* 0: V-cycles only, 1: one FMG cycle then V-cycles */
    int n_down, n_up, n_base;
    double tol;     /* stop when max|r| <= tol * max|r0| */
    int max_cycles;
    int fixed_cycles; /* > 0: run exactly this many V-cycles, no stop test */
    int use_guess;
    int homog;      /* zero Dirichlet values */
} or_opts;

typedef struct {
    int status;     /* 0 converged, 1 not converged */
    int cycles;     /* V-cycles run (FMG not counted) */
    double r0_max, r0_l2, r_max, r_l2;
    double hist_max[128];
    double hist_l2[128];
} or_stats;

static void vcycle(otree *t, int top, const or_opts *o) {
    int homog = o->homog;
    for (int l = top; l > t->lmin; l--) {
        gsrb(t, l, o->n_down, homog);
        fill_gc(t, l, t->u, homog);
#pragma omp parallel for schedule(dynamic, 16)
        for (int m = 0; m < lvl_count(t, l); m++) {
            int b = lvl_box(t, l, m);
            box_residual(t, b, t->res);
            restrict_box(t, b, t->u, t->u);
            restrict_box(t, b, t->res, t->res);
        }
        fill_gc(t, l - 1, t->u, homog);
        double H = level_h(t, l - 1), iH2 = 1.0 / (H * H);
#pragma omp parallel for schedule(dynamic, 16)
        for (int m = 0; m < lvl_count(t, l - 1); m++) {
            int b = lvl_box(t, l - 1, m);
            copy_box_padded(t, b, t->u, t->uold);
            if (t->leaf[b]) continue;
            FOR_CELLS(t, b, i, j, k) {
                int64_t c = PX(t, b, i, j, k);
                t->rho[c] = t->res[c] + op_h2(t, t->u, b, i, j, k) * iH2;
            }
        }
    }
    gsrb(t, t->lmin, o->n_base, homog);
    for (int l = t->lmin + 1; l <= top; l++) {
        fill_gc(t, l - 1, t->u, homog);
#pragma omp parallel for schedule(dynamic, 16)
        for (int m = 0; m < lvl_count(t, l); m++) prolong_correct_box(t, lvl_box(t, l, m));
        gsrb(t, l, o->n_up, homog);
    }
}

/* restrict u into all parents, fill ghosts, composite residual on leaves.
   Returns max|r| and sqrt(sum r^2 h^D). */
static void finalize(otree *t, int homog, double *rmax, double *rl2) {
    for (int l = t->lmax; l > t->lmin; l--) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int m = 0; m < lvl_count(t, l); m++) restrict_box(t, lvl_box(t, l, m), t->u, t->u);
    }
    double mx = 0.0, s2 = 0.0;
    for (int l = 1; l <= t->lmax; l++) {
        fill_gc(t, l, t->u, homog);
        double h = level_h(t, l), hD = t->dim == 3 ? h * h * h : h * h;
        double lmx = 0.0, ls2 = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : lmx) reduction(+ : ls2)
        for (int m = 0; m < lvl_count(t, l); m++) {
            int b = lvl_box(t, l, m);
            if (!t->leaf[b]) continue;
            box_residual(t, b, t->res);
            FOR_CELLS(t, b, i, j, k) {
                double r = t->res[PX(t, b, i, j, k)];
                if (fabs(r) > lmx) lmx = fabs(r);
                ls2 += r * r;
            }
        }
        if (lmx > mx) mx = lmx;
        s2 += ls2 * hD;
    }
    *rmax = mx;
    *rl2 = sqrt(s2);
}

static void fmg(otree *t, const or_opts *o) {
    int homog = o->homog;
    memset(t->u, 0, sizeof(double) * t->ntot);
    for (int l = t->lmax; l > t->lmin; l--) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int m = 0; m < lvl_count(t, l); m++) restrict_box(t, lvl_box(t, l, m), t->rho, t->rho);
    }
    for (int l = t->lmin; l <= t->lmax; l++) {
        fill_gc(t, l, t->u, homog);
#pragma omp parallel for schedule(dynamic, 16)
        for (int m = 0; m < lvl_count(t, l); m++) copy_box_padded(t, lvl_box(t, l, m), t->u, t->uold);
        if (l > t->lmin) {
            fill_gc(t, l - 1, t->u, homog);
#pragma omp parallel for schedule(dynamic, 16)
            for (int m = 0; m < lvl_count(t, l); m++) prolong_correct_box(t, lvl_box(t, l, m));
        }
        if (l == t->lmin) gsrb(t, l, o->n_base, homog);
        else vcycle(t, l, o);
    }
}

static int load_inputs(otree *t, const double *rho_leaf, const double *bc_leaf, const double *u_leaf,
                       int use_guess) {
    memset(t->u, 0, sizeof(double) * t->ntot);
    memset(t->rho, 0, sizeof(double) * t->ntot);
    memset(t->uold, 0, sizeof(double) * t->ntot);
    memset(t->res, 0, sizeof(double) * t->ntot);
    load_leaf_field(t, t->rho, rho_leaf);
    if (bc_leaf) set_bc(t, bc_leaf);
    else for (int64_t i = 0; i < t->nbc; i++) t->bc[i] = 0.0;
    if (use_guess && u_leaf) load_leaf_field(t, t->u, u_leaf);
    return 0;
}

/* Solve lap_h u = rho.  rho_leaf: [n_leaves][N^D]; bc_leaf: [n_leaves][2D][N^(D-1)]
   (NULL = zero); u_leaf: in (guess if use_guess) / out. */
int or_solve(void *p, const double *rho_leaf, const double *bc_leaf, double *u_leaf,
             const or_opts *o, or_stats *st) {
    otree *t = (otree *)p;
    memset(st, 0, sizeof(*st));
    load_inputs(t, rho_leaf, bc_leaf, u_leaf, o->use_guess);
    double r0m, r0l;
    finalize(t, o->homog, &r0m, &r0l);
    st->r0_max = r0m; st->r0_l2 = r0l;
    st->r_max = r0m; st->r_l2 = r0l;
    if (!isfinite(r0m)) { st->status = -5; return -5; }
    if (o->cycle == 1 && !o->use_guess) {
        fmg(t, o);
        finalize(t, o->homog, &st->r_max, &st->r_l2);
    }
    int conv = 0;
    if (o->fixed_cycles <= 0 && st->r_max <= o->tol * r0m) conv = 1;
    int nmax = o->fixed_cycles > 0 ? o->fixed_cycles : o->max_cycles;
    while (!conv && st->cycles < nmax) {
        vcycle(t, t->lmax, o);
        finalize(t, o->homog, &st->r_max, &st->r_l2);
        if (st->cycles < 128) { st->hist_max[st->cycles] = st->r_max; st->hist_l2[st->cycles] = st->r_l2; }
        st->cycles++;
        if (!isfinite(st->r_max)) { st->status = -5; store_leaf_field(t, t->u, u_leaf); return -5; }
        if (o->fixed_cycles <= 0 && st->r_max <= o->tol * r0m) conv = 1;
    }
    store_leaf_field(t, t->u, u_leaf);
    st->status = (o->fixed_cycles > 0 || conv) ? 0 : 1;
    return st->status;
}

/* ------------------------------------------------------------------------ */
/* entry points used by the pins                                             */
/* ------------------------------------------------------------------------ */

/* Composite operator on leaves: out = L u (homog = zero Dirichlet values) or
   out = L u + boundary part.  Parents get the restriction of u first. */
void or_apply_L(void *p, const double *u_leaf, const double *bc_leaf, double *out_leaf, int homog) {
    otree *t = (otree *)p;
    int nleaf = t->nleaf_in, N = t->N, D = t->dim;
    int64_t nc = D == 3 ? (int64_t)N * N * N : (int64_t)N * N;
    double *zero = calloc((size_t)nleaf * nc, sizeof(double));
    load_inputs(t, zero, bc_leaf, u_leaf, 1);
    free(zero);
    double a, bq;
    finalize(t, homog, &a, &bq); /* res = rho - L u = -L u */
    store_leaf_field(t, t->res, out_leaf);
    for (int64_t i = 0; i < (int64_t)nleaf * nc; i++) out_leaf[i] = -out_leaf[i];
}

/* Load a state: u on leaves (restricted into parents), rho, bc. */
void or_load(void *p, const double *rho_leaf, const double *bc_leaf, const double *u_leaf) {
    otree *t = (otree *)p;
    load_inputs(t, rho_leaf, bc_leaf, u_leaf, u_leaf != NULL);
    double a, b;
    finalize(t, 0, &a, &b);
}
void or_fill_gc(void *p, int l, int which, int homog) { otree *t = (otree *)p; fill_gc(t, l, fld(t, which), homog); }
void or_half_sweep(void *p, int l, int colour, int homog) { half_sweep((otree *)p, l, colour, homog); }
void or_vcycle(void *p, const or_opts *o) { otree *t = (otree *)p; vcycle(t, t->lmax, o); }
void or_fmg(void *p, const or_opts *o) { fmg((otree *)p, o); }
void or_finalize(void *p, int homog, double *out2) { finalize((otree *)p, homog, out2, out2 + 1); }
void or_restrict_level(void *p, int l, int which) {
    otree *t = (otree *)p;
    double *f = fld(t, which);
    for (int m = 0; m < lvl_count(t, l); m++) restrict_box(t, lvl_box(t, l, m), f, f);
}
/* u_old <- u on every box of level l (incl. ghosts) */
void or_copy_uold(void *p, int l) {
    otree *t = (otree *)p;
    for (int m = 0; m < lvl_count(t, l); m++) copy_box_padded(t, lvl_box(t, l, m), t->u, t->uold);
}
/* the residual of level l restricted, with u, into the parents (the first
   half of the V-cycle's step at level l) */
void or_resid_restrict_level(void *p, int l, int homog) {
    otree *t = (otree *)p;
    fill_gc(t, l, t->u, homog);
    for (int m = 0; m < lvl_count(t, l); m++) {
        int b = lvl_box(t, l, m);
        box_residual(t, b, t->res);
        restrict_box(t, b, t->u, t->u);
        restrict_box(t, b, t->res, t->res);
    }
}
/* on level l: u_old <- u, and rho <- res + L u on parents (the second half
   of the V-cycle's step at level l+1) */
void or_coarse_rhs_level(void *p, int l, int homog) {
    otree *t = (otree *)p;
    fill_gc(t, l, t->u, homog);
    double H = level_h(t, l), iH2 = 1.0 / (H * H);
    for (int m = 0; m < lvl_count(t, l); m++) {
        int b = lvl_box(t, l, m);
        copy_box_padded(t, b, t->u, t->uold);
        if (t->leaf[b]) continue;
        FOR_CELLS(t, b, i, j, k) {
            int64_t c = PX(t, b, i, j, k);
            t->rho[c] = t->res[c] + op_h2(t, t->u, b, i, j, k) * iH2;
        }
    }
}
/* the V-cycle from level top */
void or_vcycle_from(void *p, int top, const or_opts *o) { vcycle((otree *)p, top, o); }
void or_prolong_level(void *p, int l) {
    otree *t = (otree *)p;
    for (int m = 0; m < lvl_count(t, l); m++) prolong_correct_box(t, lvl_box(t, l, m));
}
/* padded box array of a field: (n+2)^D values, x fastest */
void or_get_box(void *p, int b, int which, double *out) {
    otree *t = (otree *)p;
    int64_t m = or_np(t, b), sz = t->dim == 3 ? m * m * m : m * m;
    memcpy(out, fld(t, which) + t->off[b], sizeof(double) * sz);
}
void or_set_box(void *p, int b, int which, const double *in) {
    otree *t = (otree *)p;
    int64_t m = or_np(t, b), sz = t->dim == 3 ? m * m * m : m * m;
    memcpy(fld(t, which) + t->off[b], in, sizeof(double) * sz);
}
void or_get_leaf_field(void *p, int which, double *out) { otree *t = (otree *)p; store_leaf_field(t, fld(t, which), out); }
/* Dirichlet values in use for box b side s (n^(D-1) values); returns 0 if the
   side is not physical */
int or_get_bc(void *p, int b, int s, double *out) {
    otree *t = (otree *)p;
    int64_t o = t->bcoff[6 * b + s];
    if (o < 0) return 0;
    int64_t nf = t->dim == 3 ? (int64_t)t->n[b] * t->n[b] : t->n[b];
    memcpy(out, t->bc + o, sizeof(double) * nf);
    return 1;
}
int or_num_threads(void) { return omp_get_max_threads(); }

/* Operator of later solves (paper §3.4, §3.5): kind = OR_OP_EPS and / or
   OR_OP_CYL bits (0: the Laplacian); eps_leaf [n_leaves][N^D] (x fastest),
   positive, required with OR_OP_EPS; prolong = 1 selects the eps-weighted
   prolongation (needs OR_OP_EPS).  eps of parents and of the coarse grids
   is the mean over their children (paper §2.5), so a jump on a coarse-grid
   face stays on a face on every level.  Returns 0, or -1 with a message. */
int or_set_operator(void *p, int kind, const double *eps_leaf, int prolong) {
    otree *t = (otree *)p;
    if (kind < 0 || kind > (OR_OP_EPS | OR_OP_CYL)) { seterr(NULL, 0, "bad operator kind"); return -1; }
    if (prolong < 0 || prolong > 2) { seterr(NULL, 0, "bad prolongation"); return -1; }
    if ((kind & OR_OP_CYL) && t->dim != 2) { seterr(NULL, 0, "the cylindrical operator is 2D (r, z)"); return -1; }
    if ((kind & OR_OP_EPS) && !eps_leaf) { seterr(NULL, 0, "eps missing"); return -1; }
    if (prolong == 1 && !(kind & OR_OP_EPS)) { seterr(NULL, 0, "the eps prolongation needs eps"); return -1; }
    int64_t nc = t->dim == 3 ? (int64_t)t->N * t->N * t->N : (int64_t)t->N * t->N;
    if (kind & OR_OP_EPS)
        for (int64_t i = 0; i < nc * t->nleaf_in; i++)
            if (!(eps_leaf[i] > 0.0) || !isfinite(eps_leaf[i])) { seterr(NULL, 0, "eps must be positive and finite"); return -1; }
    free(t->eps);
    t->eps = NULL;
    t->opk = kind | (prolong == 1 ? OR_OP_PROLONG_EPS : 0);
    t->prolong_lin = prolong == 2;
    if (!(kind & OR_OP_EPS)) return 0;
    t->eps = calloc(t->ntot, sizeof(double));
    load_leaf_field(t, t->eps, eps_leaf);
    for (int l = t->lmax; l > t->lmin; l--)
        for (int m = 0; m < lvl_count(t, l); m++) restrict_box(t, lvl_box(t, l, m), t->eps, t->eps);
    for (int l = t->lmin; l <= t->lmax; l++) fill_eps_gc(t, l);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* sparse assembly of the composite operator (for the adjoint oracle)        */
/* ------------------------------------------------------------------------ */
/* Row of leaf cell c: (sum over its 2D sides of u_nb - 2D u_c) / h^2 with the
   neighbour value of each side written out as a combination of leaf cells:
     same-level leaf cell      -> that cell
     same-level refined cell   -> mean of its 2^D children (leaf cells, 2:1)
     physical side (b = 0)     -> -u_c
     refinement boundary       -> 1/2 u_H + k1 u_c - 1/4 (u_c2 + partners),
                                  k1 = 1 (2D), 5/4 (3D)
   This is the same operator as fill_gc + the stencil (homogeneous values).
   Unknowns are numbered q * N^D + (x-fastest cell) in the caller's leaf
   order.  Call with rows == NULL to get the number of entries. */
static int64_t leaf_unknown(const otree *t, const int *leaf_of_box, int b, int i, int j, int k) {
    int q = leaf_of_box[b];
    int N = t->N;
    int64_t cell = t->dim == 3 ? (i - 1) + (int64_t)N * ((j - 1) + (int64_t)N * (k - 1)) : (i - 1) + (int64_t)N * (j - 1);
    return (int64_t)q * (t->dim == 3 ? (int64_t)N * N * N : (int64_t)N * N) + cell;
}

/* Refinement-boundary ghost scheme of later solves: 0 the default (from the
   two closest fine values), 1 bilinear (3D: trilinear) extrapolation (paper
   §3.3).  Both keep the coarse flux equal to the mean of the fine fluxes. */
int or_set_ghost_scheme(void *p, int scheme) {
    otree *t = (otree *)p;
    if (scheme != 0 && scheme != 1) { seterr(NULL, 0, "bad ghost scheme"); return -1; }
    t->ghost_bil = scheme;
    return 0;
}

int64_t or_assemble_L(void *p, int32_t *rows, int32_t *cols, double *vals) {
    otree *t = (otree *)p;
    if (t->opk || t->ghost_bil) { seterr(NULL, 0, "assembly covers the Laplacian with the default ghosts only"); return -1; }
    int D = t->dim, N = t->N;
    int *leaf_of_box = malloc(sizeof(int) * t->nbox);
    for (int b = 0; b < t->nbox; b++) leaf_of_box[b] = -1;
    for (int q = 0; q < t->nleaf_in; q++) leaf_of_box[t->leaf_box[q]] = q;
    int64_t n = 0;
#define PUT(r, c, v)                                   \
    do {                                               \
        if (rows) { rows[n] = (int32_t)(r); cols[n] = (int32_t)(c); vals[n] = (v); } \
        n++;                                           \
    } while (0)
    for (int qq = 0; qq < t->nleaf_in; qq++) {
        int b = t->leaf_box[qq];
        double h = level_h(t, t->lev[b]), ih2 = 1.0 / (h * h);
        FOR_CELLS(t, b, i, j, k) {
            int64_t row = leaf_unknown(t, leaf_of_box, b, i, j, D == 3 ? k : 1);
            double diag = -2.0 * D * ih2;
            int c[3] = {i, j, D == 3 ? k : 1};
            for (int s = 0; s < 2 * D; s++) {
                int d = s / 2, hi = s % 2;
                int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                int x[3] = {c[0], c[1], c[2]};
                x[d] += hi ? 1 : -1;
                if (x[d] >= 1 && x[d] <= N) { /* inside the box */
                    PUT(row, leaf_unknown(t, leaf_of_box, b, x[0], x[1], x[2]), ih2);
                    continue;
                }
                if (c[d] != (hi ? N : 1)) continue;
                int nb = t->nbr[6 * b + s];
                if (nb >= 0) {
                    int y[3] = {c[0], c[1], c[2]};
                    y[d] = hi ? 1 : N;
                    if (t->leaf[nb]) {
                        PUT(row, leaf_unknown(t, leaf_of_box, nb, y[0], y[1], y[2]), ih2);
                    } else {
                        /* refined neighbour: mean of the 2^D children of cell y */
                        double w = ih2 / (D == 3 ? 8.0 : 4.0);
                        for (int oc = 0; oc < (1 << D); oc++) {
                            int f[3];
                            f[0] = 2 * y[0] - 1 + (oc & 1);
                            f[1] = 2 * y[1] - 1 + ((oc >> 1) & 1);
                            f[2] = D == 3 ? 2 * y[2] - 1 + ((oc >> 2) & 1) : 1;
                            int bits = ((f[0] - 1) / N) | (((f[1] - 1) / N) << 1) | (D == 3 ? (((f[2] - 1) / N) << 2) : 0);
                            int ch = t->child[8 * nb + bits];
                            PUT(row, leaf_unknown(t, leaf_of_box, ch, (f[0] - 1) % N + 1, (f[1] - 1) % N + 1,
                                                  D == 3 ? (f[2] - 1) % N + 1 : 1), w);
                        }
                    }
                } else if (nb == -1) {
                    /* physical side: ghost -u_c (Dirichlet) or +u_c (Neumann) */
                    diag += t->bctype[s] == OR_NEUMANN ? ih2 : -ih2;
                } else {
                    int par = t->parent[b];
                    int cb = t->nbr[6 * par + s];
                    int qc[3];
                    qc[d] = hi ? 1 : N;
                    qc[t1] = child_offset(t, b, t1) + (c[t1] + 1) / 2;
                    qc[t2] = D == 3 ? child_offset(t, b, t2) + (c[t2] + 1) / 2 : 1;
                    PUT(row, leaf_unknown(t, leaf_of_box, cb, qc[0], qc[1], qc[2]), 0.5 * ih2);
                    diag += (D == 3 ? 1.25 : 1.0) * ih2;
                    int y[3] = {c[0], c[1], c[2]};
                    y[d] = hi ? N - 1 : 2;
                    PUT(row, leaf_unknown(t, leaf_of_box, b, y[0], y[1], y[2]), -0.25 * ih2);
                    int p1[3] = {c[0], c[1], c[2]};
                    p1[t1] = (c[t1] % 2) ? c[t1] + 1 : c[t1] - 1;
                    PUT(row, leaf_unknown(t, leaf_of_box, b, p1[0], p1[1], p1[2]), -0.25 * ih2);
                    if (D == 3) {
                        int p2[3] = {c[0], c[1], c[2]};
                        p2[t2] = (c[t2] % 2) ? c[t2] + 1 : c[t2] - 1;
                        PUT(row, leaf_unknown(t, leaf_of_box, b, p2[0], p2[1], p2[2]), -0.25 * ih2);
                    }
                }
            }
            PUT(row, row, diag);
        }
    }
#undef PUT
    free(leaf_of_box);
    return n;
}
