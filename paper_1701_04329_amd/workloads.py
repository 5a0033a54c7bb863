"""Seeded synthetic inputs for the multigrid Poisson solve.

This module only produces inputs: leaf lists of quadtree/octree grids and
analytic fields sampled on them.  It holds none of the solver's arithmetic
(no ghost cells, no stencils, no cycles), so the FP64 oracle and the HIP
path can both consume what it returns without sharing any solver code.

Conventions (shared by every consumer):

* Domain [0,1]^D covered by one root box at level 1.  A box at level l has
  N^D cells of size h_l = 1 / (N * 2^(l-1)) and a 1-based spatial index
  (i, j[, k]); its children have indices (2i-1 .. 2i, ...)  (paper §2.1).
* A grid is given by its leaves: ``level`` int32 [n], ``idx`` int32 [n, 3]
  (third column 1 in 2D).
* Cell fields per leaf are float64 [n, N^D], x fastest.
* Dirichlet values per leaf are float64 [n, 2D, N^(D-1)] at the face
  centres of the box sides ordered (-x, +x, -y, +y, -z, +z); on each side the
  tangential axes are taken in increasing axis order, the first fastest.
  Only sides on the physical boundary are meaningful; the rest are zero.
* Sign convention: the solver solves lap_h(u) = rho, so a manufactured
  solution u gives rho = lap(u) sampled at cell centres (paper §4.1 uses the
  same form of the Poisson equation).

Refinement follows the flag rules of paper §2.3: a box is refined when any of
its cells is flagged, boxes whose cells lie within N_buf = 2 cells of a
flagged cell (diagonal neighbours included) are refined too, and coarser
neighbours are refined to keep 2:1 balance (diagonal neighbours included).
The flag criterion is the form used in paper §4.1, |lap u| h^2 > threshold.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

BOX_N_DEFAULT = 8


# ----------------------------------------------------------------------------
# analytic sources
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class GaussMix:
    """u(x) = sum_k amp_k * exp(-|x - c_k|^2 / sigma_k^2)."""

    centres: np.ndarray  # [K, D]
    sigmas: np.ndarray  # [K]
    amps: np.ndarray  # [K]

    @property
    def dim(self) -> int:
        return self.centres.shape[1]

    def value(self, x: np.ndarray) -> np.ndarray:
        """x: [..., D] -> [...]"""
        out = np.zeros(x.shape[:-1])
        for c, s, a in zip(self.centres, self.sigmas, self.amps):
            r2 = np.sum((x - c) ** 2, axis=-1)
            out += a * np.exp(-r2 / (s * s))
        return out

    def gradient(self, x: np.ndarray) -> np.ndarray:
        """x: [..., D] -> [..., D]: sum_k -2 (x - c_k) / s_k^2 * g_k."""
        out = np.zeros(x.shape)
        for c, s, a in zip(self.centres, self.sigmas, self.amps):
            r2 = np.sum((x - c) ** 2, axis=-1)
            g = a * np.exp(-r2 / (s * s))
            out += (-2.0 / (s * s)) * (x - c) * g[..., None]
        return out

    def laplacian(self, x: np.ndarray) -> np.ndarray:
        """Analytic Laplacian: (4 r^2 / s^4 - 2 D / s^2) * g for each term."""
        d = x.shape[-1]
        out = np.zeros(x.shape[:-1])
        for c, s, a in zip(self.centres, self.sigmas, self.amps):
            r2 = np.sum((x - c) ** 2, axis=-1)
            g = a * np.exp(-r2 / (s * s))
            out += g * (4.0 * r2 / s**4 - 2.0 * d / s**2)
        return out


def gauss_mix_seeded(dim, n, seed, lo=0.1, hi=0.9, sigma_range=(0.05, 0.05),
                     log_sigma=False):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(n, dim))
    s0, s1 = sigma_range
    if log_sigma:
        sig = np.exp(rng.uniform(math.log(s0), math.log(s1), size=n))
    else:
        sig = rng.uniform(s0, s1, size=n)
    return GaussMix(centres, sig, np.ones(n))


# ----------------------------------------------------------------------------
# grid geometry helpers (pure index arithmetic)
# ----------------------------------------------------------------------------


def box_h(level, n_cells=BOX_N_DEFAULT):
    return 1.0 / (n_cells * 2.0 ** (np.asarray(level, dtype=np.float64) - 1.0))


def cell_centres(dim, N, level, idx):
    """Cell centres of the given boxes: [n, N^D, D] (x fastest)."""
    level = np.asarray(level)
    idx = np.asarray(idx)
    h = box_h(level, N)  # [n]
    loc = (np.arange(N) + 0.5)
    grids = np.meshgrid(*([loc] * dim), indexing="ij")  # grid[d][i0, i1, ...]
    # x fastest: flatten with axis order (z, y, x)
    offs = []
    for d in range(dim):
        g = np.transpose(grids[d], axes=list(range(dim))[::-1]).reshape(-1)
        offs.append(g)
    offs = np.stack(offs, axis=-1)  # [N^D, D]
    origin = (idx[:, :dim] - 1).astype(np.float64) * N * h[:, None]  # [n, D]
    return origin[:, None, :] + offs[None, :, :] * h[:, None, None]


def face_centres(dim, N, level, idx, side):
    """Face centres of side `side` of each box: [n, N^(D-1), D]."""
    level = np.asarray(level)
    idx = np.asarray(idx)
    h = box_h(level, N)
    axis, hi = side // 2, side % 2
    tang = [d for d in range(dim) if d != axis]
    loc = np.arange(N) + 0.5
    if dim == 2:
        t = [loc]
    else:
        a, b = np.meshgrid(loc, loc, indexing="ij")
        t = [np.transpose(a).reshape(-1), np.transpose(b).reshape(-1)]
    n = len(level)
    out = np.zeros((n, N ** (dim - 1), dim))
    origin = (idx[:, :dim] - 1).astype(np.float64) * N * h[:, None]
    for m, d in enumerate(tang):
        out[:, :, d] = origin[:, d:d + 1] + t[m][None, :] * h[:, None]
    out[:, :, axis] = origin[:, axis:axis + 1] + (N * h[:, None] if hi else 0.0)
    return out


def physical_side_mask(dim, level, idx):
    """[n, 2D] bool: side lies on the boundary of [0,1]^D."""
    level = np.asarray(level)
    idx = np.asarray(idx)
    nmax = 2 ** (level - 1)
    m = np.zeros((len(level), 2 * dim), dtype=bool)
    for d in range(dim):
        m[:, 2 * d] = idx[:, d] == 1
        m[:, 2 * d + 1] = idx[:, d] == nmax
    return m


def domain_side_mask(dim, level, idx, bc_type=None):
    """[n, 2D] bool: the side of each leaf lies on the domain boundary.  The
    domain is the union of the level-1 boxes holding the leaves (unit boxes
    on the integer lattice); a side is on the boundary when the position
    across it is outside the lattice on a non-periodic axis or in a lattice
    position without a level-1 box.  bc_type: None, one name, or 2D names
    among "dirichlet", "neumann", "periodic" (pairs per axis)."""
    level = np.asarray(level)
    idx = np.asarray(idx)
    types = side_types(dim, bc_type)
    roots = {tuple(((idx[q, d] - 1) >> (level[q] - 1)) + 1 for d in range(dim)) for q in range(len(level))}
    ext = [max(r[d] for r in roots) for d in range(dim)]
    m = np.zeros((len(level), 2 * dim), dtype=bool)
    for q in range(len(level)):
        l = int(level[q])
        for s in range(2 * dim):
            d, dr = s // 2, (1 if s % 2 else -1)
            p = [int(idx[q, e]) for e in range(dim)]
            p[d] += dr
            n1 = ext[d] * 2 ** (l - 1)
            if not 1 <= p[d] <= n1:
                if types[s] != "periodic":
                    m[q, s] = True
                    continue
                p[d] = (p[d] - 1) % n1 + 1
            root = tuple((p[e] - 1) // 2 ** (l - 1) + 1 for e in range(dim))
            m[q, s] = root not in roots
    return m


def side_types(dim, bc_type):
    if bc_type is None:
        return ["dirichlet"] * (2 * dim)
    if isinstance(bc_type, str):
        return [bc_type] * (2 * dim)
    return list(bc_type)


def domain_leaves(dim, N, roots, lmax, centre, radius=0.0, n_buf=0, periodic=None):
    """Leaves over a coarse grid of several level-1 boxes (roots: lattice
    positions, 1-based), refined to lmax around a ball; periodic: per axis."""
    return adaptive_leaves(dim, N, ball_flag(dim, N, centre, radius), lmax, n_buf=n_buf, roots=roots,
                           periodic=periodic)


def domain_fields(dim, N, level, idx, seed, bc_type=None):
    """Seeded random rho and boundary values (Dirichlet values or outward
    derivatives, per the side types) on a general domain.  Without any
    Dirichlet side the problem is singular: rho is then shifted by a
    constant so that the volume integral of rho equals the boundary integral
    of the Neumann derivatives, the discrete compatibility condition."""
    rng = np.random.default_rng(seed)
    level = np.asarray(level, np.int32)
    idx = np.asarray(idx, np.int32)
    n = len(level)
    types = side_types(dim, bc_type)
    rho = rng.standard_normal((n, N ** dim))
    bc = rng.standard_normal((n, 2 * dim, N ** (dim - 1)))
    bc *= domain_side_mask(dim, level, idx, types)[:, :, None]
    if "dirichlet" not in types:
        h = box_h(level, N)
        vol = np.sum(h ** dim) * N ** dim
        flux = 0.0
        for s in range(2 * dim):
            if types[s] == "neumann":
                flux += np.sum(bc[:, s, :] * (h[:, None] ** (dim - 1)))
        excess = np.sum(rho * (h[:, None] ** dim)) - flux
        rho -= excess / vol
    name = f"domain_{dim}d_{'_'.join(t[0] for t in types)}_s{seed}"
    return Workload(name, dim, N, level, idx, rho, bc)


# ----------------------------------------------------------------------------
# leaf lists
# ----------------------------------------------------------------------------


def uniform_leaves(dim, level):
    n1 = 2 ** (level - 1)
    r = np.arange(1, n1 + 1, dtype=np.int32)
    if dim == 2:
        j, i = np.meshgrid(r, r, indexing="ij")
        idx = np.stack([i.ravel(), j.ravel(), np.ones(i.size, np.int32)], 1)
    else:
        k, j, i = np.meshgrid(r, r, r, indexing="ij")
        idx = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)
    lev = np.full(len(idx), level, dtype=np.int32)
    return lev, idx.astype(np.int32)


def _neighbour_offsets(dim):
    rng = [-1, 0, 1]
    if dim == 2:
        return [(a, b, 0) for b in rng for a in rng if (a, b) != (0, 0)]
    return [(a, b, c) for c in rng for b in rng for a in rng if (a, b, c) != (0, 0, 0)]


class _LeafSet:
    """Mutable set of leaves keyed by (level, i, j, k); used only to build
    input grids.  The coarse grid is a set of level-1 boxes (roots) at
    1-based lattice positions; a periodic axis wraps positions around the
    lattice's extent."""

    def __init__(self, dim, roots=None, periodic=None):
        self.dim = dim
        roots = [(1, 1, 1)] if roots is None else [tuple(int(v) for v in r) for r in roots]
        if dim == 2:
            roots = [(r[0], r[1], 1) for r in roots]
        self.roots = set(roots)
        self.ext = tuple(max(r[d] for r in roots) for d in range(3))
        self.periodic = tuple(periodic) if periodic is not None else (False, False, False)
        self.leaves = {(1,) + r for r in roots}

    def wrap(self, level, i, j, k):
        """The position (level, i, j, k) inside the domain (periodic axes
        wrapped), or None outside it or in a hole of the coarse grid."""
        q = [i, j, k]
        for d in range(self.dim):
            n1 = self.ext[d] * 2 ** (level - 1)
            if not 1 <= q[d] <= n1:
                if not self.periodic[d]:
                    return None
                q[d] = (q[d] - 1) % n1 + 1
        root = tuple((q[d] - 1) // 2 ** (level - 1) + 1 for d in range(self.dim)) + ((1,) if self.dim == 2 else ())
        if root not in self.roots:
            return None
        return (level, q[0], q[1], q[2] if self.dim == 3 else 1)

    def covering_leaf(self, level, i, j, k):
        """The leaf covering box position (level, i, j, k), or None if that
        position is refined further (or outside the domain)."""
        w = self.wrap(level, i, j, k)
        if w is None:
            return None
        l, a, b, c = w
        while l >= 1:
            if (l, a, b, c) in self.leaves:
                return (l, a, b, c)
            l -= 1
            a, b = (a + 1) // 2, (b + 1) // 2
            c = (c + 1) // 2 if self.dim == 3 else 1
        return None

    def refine(self, key):
        l, i, j, k = key
        self.leaves.remove(key)
        ks = (0, 1) if self.dim == 3 else (0,)
        for dk in ks:
            for dj in (0, 1):
                for di in (0, 1):
                    kk = 2 * k - 1 + dk if self.dim == 3 else 1
                    self.leaves.add((l + 1, 2 * i - 1 + di, 2 * j - 1 + dj, kk))

    def arrays(self):
        keys = sorted(self.leaves)
        lev = np.array([k[0] for k in keys], dtype=np.int32)
        idx = np.array([k[1:] for k in keys], dtype=np.int32).reshape(-1, 3)
        return lev, idx


def adaptive_leaves(dim, N, flag_fn, lmax, n_buf=2, roots=None, periodic=None):
    """Refine from the root (or the given roots) until stable.

    flag_fn(level, idx[n,3]) -> bool [n, N^D] cell flags for the given boxes.
    A box is refined when any cell is flagged (and its level < lmax); same-level
    neighbours whose cells lie within n_buf cells of a flagged cell are refined
    too; coarser neighbours (diagonals included) are refined for 2:1 balance.
    roots: lattice positions of the level-1 boxes (default the unit box);
    periodic: per axis, whether neighbours wrap around the lattice.
    """
    ls = _LeafSet(dim, roots, periodic)
    offs = _neighbour_offsets(dim)
    evaluated = set()
    while True:
        cand = sorted(k for k in ls.leaves if k[0] < lmax and k not in evaluated)
        flagged = set()
        if cand:
            lev = np.array([k[0] for k in cand], dtype=np.int32)
            idx = np.array([k[1:] for k in cand], dtype=np.int32)
            cf = flag_fn(lev, idx).reshape((len(cand),) + (N,) * dim)  # [n, (z,) y, x]
            for key in cand:
                evaluated.add(key)
            for m, key in enumerate(cand):
                f = cf[m]
                if not f.any():
                    continue
                flagged.add(key)
                # buffer: which neighbour directions contain a cell within
                # n_buf cells of a flagged cell
                for o in offs:
                    sl = []
                    for d in range(dim):
                        od = o[d]
                        if od == -1:
                            sl.append(slice(0, n_buf))
                        elif od == 1:
                            sl.append(slice(N - n_buf, N))
                        else:
                            sl.append(slice(0, N))
                    sl = tuple(sl[::-1])  # array axes are (z,) y, x
                    if f[sl].any():
                        l, i, j, k = key
                        nb = ls.wrap(l, i + o[0], j + o[1], k + o[2] if dim == 3 else 1)
                        if nb in ls.leaves:
                            flagged.add(nb)
        flagged = {k for k in flagged if k[0] < lmax}
        if not flagged:
            break
        # 2:1 balance: coarser neighbours of a box to be refined get refined
        work = list(flagged)
        while work:
            key = work.pop()
            l, i, j, k = key
            for o in offs:
                nb = ls.covering_leaf(l, i + o[0], j + o[1], (k + o[2]) if dim == 3 else 1)
                if nb is not None and nb[0] < l and nb not in flagged:
                    flagged.add(nb)
                    work.append(nb)
        for key in sorted(flagged):
            ls.refine(key)
    return ls.arrays()


def laplacian_flag(mix: GaussMix, N, threshold):
    def fn(level, idx):
        xc = cell_centres(mix.dim, N, level, idx)
        h = box_h(level, N)
        return np.abs(mix.laplacian(xc)) * (h[:, None] ** 2) > threshold
    return fn


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    N: int
    level: np.ndarray  # int32 [n]
    idx: np.ndarray  # int32 [n, 3]
    rho: np.ndarray  # float64 [n, N^D]
    bc: np.ndarray  # float64 [n, 2D, N^(D-1)]
    u_exact: np.ndarray | None = None  # float64 [n, N^D] analytic at centres
    mix: GaussMix | None = None
    eps: np.ndarray | None = None  # float64 [n, N^D] cell coefficients (variable operators)

    @property
    def n_leaves(self):
        return len(self.level)

    @property
    def n_unknowns(self):
        return len(self.level) * self.N ** self.dim

    @property
    def lmax(self):
        return int(self.level.max())


def sample_workload(name, dim, N, level, idx, mix: GaussMix | None, bc_from_mix=True,
                    rho_const=None, with_exact=True):
    """Sample rho = lap(u) at cell centres and Dirichlet values u at physical
    face centres.  rho_const overrides rho with a constant (EX4-style)."""
    level = np.asarray(level, dtype=np.int32)
    idx = np.asarray(idx, dtype=np.int32)
    n = len(level)
    nf = N ** (dim - 1)
    bc = np.zeros((n, 2 * dim, nf))
    if rho_const is not None:
        rho = np.full((n, N ** dim), float(rho_const))
        u_ex = None
    else:
        xc = cell_centres(dim, N, level, idx)
        rho = mix.laplacian(xc)
        u_ex = mix.value(xc) if with_exact else None
        if bc_from_mix:
            phys = physical_side_mask(dim, level, idx)
            for s in range(2 * dim):
                sel = np.nonzero(phys[:, s])[0]
                if len(sel):
                    fc = face_centres(dim, N, level[sel], idx[sel], s)
                    bc[sel, s, :] = mix.value(fc)
    return Workload(name, dim, N, level, idx, np.ascontiguousarray(rho), bc, u_ex, mix)


def config1(N=BOX_N_DEFAULT):
    """2D, uniform 128^2 (levels 1..5 with 8^2 boxes), u = exp(-|x-x0|^2/0.01),
    x0 = (0.5, 0.5), zero Dirichlet values."""
    lmax = 1 + int(round(math.log2(128 // N)))
    lev, idx = uniform_leaves(2, lmax)
    mix = GaussMix(np.array([[0.5, 0.5]]), np.array([0.1]), np.array([1.0]))
    return sample_workload("c1_2d_uniform_128", 2, N, lev, idx, mix, bc_from_mix=False)


def config2(N=BOX_N_DEFAULT, res=256, seed=2):
    """3D, uniform res^3, two Gaussians sigma = 0.05 with seeded centres in
    [0.1, 0.9]^3, Dirichlet values from the analytic solution."""
    lmax = 1 + int(round(math.log2(res // N)))
    lev, idx = uniform_leaves(3, lmax)
    mix = gauss_mix_seeded(3, 2, seed, 0.1, 0.9, (0.05, 0.05))
    return sample_workload(f"c2_3d_uniform_{res}", 3, N, lev, idx, mix)


def config3(N=BOX_N_DEFAULT, lmax=8, threshold=1e-4, seed=3, n_src=4,
            sigma_range=(0.01, 0.05)):
    """3D adaptive octree refined where |lap u| h^2 > threshold around n_src
    seeded Gaussians (sigma log-uniform in sigma_range)."""
    mix = gauss_mix_seeded(3, n_src, seed, 0.1, 0.9, sigma_range, log_sigma=True)
    lev, idx = adaptive_leaves(3, N, laplacian_flag(mix, N, threshold), lmax)
    return sample_workload(f"c3_3d_adaptive_l{lmax}", 3, N, lev, idx, mix)


def config5(N=BOX_N_DEFAULT, lmax=7, threshold=2e-3):
    """3D adaptive octree for the adjoint (about 4e6 unknowns): rho and the
    Dirichlet values from mixture A (4 Gaussians, centres in [0.1, 0.9]^3,
    sigma log-uniform in [0.01, 0.05], seed 5000), refined where
    |lap u| h^2 > threshold; the loss target u_t at the leaf cell centres from
    mixture B (3 Gaussians, sigma uniform in [0.05, 0.1], seed 5001).
    Returns (workload, u_t [n_leaves, N^3])."""
    mix_a = gauss_mix_seeded(3, 4, 5000, 0.1, 0.9, (0.01, 0.05), log_sigma=True)
    lev, idx = adaptive_leaves(3, N, laplacian_flag(mix_a, N, threshold), lmax)
    w = sample_workload(f"c5_3d_adaptive_l{lmax}", 3, N, lev, idx, mix_a)
    mix_b = gauss_mix_seeded(3, 3, 5001, 0.1, 0.9, (0.05, 0.1))
    return w, mix_b.value(cell_centres(3, N, lev, idx))


def adaptive_small(dim, N, lmax, threshold, seed, n_src=2, sigma_range=(0.03, 0.08),
                   name=None):
    """Small adaptive grid for tests: Gaussians in [0.1, 0.9]^D."""
    mix = gauss_mix_seeded(dim, n_src, seed, 0.1, 0.9, sigma_range, log_sigma=True)
    lev, idx = adaptive_leaves(dim, N, laplacian_flag(mix, N, threshold), lmax)
    return sample_workload(name or f"adaptive_{dim}d_l{lmax}_s{seed}", dim, N, lev, idx, mix)


def uniform_const_rhs(dim, N, res, value=1.0):
    """The paper's scaling problem (§4.2): lap(phi) = 1, phi = 0 on the
    boundary, uniform res^D."""
    lmax = 1 + int(round(math.log2(res // N)))
    lev, idx = uniform_leaves(dim, lmax)
    return sample_workload(f"ex4_{dim}d_uniform_{res}", dim, N, lev, idx, None,
                           bc_from_mix=False, rho_const=value)


def random_fields(dim, N, level, idx, seed):
    """Seeded random rho and Dirichlet values (no analytic solution)."""
    rng = np.random.default_rng(seed)
    n = len(level)
    rho = rng.standard_normal((n, N ** dim))
    bc = rng.standard_normal((n, 2 * dim, N ** (dim - 1)))
    bc *= physical_side_mask(dim, level, idx)[:, :, None]
    return Workload(f"random_{dim}d_s{seed}", dim, N, np.asarray(level, np.int32),
                    np.asarray(idx, np.int32), rho, bc)


def _morton_key(dim, i, j, k):
    key, bit = 0, 0
    a, b, c = i - 1, j - 1, k - 1
    while a or b or c:
        key |= (a & 1) << bit | (b & 1) << (bit + 1)
        if dim == 3:
            key |= (c & 1) << (bit + 2)
        a, b, c = a >> 1, b >> 1, c >> 1
        bit += dim
    return key


def greedy_leaves(dim, N, mix: GaussMix, target_boxes, max_level=None):
    """Refine one leaf at a time, the leaf with the largest max |lap u| h^2
    first (ties: coarser level, then lower Morton key), until the tree holds
    at least target_boxes boxes (parents and leaves, levels >= 1).  Before a
    leaf is refined its coarser neighbours (diagonals included) are refined,
    recursively, so the grid stays 2:1 balanced."""
    import heapq

    ls = _LeafSet(dim)
    offs = _neighbour_offsets(dim)
    max_level = max_level or (12 if dim == 3 else 16)
    heap = []
    n_boxes = 1

    def push(keys):
        lev = np.array([k[0] for k in keys], dtype=np.int32)
        idx = np.array([k[1:] for k in keys], dtype=np.int32)
        h = box_h(lev, N)
        score = (np.abs(mix.laplacian(cell_centres(dim, N, lev, idx))) * (h[:, None] ** 2)).max(axis=1)
        for key, sc in zip(keys, score):
            heapq.heappush(heap, (-float(sc), key[0], _morton_key(dim, *key[1:]), key))

    def children(key):
        l, i, j, k = key
        out = []
        for dk in ((0, 1) if dim == 3 else (0,)):
            for dj in (0, 1):
                for di in (0, 1):
                    out.append((l + 1, 2 * i - 1 + di, 2 * j - 1 + dj, 2 * k - 1 + dk if dim == 3 else 1))
        return out

    def refine(key):
        nonlocal n_boxes
        l, i, j, k = key
        for o in offs:
            nb = ls.covering_leaf(l, i + o[0], j + o[1], (k + o[2]) if dim == 3 else 1)
            if nb is not None and nb[0] < l:
                refine(nb)
        ls.refine(key)
        n_boxes += 2 ** dim
        push(children(key))

    push([(1, 1, 1, 1)])
    while n_boxes < target_boxes and heap:
        _, _, _, key = heapq.heappop(heap)
        if key in ls.leaves and key[0] < max_level:
            refine(key)
    return ls.arrays()


def config4_tree(j, N=BOX_N_DEFAULT, box_range=(64, 8192), seed_base=4000):
    """Tree j of the batch workload: D = 2 for even j, 3 for odd j; 1-3
    Gaussians with centres in [0.25, 0.75]^D and sigma log-uniform in
    [0.02, 0.1]; a box target log-uniform in box_range; zero Dirichlet
    values.  All draws come from one generator seeded with seed_base + j."""
    dim = 2 if j % 2 == 0 else 3
    rng = np.random.default_rng(seed_base + j)
    n_src = int(rng.integers(1, 4))
    centres = rng.uniform(0.25, 0.75, size=(n_src, dim))
    sig = np.exp(rng.uniform(math.log(0.02), math.log(0.1), size=n_src))
    target = int(round(math.exp(rng.uniform(math.log(box_range[0]), math.log(box_range[1])))))
    mix = GaussMix(centres, sig, np.ones(n_src))
    lev, idx = greedy_leaves(dim, N, mix, target)
    w = sample_workload(f"c4_tree{j}_{dim}d", dim, N, lev, idx, mix, bc_from_mix=False)
    return w


def _config4_one(args):
    return config4_tree(*args)


def config4(n_trees=256, N=BOX_N_DEFAULT, box_range=(64, 8192), seed_base=4000, workers=1):
    """The batch workload: n_trees independent trees (config4_tree), built
    in `workers` fresh processes when workers > 1."""
    args = [(j, N, box_range, seed_base) for j in range(n_trees)]
    if workers <= 1:
        return [_config4_one(a) for a in args]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_config4_one, args, chunksize=4))


def ball_flag(dim, N, centre, radius):
    """Flag the cells that intersect the ball |x - centre| <= radius."""
    p = np.asarray(centre, dtype=np.float64)[:dim]

    def fn(level, idx):
        xc = cell_centres(dim, N, level, idx)
        h = box_h(level, N)
        return np.linalg.norm(xc - p, axis=-1) < radius + 0.5 * math.sqrt(dim) * h[:, None]
    return fn


def ball_leaves(dim, N, lmax, centre, radius=0.0, n_buf=0):
    """Grid refined to lmax around a ball (small grids with refinement
    boundaries at several levels, used by tests)."""
    return adaptive_leaves(dim, N, ball_flag(dim, N, centre, radius), lmax, n_buf=n_buf)


# ----------------------------------------------------------------------------
# variable coefficients and the cylindrical form (paper §3.4, §3.5, §4.1)
# ----------------------------------------------------------------------------


def random_eps(n_leaves, N, dim, seed, lo=0.5, hi=2.0):
    """Cell coefficients log-uniform in [lo, hi], one per leaf cell."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=(n_leaves, N ** dim)))


def eps_sampled(eps_fn, dim, N, level, idx):
    """eps_fn(x [..., D]) sampled at the leaf cell centres."""
    return np.ascontiguousarray(eps_fn(cell_centres(dim, N, level, idx)))


def case2_eps(x):
    """Paper §4.1, case 2: eps = 100 in the lower left quadrant [0, 0.25]^2
    of the (r, z) domain, 1 elsewhere."""
    return np.where((x[..., 0] < 0.25) & (x[..., 1] < 0.25), 100.0, 1.0)


def case2_mix():
    """u = sum of two Gaussians at (0.25, 0.25) and (0.75, 0.75), sigma 0.04
    (the manufactured solution of paper §4.1, read as Gaussians)."""
    return GaussMix(np.array([[0.25, 0.25], [0.75, 0.75]]), np.array([0.04, 0.04]), np.ones(2))


def divergence_source(mix: GaussMix, eps_fn, dim, N, level, idx, cyl=False):
    """Cell values of rho = div(eps grad u) for a smooth u and a piecewise
    constant eps (cylindrical: (1/r) d/dr (r eps du/dr) + d/dz (eps du/dz),
    x = r).  Away from jumps this is eps(x_c) times the Laplacian of u at the
    cell centre.  A jump of eps on a cell face adds the surface source
    (eps_across - eps_own) du/dn at the face centre (n the outward normal),
    spread over the two cells that share the face, half to each: each takes
    its half times face area / cell volume, 1/(2h) (times r_face / r_c on a
    radial face of the cylindrical form)."""
    level = np.asarray(level)
    idx = np.asarray(idx)
    xc = cell_centres(dim, N, level, idx)
    h = box_h(level, N)[:, None]
    e_c = eps_fn(xc)
    lap = mix.laplacian(xc)
    if cyl:
        lap = lap + mix.gradient(xc)[..., 0] / xc[..., 0]
    rho = e_c * lap
    for d in range(dim):
        for sgn in (-1.0, 1.0):
            off = np.zeros(dim)
            off[d] = sgn
            e_o = eps_fn(xc + off * h[..., None])
            jump = e_o != e_c
            if not jump.any():
                continue
            xf = xc + 0.5 * off * h[..., None]
            dn = sgn * mix.gradient(xf)[..., d]
            geo = xf[..., 0] / xc[..., 0] if (cyl and d == 0) else 1.0
            rho = rho + np.where(jump, 0.5 * (e_o - e_c) * dn * geo / h, 0.0)
    return rho


def case2_workload(N=BOX_N_DEFAULT, lmax=7, threshold=1e-3):
    """Paper §4.1, case 2: the cylindrical (r, z) problem with eps = 100 in
    [0, 0.25]^2 on [0, 1]^2, Dirichlet values from u on every side (the one
    on the axis r = 0 carries no flux), boxes refined where
    h^2 |rho| / eps > threshold."""
    mix = case2_mix()

    def flag(level, idx):
        rho = divergence_source(mix, case2_eps, 2, N, level, idx, cyl=True)
        e = eps_sampled(case2_eps, 2, N, level, idx)
        return np.abs(rho) * box_h(level, N)[:, None] ** 2 / e > threshold

    lev, idx = adaptive_leaves(2, N, flag, lmax)
    w = sample_workload("case2", 2, N, lev, idx, mix)
    w.rho = np.ascontiguousarray(divergence_source(mix, case2_eps, 2, N, lev, idx, cyl=True))
    w.eps = eps_sampled(case2_eps, 2, N, lev, idx)
    return w
