"""Mesh adaptation (paper §2.3) and the transfer of a cell field onto the
adapted grid (paper §2.3, with the prolongation and restriction of §2.5).

TEST INFRASTRUCTURE ONLY: the slow, plain reference that the GPU library's
adaptation is checked against.  Only tests, the smoke check and the
benchmark's CPU leg use it.  It shares no code with the library.

A grid is a leaf list: level int [n], idx int [n, 3] (1-based box indices,
third column 1 in 2D).  The coarse grid is the set of level-1 boxes under
the leaves (unit boxes on an integer lattice, paper §2.2); periodic axes wrap
around the lattice extent.

Adaptation rules, in the paper's order (§2.3), from per-cell flags
(+1 refine, -1 derefine, 0 keep) on the leaves:
  1. a leaf with a cell flagged for refinement is refined;
  2. a same-level leaf neighbour (diagonal neighbours included) is refined
     too when a refine-flagged cell lies within n_buf cells of it: along
     each axis where the neighbour is offset, the cell is among the n_buf
     cells next to that side;
  3. 2:1 balance: a leaf to be refined at level l makes every coarser leaf
     that touches it (sides, edges, corners) be refined too, recursively;
  4. a leaf whose cells are all flagged for derefinement is marked for
     removal; the 2^D children of a box are removed (the box becomes a leaf)
     when all are leaves, all are marked, none is to be refined, and the
     box as a leaf would keep 2:1 balance with the refined grid (no leaf
     finer than one level above it touches it);
  5. a grid changes by at most one level per adaptation; boxes at the
     maximum level are not refined.
"""

from __future__ import annotations

import itertools

import numpy as np


def _offsets(dim):
    return [o for o in itertools.product((-1, 0, 1), repeat=dim) if any(o)]


class _Grid:
    def __init__(self, dim, level, idx, periodic):
        self.dim = dim
        self.leaves = {}
        for q, (l, i) in enumerate(zip(level, idx)):
            self.leaves[(int(l),) + tuple(int(v) for v in i[:dim])] = q
        self.boxes = set()
        for k in self.leaves:
            l, p = k[0], list(k[1:])
            while l >= 1:
                self.boxes.add((l,) + tuple(p))
                l -= 1
                p = [(v + 1) // 2 for v in p]
        self.roots = {k[1:] for k in self.boxes if k[0] == 1}
        self.ext = [max(r[d] for r in self.roots) for d in range(dim)]
        self.periodic = [bool(periodic[d]) if periodic is not None else False for d in range(dim)]

    def wrap(self, key):
        """key inside the domain (periodic axes wrapped), or None"""
        l, p = key[0], list(key[1:])
        for d in range(self.dim):
            n = self.ext[d] << (l - 1)
            if p[d] < 1 or p[d] > n:
                if not self.periodic[d]:
                    return None
                p[d] = (p[d] - 1) % n + 1
        root = tuple(((v - 1) >> (l - 1)) + 1 for v in p)
        if root not in self.roots:
            return None
        return (l,) + tuple(p)

    def covering_leaf(self, key):
        key = self.wrap(key)
        if key is None:
            return None
        l, p = key[0], list(key[1:])
        while l >= 1:
            k = (l,) + tuple(p)
            if k in self.leaves:
                return k
            l -= 1
            p = [(v + 1) // 2 for v in p]
        return None

    def children(self, key):
        l, p = key[0], key[1:]
        return [(l + 1,) + tuple(2 * p[d] - 1 + o[d] for d in range(self.dim))
                for o in itertools.product((0, 1), repeat=self.dim)]


def max_level(dim):
    """the deepest level the library keeps (box counts and indices fit in int32)"""
    return 17 if dim == 3 else 20


def adapt(dim, N, level, idx, flags, n_buf=2, periodic=None, lmax=None):
    """New leaf list (level, idx), sorted by level then index."""
    level = np.asarray(level)
    idx = np.asarray(idx).reshape(-1, 3)
    flags = np.asarray(flags).reshape((len(level),) + (N,) * dim)  # axes (z,) y, x
    g = _Grid(dim, level, idx, periodic)
    lmax = max_level(dim) if lmax is None else lmax
    keys = [(int(l),) + tuple(int(v) for v in i[:dim]) for l, i in zip(level, idx)]
    refine = set()
    # rules 1 and 2: flagged leaves and their buffer neighbours
    for q, key in enumerate(keys):
        f = flags[q]
        cells = np.argwhere(f > 0)  # rows of (z,) y, x
        if len(cells) == 0:
            continue
        if key[0] < lmax:
            refine.add(key)
        for o in _offsets(dim):
            near = np.ones(len(cells), bool)
            for d in range(dim):
                c = cells[:, dim - 1 - d]
                if o[d] == -1:
                    near &= c < n_buf
                elif o[d] == 1:
                    near &= c >= N - n_buf
            if not near.any():
                continue
            nb = g.wrap((key[0],) + tuple(key[1 + d] + o[d] for d in range(dim)))
            if nb is not None and nb in g.leaves and nb[0] < lmax:
                refine.add(nb)
    # rule 3: 2:1 balance, diagonal neighbours included
    work = list(refine)
    while work:
        key = work.pop()
        for o in _offsets(dim):
            nb = g.covering_leaf((key[0],) + tuple(key[1 + d] + o[d] for d in range(dim)))
            if nb is not None and nb[0] < key[0] and nb not in refine:
                refine.add(nb)
                work.append(nb)
    # rule 4: removal of children
    marked = {key for q, key in enumerate(keys) if np.all(flags[q] < 0) and key not in refine}
    parents = {(k[0] - 1,) + tuple((v + 1) // 2 for v in k[1:]) for k in marked if k[0] >= 2}
    coarsen = set()
    for p in sorted(parents):
        kids = g.children(p)
        if not all(k in marked for k in kids):
            continue
        ok = True
        for o in _offsets(dim):
            nb = g.wrap((p[0],) + tuple(p[1 + d] + o[d] for d in range(dim)))
            if nb is None or nb not in g.boxes or nb in g.leaves:
                continue  # outside, covered by a coarser leaf, or a leaf (refined or not: one level up)
            # the neighbour's children that touch p must stay leaves
            for c in g.children(nb):
                touches = all((o[d] == 0) or (o[d] == -1 and (c[1 + d] - 1) % 2 == 1)
                              or (o[d] == 1 and (c[1 + d] - 1) % 2 == 0) for d in range(dim))
                if touches and (c not in g.leaves or c in refine):
                    ok = False
        if ok:
            coarsen.add(p)
    out = set()
    for key in keys:
        if key in refine:
            out.update(g.children(key))
        elif key[0] >= 2 and (key[0] - 1,) + tuple((v + 1) // 2 for v in key[1:]) in coarsen:
            continue
        else:
            out.add(key)
    out.update(coarsen)
    keys = sorted(out)
    lev = np.array([k[0] for k in keys], np.int32)
    ix = np.ones((len(keys), 3), np.int32)
    for q, k in enumerate(keys):
        ix[q, :dim] = k[1:]
    return lev, ix


def transfer(old_tree, new_level, new_idx, u_old, bc_old=None):
    """The cell field u_old [n_old_leaves, N^D] (x fastest) of the oracle
    tree old_tree on the adapted leaves: a leaf that existed keeps its
    values; a leaf whose children were removed takes their mean (the
    restriction of §2.5, through the old tree's parents); a new child takes
    the default prolongation of §2.5 from its parent (an old leaf), whose
    side ghosts are those of the solve (neighbour values, boundary values
    bc_old, refinement-boundary ghosts)."""
    dim, N = old_tree.dim, old_tree.N
    C = N ** dim
    old_tree.load(np.zeros((old_tree.n_leaves, C)), bc_old, np.asarray(u_old, dtype=np.float64))
    box_of = {}
    for b in range(old_tree.nbox):
        i = old_tree.box_info(b)
        if i["level"] >= 1:
            box_of[(i["level"], i["ix"], i["iy"], i["iz"] if dim == 3 else 1)] = b
    inner = tuple(slice(1, -1) for _ in range(dim))
    out = np.zeros((len(new_level), C))
    for q, (l, i) in enumerate(zip(new_level, np.asarray(new_idx).reshape(-1, 3))):
        key = (int(l), int(i[0]), int(i[1]), int(i[2]) if dim == 3 else 1)
        if key in box_of:
            out[q] = old_tree.box_padded(box_of[key])[inner].ravel()
            continue
        pkey = (key[0] - 1,) + tuple((v + 1) // 2 for v in key[1:1 + dim]) + ((1,) if dim == 2 else ())
        P = old_tree.box_padded(box_of[pkey])  # axes (z,) y, x with the ghost layer
        off = [((key[1 + d] - 1) & 1) * (N // 2) for d in range(dim)]
        fine = np.zeros((N,) * dim)
        for cell in itertools.product(range(N), repeat=dim):  # cell = (x, y[, z])
            c = [off[d] + cell[d] // 2 + 1 for d in range(dim)]  # padded parent index
            s = [1 if cell[d] % 2 else -1 for d in range(dim)]

            def at(cc):
                return P[tuple(cc[::-1])]

            nb = []
            for d in range(dim):
                cc = list(c)
                cc[d] += s[d]
                nb.append(at(cc))
            if dim == 2:
                v = 0.5 * at(c) + 0.25 * nb[0] + 0.25 * nb[1]
            else:
                v = 0.25 * (at(c) + nb[0] + nb[1] + nb[2])
            fine[tuple(cell[::-1])] = v
        out[q] = fine.ravel()
    return out
