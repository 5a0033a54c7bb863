"""Brute-force composite operator for tiny grids (test helper).

Assembles, cell by cell from the geometry of the leaf cells, the dense matrix
of the composite discretisation that the multigrid method converges to:

  (sum over the 2D faces of u_nb - 2D u_c) / h_c^2 = rho_c

where u_nb across a face is (paper §2.4, §3.3):
  * the neighbouring leaf cell at the same level;
  * the mean of the 2^D leaf cells that refine the neighbouring cell when that
    neighbour is refined (its value is the restriction, paper §2.5);
  * 2 b - u_c at a physical Dirichlet face with value b, u_c + h q at a
    Neumann face with outward derivative q (paper §3: Dirichlet, Neumann or
    periodic boundaries; periodic axes wrap around the domain);
  * the default refinement-boundary ghost of paper §3.3 when the neighbour is
    coarser: 1/2 u_H + u_c - 1/4 (u_c' + u_c2) in 2D and
    1/2 u_H + 5/4 u_c - 1/4 (u_c2 + u_c' + u_c'') in 3D, with u_H the coarse
    leaf cell containing the ghost centre, u_c2 the next cell inward and
    u_c', u_c'' the tangential partners of u_c inside the same coarse cell.

The domain is the union of the level-1 boxes holding the leaves (unit boxes
on the integer lattice, paper §2.2); a face is physical when the cell across
it lies outside the lattice on a non-periodic axis or in a lattice position
without a level-1 box.

This is written independently of the oracle (global cell indices instead of
boxes with stored ghost layers) and only serves to pin it.
"""

from __future__ import annotations

import numpy as np


def assemble(dim, N, level, idx, bc=None, bc_type=None):
    """Return (A, g) with A u = rho - g for the leaf unknowns in leaf-list
    order (x fastest within each leaf), g the boundary part.  bc_type: None
    (all Dirichlet), one name or 2D names among "dirichlet", "neumann",
    "periodic"."""
    level = np.asarray(level)
    idx = np.asarray(idx)
    n_leaf = len(level)
    if bc_type is None:
        types = ["dirichlet"] * (2 * dim)
    elif isinstance(bc_type, str):
        types = [bc_type] * (2 * dim)
    else:
        types = list(bc_type)
    roots = {tuple(((int(idx[q, d]) - 1) >> (int(level[q]) - 1)) + 1 for d in range(dim)) for q in range(n_leaf)}
    ext = [max(r[d] for r in roots) for d in range(dim)]
    boxes = set()
    leaves = {}
    for q in range(n_leaf):
        l = int(level[q])
        key = (l,) + tuple(int(v) for v in idx[q, :dim])
        leaves[key] = q
        while l >= 1:
            boxes.add(key)
            l -= 1
            key = (l,) + tuple((v + 1) // 2 for v in key[1:])
    ncell = N ** dim
    n = n_leaf * ncell

    def local_iter():
        if dim == 2:
            for j in range(N):
                for i in range(N):
                    yield (i, j)
        else:
            for k in range(N):
                for j in range(N):
                    for i in range(N):
                        yield (i, j, k)

    locs = list(local_iter())
    loc_pos = {loc: m for m, loc in enumerate(locs)}

    def cell_unknown(l, G):
        """unknown index of leaf cell with global 0-based index G at level l,
        or None if that cell is not a leaf cell."""
        B = (l,) + tuple(g // N + 1 for g in G)
        q = leaves.get(B)
        if q is None:
            return None
        loc = tuple(g % N for g in G)
        return q * ncell + loc_pos[loc]

    def box_exists(l, G):
        return ((l,) + tuple(g // N + 1 for g in G)) in boxes

    A = np.zeros((n, n))
    gvec = np.zeros(n)
    for q in range(n_leaf):
        l = int(level[q])
        h = 1.0 / (N * 2.0 ** (l - 1))
        ih2 = 1.0 / (h * h)
        per_root = N * 2 ** (l - 1)  # cells per axis of one level-1 box at level l
        org = [(int(idx[q, d]) - 1) * N for d in range(dim)]
        for loc in locs:
            row = q * ncell + loc_pos[loc]
            G = [org[d] + loc[d] for d in range(dim)]
            A[row, row] -= 2 * dim * ih2
            for d in range(dim):
                for sgn in (-1, 1):
                    side = 2 * d + (1 if sgn > 0 else 0)
                    Gn = list(G)
                    Gn[d] += sgn
                    nl = ext[d] * per_root
                    outside = Gn[d] < 0 or Gn[d] >= nl
                    if outside and types[side] == "periodic":
                        Gn[d] %= nl
                        outside = False
                    if not outside:
                        outside = tuple(g // per_root + 1 for g in Gn) not in roots  # a hole
                    if outside:
                        tang = [loc[e] for e in range(dim) if e != d]
                        fi = tang[0] + (N * tang[1] if dim == 3 else 0)
                        bv = 0.0 if bc is None else bc[q, side, fi]
                        if types[side] == "neumann":
                            # ghost = u_c + h q
                            A[row, row] += ih2
                            gvec[row] += bv * h * ih2
                        else:
                            # Dirichlet: ghost = 2 b - u_c
                            A[row, row] -= ih2
                            gvec[row] += 2.0 * bv * ih2
                        continue
                    if box_exists(l, Gn):
                        col = cell_unknown(l, Gn)
                        if col is not None:
                            A[row, col] += ih2
                        else:
                            # refined neighbour: mean of its 2^D children
                            w = ih2 / 2 ** dim
                            for off in np.ndindex(*([2] * dim)):
                                Gc = [2 * Gn[e] + off[e] for e in range(dim)]
                                cc = cell_unknown(l + 1, Gc)
                                assert cc is not None, "2:1 balance violated"
                                A[row, cc] += w
                        continue
                    # coarser neighbour: default refinement-boundary ghost
                    GH = [g // 2 for g in Gn]
                    cH = cell_unknown(l - 1, GH)
                    assert cH is not None, "coarse neighbour is not a leaf"
                    G2 = list(G)
                    G2[d] -= sgn
                    c2 = cell_unknown(l, G2)
                    tang = [e for e in range(dim) if e != d]
                    partners = []
                    for e in tang:
                        Gp = list(G)
                        Gp[e] ^= 1
                        partners.append(cell_unknown(l, Gp))
                    A[row, cH] += 0.5 * ih2
                    if dim == 2:
                        A[row, row] += 1.0 * ih2
                        A[row, partners[0]] -= 0.25 * ih2
                        A[row, c2] -= 0.25 * ih2
                    else:
                        A[row, row] += 1.25 * ih2
                        A[row, c2] -= 0.25 * ih2
                        A[row, partners[0]] -= 0.25 * ih2
                        A[row, partners[1]] -= 0.25 * ih2
    return A, gvec


def leaf_cell_volumes(dim, N, level):
    h = 1.0 / (N * 2.0 ** (np.asarray(level, dtype=np.float64) - 1))
    return np.repeat(h ** dim, N ** dim)
