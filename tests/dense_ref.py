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

Variable coefficients and the cylindrical form (paper §3.4, §3.5): each face
term (u_nb - u_c) / h^2 is multiplied by a face weight w, the harmonic mean
2 e_c e_nb / (e_c + e_nb) of the coefficient of the cell and of the cell
across the face (its own value at a physical face; for a refined neighbour
the volume mean of the children's values; for a coarser neighbour the value
of the coarse leaf cell), times r_face / r_c on the radial faces of the
cylindrical form (x = r, the face on the axis has weight 0).  In the
cylindrical form the value of a refined cell (u and eps) is the mean over
its volume: children weighted by their radius.

This is written independently of the oracle (global cell indices instead of
boxes with stored ghost layers) and only serves to pin it.
"""

from __future__ import annotations

import numpy as np


def assemble(dim, N, level, idx, bc=None, bc_type=None, eps=None, cyl=False, ghost="default"):
    """Return (A, g) with A u = rho - g for the leaf unknowns in leaf-list
    order (x fastest within each leaf), g the boundary part.  bc_type: None
    (all Dirichlet), one name or 2D names among "dirichlet", "neumann",
    "periodic".  eps: [n_leaves, N^D] cell coefficients (None: 1); cyl: the
    cylindrical (r, z) form (2D); ghost: "default" or "bilinear", the
    bilinear-extrapolation refinement ghost of paper §3.3: in 2D
    1/2 u_H + 9/8 u_c - 3/8 (u_p + u_c2) + 1/8 u_c2p, in 3D the same
    construction with one more tangential axis,
    1/2 u_H + 27/16 u_c - 9/16 (u_c2 + u_p + u_q) + 3/16 (u_c2p + u_c2q + u_pq)
    - 1/16 u_c2pq (p, q: partner along the first, second tangential axis)."""
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

    epsf = None if eps is None else np.asarray(eps, dtype=np.float64).reshape(n_leaf, ncell)

    def child_weights(l, G):
        """children of cell G of level l and their volume fractions"""
        kids = [[2 * G[e] + off[e] for e in range(dim)] for off in np.ndindex(*([2] * dim))]
        if cyl:
            hc = 1.0 / (N * 2.0 ** l)  # child cell size
            r = np.array([(k[0] + 0.5) * hc for k in kids])
            return kids, r / r.sum()
        return kids, np.full(len(kids), 1.0 / len(kids))

    def cell_eps(l, G):
        """volume mean of the leaf coefficients inside cell G of level l"""
        u = cell_unknown(l, G)
        if u is not None:
            return epsf.reshape(-1)[u]
        kids, wk = child_weights(l, G)
        return float(sum(w * cell_eps(l + 1, k) for k, w in zip(kids, wk)))

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
            e_c = None if epsf is None else epsf[q, loc_pos[loc]]
            for d in range(dim):
                for sgn in (-1, 1):
                    # face weight: geometric factor now, the coefficient part
                    # once the cell across the face is known
                    geo = 1.0
                    if cyl and d == 0:
                        r_c = (G[0] + 0.5) * h
                        geo = (G[0] + (1.0 if sgn > 0 else 0.0)) * h / r_c
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
                        # the coefficient across a physical face is the cell's own
                        wf = geo * (1.0 if e_c is None else e_c) * ih2
                        A[row, row] -= wf
                        tang = [loc[e] for e in range(dim) if e != d]
                        fi = tang[0] + (N * tang[1] if dim == 3 else 0)
                        bv = 0.0 if bc is None else bc[q, side, fi]
                        if types[side] == "neumann":
                            # ghost = u_c + h q
                            A[row, row] += wf
                            gvec[row] += bv * h * wf
                        else:
                            # Dirichlet: ghost = 2 b - u_c
                            A[row, row] -= wf
                            gvec[row] += 2.0 * bv * wf
                        continue

                    def harm(e_n):
                        return 1.0 if e_c is None else 2.0 * e_c * e_n / (e_c + e_n)

                    if box_exists(l, Gn):
                        col = cell_unknown(l, Gn)
                        wf = geo * (1.0 if e_c is None else harm(cell_eps(l, Gn))) * ih2
                        A[row, row] -= wf
                        if col is not None:
                            A[row, col] += wf
                        else:
                            # refined neighbour: mean of its 2^D children
                            kids, wk = child_weights(l, Gn)
                            for Gc, w in zip(kids, wk):
                                cc = cell_unknown(l + 1, Gc)
                                assert cc is not None, "2:1 balance violated"
                                A[row, cc] += wf * w
                        continue
                    # coarser neighbour: default refinement-boundary ghost
                    GH = [g // 2 for g in Gn]
                    cH = cell_unknown(l - 1, GH)
                    assert cH is not None, "coarse neighbour is not a leaf"
                    wf = geo * (1.0 if e_c is None else harm(epsf.reshape(-1)[cH])) * ih2
                    A[row, row] -= wf
                    G2 = list(G)
                    G2[d] -= sgn
                    c2 = cell_unknown(l, G2)
                    tang = [e for e in range(dim) if e != d]
                    partners = []
                    for e in tang:
                        Gp = list(G)
                        Gp[e] ^= 1
                        partners.append(cell_unknown(l, Gp))
                    A[row, cH] += 0.5 * wf
                    if ghost == "bilinear":
                        def cell(G0, flips):
                            Gq = list(G0)
                            for e in flips:
                                Gq[e] ^= 1
                            return cell_unknown(l, Gq)
                        if dim == 2:
                            e1 = tang[0]
                            A[row, row] += 1.125 * wf
                            A[row, partners[0]] -= 0.375 * wf
                            A[row, c2] -= 0.375 * wf
                            A[row, cell(G2, [e1])] += 0.125 * wf
                        else:
                            e1, e2 = tang
                            A[row, row] += 27.0 / 16.0 * wf
                            for c_ in (c2, partners[0], partners[1]):
                                A[row, c_] -= 9.0 / 16.0 * wf
                            for c_ in (cell(G2, [e1]), cell(G2, [e2]), cell(G, [e1, e2])):
                                A[row, c_] += 3.0 / 16.0 * wf
                            A[row, cell(G2, [e1, e2])] -= 1.0 / 16.0 * wf
                        continue
                    if dim == 2:
                        A[row, row] += 1.0 * wf
                        A[row, partners[0]] -= 0.25 * wf
                        A[row, c2] -= 0.25 * wf
                    else:
                        A[row, row] += 1.25 * wf
                        A[row, c2] -= 0.25 * wf
                        A[row, partners[0]] -= 0.25 * wf
                        A[row, partners[1]] -= 0.25 * wf
    return A, gvec


def leaf_cell_volumes(dim, N, level):
    h = 1.0 / (N * 2.0 ** (np.asarray(level, dtype=np.float64) - 1))
    return np.repeat(h ** dim, N ** dim)
