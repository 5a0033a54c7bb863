"""Pins of the oracle's mesh adaptation and field transfer (paper §2.3, §2.5):

* hand-worked cases of each rule (a flagged cell deep inside a box, at a
  face and at a corner with the buffer, 2:1 propagation to a coarser
  neighbour, removal of four marked children, removal blocked by three
  marks, by a neighbour's refinement and by a finer neighbour);
* properties on random flags, checked by brute force over box geometry:
  the result tiles the domain, keeps 2:1 balance across sides, edges and
  corners (periodic axes wrapped), changes every location by at most one
  level, refines every leaf with a refine-flagged cell and removes only
  fully marked sibling groups;
* transfer: a linear field is carried exactly (the default prolongation,
  the ghosts of the solve and the mean are exact for it); unchanged leaves
  keep their values bitwise; a constant field stays constant on a periodic
  domain.
"""

import itertools

import numpy as np
import pytest

from oracle import adapt as AD
from oracle import oracle as O
from paper_1701_04329_amd import workloads as W


def keyset(level, idx, dim):
    return {(int(l),) + tuple(int(v) for v in i[:dim]) for l, i in zip(level, np.asarray(idx).reshape(-1, 3))}


def flags_zero(level, N, dim):
    return np.zeros((len(level), N ** dim), np.int8)


def set_cell(flags, q, cell, N, val):
    """cell (x, y[, z]) 0-based of leaf q"""
    p = 0
    for d in reversed(range(len(cell))):
        p = p * N + cell[d]
    flags[q, p] = val


def leaf_index(level, idx, key, dim):
    for q, (l, i) in enumerate(zip(level, idx)):
        if (int(l),) + tuple(int(v) for v in i[:dim]) == key:
            return q
    raise KeyError(key)


# ---------------------------------------------------------------------------
# brute-force geometry checks
# ---------------------------------------------------------------------------
def box_interval(key, dim):
    l = key[0]
    w = 2.0 ** (1 - l)
    return [((key[1 + d] - 1) * w, key[1 + d] * w) for d in range(dim)]


def touches(a, b, dim, ext, periodic):
    ia, ib = box_interval(a, dim), box_interval(b, dim)
    for shift in itertools.product(*[((-ext[d], 0, ext[d]) if periodic[d] else (0,)) for d in range(dim)]):
        if all(ia[d][0] <= ib[d][1] + shift[d] + 1e-12 and ib[d][0] + shift[d] <= ia[d][1] + 1e-12
               for d in range(dim)):
            return True
    return False


def check_grid(keys, dim, ext, periodic, roots):
    keys = list(keys)
    vol = sum(2.0 ** (dim * (1 - k[0])) for k in keys)
    assert abs(vol - len(roots)) < 1e-9, "leaves do not tile the domain"
    for a, b in itertools.combinations(keys, 2):
        ia, ib = box_interval(a, dim), box_interval(b, dim)
        overlap = all(min(ia[d][1], ib[d][1]) - max(ia[d][0], ib[d][0]) > 1e-12 for d in range(dim))
        assert not overlap, (a, b)
        if abs(a[0] - b[0]) > 1 and touches(a, b, dim, ext, periodic):
            raise AssertionError(f"2:1 balance broken between {a} and {b}")


# ---------------------------------------------------------------------------
# hand-worked cases
# ---------------------------------------------------------------------------
def uniform(dim, level):
    return W.uniform_leaves(dim, level)


def test_no_flags_no_change():
    for dim in (2, 3):
        lev, idx = W.ball_leaves(dim, 4, 4, (0.3, 0.6, 0.4), 0.0, 1)
        nl, ni = AD.adapt(dim, 4, lev, idx, flags_zero(lev, 4, dim))
        assert keyset(nl, ni, dim) == keyset(lev, idx, dim)


def test_interior_cell_refines_its_box_only():
    dim, N = 2, 8
    lev, idx = uniform(2, 3)  # 4x4 boxes of level 3
    f = flags_zero(lev, N, dim)
    q = leaf_index(lev, idx, (3, 2, 3), dim)
    set_cell(f, q, (4, 3), N, 1)  # not within 2 cells of any side
    nl, ni = AD.adapt(dim, N, lev, idx, f, n_buf=2)
    want = keyset(lev, idx, dim) - {(3, 2, 3)} | {(4, 3, 5), (4, 4, 5), (4, 3, 6), (4, 4, 6)}
    assert keyset(nl, ni, dim) == want


def test_buffer_reaches_face_and_diagonal_neighbours():
    dim, N = 2, 8
    lev, idx = uniform(2, 3)
    f = flags_zero(lev, N, dim)
    q = leaf_index(lev, idx, (3, 2, 3), dim)
    set_cell(f, q, (1, 0), N, 1)  # 1 cell from -x, 0 from -y
    nl, ni = AD.adapt(dim, N, lev, idx, f, n_buf=2)
    refined = {(3, 2, 3), (3, 1, 3), (3, 2, 2), (3, 1, 2)}
    got = keyset(nl, ni, dim)
    for k in refined:
        assert k not in got and (4, 2 * k[1] - 1, 2 * k[2] - 1) in got
    assert len(got) == 16 + 3 * len(refined)
    # with n_buf = 1 the cell (1, 0) is 2 cells from -x: only the -y neighbour
    nl, ni = AD.adapt(dim, N, lev, idx, f, n_buf=1)
    assert len(keyset(nl, ni, dim)) == 16 + 3 * 2


def test_two_to_one_refines_coarser_neighbours():
    dim, N = 2, 8
    # level 2 boxes, one of them refined to level 3
    lev, idx = uniform(2, 2)
    kids = [(3, 1 + a, 1 + b) for a in (0, 1) for b in (0, 1)]
    lev = np.array([2, 2, 2] + [3] * 4, np.int32)
    idx = np.array([[2, 1, 1], [1, 2, 1], [2, 2, 1]] + [[k[1], k[2], 1] for k in kids], np.int32)
    f = flags_zero(lev, N, dim)
    q = leaf_index(lev, idx, (3, 2, 2), dim)  # touches all three level-2 boxes
    set_cell(f, q, (3, 3), N, 1)
    nl, ni = AD.adapt(dim, N, lev, idx, f, n_buf=0)
    got = keyset(nl, ni, dim)
    assert all(k[0] >= 3 for k in got), got  # the three coarser neighbours were refined
    check_grid(got, dim, [1, 1], [False, False], {(1, 1)})


def test_removal_of_marked_children():
    dim, N = 2, 8
    lev, idx = uniform(2, 3)
    f = flags_zero(lev, N, dim)
    kids = [(3, 1, 1), (3, 2, 1), (3, 1, 2), (3, 2, 2)]
    for k in kids:
        f[leaf_index(lev, idx, k, dim)] = -1
    nl, ni = AD.adapt(dim, N, lev, idx, f)
    assert keyset(nl, ni, dim) == keyset(lev, idx, dim) - set(kids) | {(2, 1, 1)}
    # three of four marked: nothing removed
    f[leaf_index(lev, idx, kids[0], dim)] = 0
    nl, ni = AD.adapt(dim, N, lev, idx, f)
    assert keyset(nl, ni, dim) == keyset(lev, idx, dim)


def test_removal_blocked_by_neighbour_refinement():
    dim, N = 2, 8
    lev, idx = uniform(2, 3)
    f = flags_zero(lev, N, dim)
    kids = [(3, 1, 1), (3, 2, 1), (3, 1, 2), (3, 2, 2)]
    for k in kids:
        f[leaf_index(lev, idx, k, dim)] = -1
    q = leaf_index(lev, idx, (3, 3, 1), dim)  # touches (2,1,1) as a leaf of level 2
    set_cell(f, q, (4, 4), N, 1)
    nl, ni = AD.adapt(dim, N, lev, idx, f, n_buf=0)
    got = keyset(nl, ni, dim)
    assert (2, 1, 1) not in got and set(kids) <= got
    # a finer neighbour that already exists blocks it too
    lev2 = np.array([l for l, i in zip(lev, idx) if (l, i[0], i[1]) != (3, 3, 1)] + [4] * 4, np.int32)
    idx2 = np.array([i for l, i in zip(lev, idx) if (l, i[0], i[1]) != (3, 3, 1)]
                    + [[5 + a, 1 + b, 1] for a in (0, 1) for b in (0, 1)], np.int32)
    f2 = flags_zero(lev2, N, dim)
    for k in kids:
        f2[leaf_index(lev2, idx2, k, dim)] = -1
    nl, ni = AD.adapt(dim, N, lev2, idx2, f2)
    assert keyset(nl, ni, dim) == keyset(lev2, idx2, dim)


# ---------------------------------------------------------------------------
# random flags: properties
# ---------------------------------------------------------------------------
RANDOM = [
    (2, 8, lambda: W.ball_leaves(2, 8, 5, (0.3, 0.6), 0.0, 1), None, 1),
    (3, 4, lambda: W.ball_leaves(3, 4, 4, (0.3, 0.6, 0.4), 0.0, 1), None, 2),
    (2, 8, lambda: W.domain_leaves(2, 8, [(1, 1), (2, 1)], 4, (1.95, 0.4), periodic=(True, False, False)),
     (True, False, False), 3),
    (2, 8, lambda: W.domain_leaves(2, 8, [(1, 1), (2, 1), (1, 2)], 4, (0.97, 0.97)), None, 4),
]


@pytest.mark.parametrize("case", range(len(RANDOM)))
def test_random_flags_properties(case):
    dim, N, grid, periodic, seed = RANDOM[case]
    lev, idx = grid()
    rng = np.random.default_rng(seed)
    for trial in range(4):
        f = np.zeros((len(lev), N ** dim), np.int8)
        kind = rng.integers(0, 3, size=len(lev))  # 0 keep, 1 a few refine cells, 2 all derefine
        for q in range(len(lev)):
            if kind[q] == 1 and rng.random() < 0.15:
                f[q, rng.integers(0, N ** dim, size=2)] = 1
            elif kind[q] == 2:
                f[q] = -1
        nl, ni = AD.adapt(dim, N, lev, idx, f, n_buf=2, periodic=periodic)
        old, new = keyset(lev, idx, dim), keyset(nl, ni, dim)
        g = AD._Grid(dim, lev, idx, periodic)
        check_grid(new, dim, g.ext, g.periodic, g.roots)
        for key in old:
            q = leaf_index(lev, idx, key, dim)
            if (f[q] > 0).any():
                assert key not in new and all(c in new for c in g.children(key)), key
        for key in new - old:
            parent = (key[0] - 1,) + tuple((v + 1) // 2 for v in key[1:])
            if parent in old:
                continue  # a new child
            # a new parent: its children were all leaves, all fully marked
            for c in g.children(key):
                assert c in old and (f[leaf_index(lev, idx, c, dim)] < 0).all(), (key, c)
        for key in old - new:
            # at most one level of change at a location
            assert any(c in new for c in g.children(key)) or \
                (key[0] - 1,) + tuple((v + 1) // 2 for v in key[1:]) in new, key


# ---------------------------------------------------------------------------
# transfer
# ---------------------------------------------------------------------------
def linear(x):
    return 0.7 + 1.3 * x[..., 0] - 0.4 * x[..., 1] + (0.9 * x[..., 2] if x.shape[-1] == 3 else 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_transfer_is_exact_for_linear_fields(dim):
    N = 8
    lev, idx = W.ball_leaves(dim, N, 4 if dim == 3 else 5, (0.3, 0.6, 0.4), 0.0, 1)
    rng = np.random.default_rng(9)
    f = np.zeros((len(lev), N ** dim), np.int8)
    for q in rng.choice(len(lev), size=len(lev) // 4, replace=False):
        f[q, rng.integers(0, N ** dim)] = 1
    for q in range(len(lev)):
        if not f[q].any() and rng.random() < 0.5:
            f[q] = -1
    nl, ni = AD.adapt(dim, N, lev, idx, f)
    assert keyset(nl, ni, dim) != keyset(lev, idx, dim)
    old = O.Tree(dim, N, lev, idx)
    u = linear(W.cell_centres(dim, N, lev, idx))
    bc = np.zeros((len(lev), 2 * dim, N ** (dim - 1)))
    for s in range(2 * dim):
        bc[:, s, :] = linear(W.face_centres(dim, N, lev, idx, s))
    bc *= W.physical_side_mask(dim, lev, idx)[:, :, None]
    out = AD.transfer(old, nl, ni, u, bc)
    want = linear(W.cell_centres(dim, N, nl, ni))
    assert np.abs(out - want).max() <= 1e-13


def test_transfer_keeps_unchanged_leaves_and_constants():
    dim, N = 2, 8
    lev, idx = W.domain_leaves(2, 8, [(1, 1), (2, 1)], 4, (1.95, 0.4), periodic=(True, False, False))
    bct = ["periodic", "periodic", "neumann", "neumann"]
    rng = np.random.default_rng(4)
    f = np.zeros((len(lev), N * N), np.int8)
    f[rng.choice(len(lev), 5, replace=False), 10] = 1
    nl, ni = AD.adapt(dim, N, lev, idx, f, periodic=(True, False))
    old = O.Tree(dim, N, lev, idx, bc_type=bct)
    u = rng.standard_normal((len(lev), N * N))
    out = AD.transfer(old, nl, ni, u, None)
    new_keys = [(int(l), int(i[0]), int(i[1])) for l, i in zip(nl, ni)]
    for q, (l, i) in enumerate(zip(lev, idx)):
        key = (int(l), int(i[0]), int(i[1]))
        if key in new_keys:
            assert np.array_equal(out[new_keys.index(key)], u[q])
    old2 = O.Tree(dim, N, lev, idx, bc_type=bct)
    out = AD.transfer(old2, nl, ni, np.full((len(lev), N * N), 2.5), None)
    assert np.abs(out - 2.5).max() <= 1e-14
