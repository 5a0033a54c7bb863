"""GPU mesh adaptation and field transfer (paper §2.3, §2.5) against the
oracle, through the C-ABI:

* afmg_tree_adapt: the leaves of the adapted tree equal the oracle's,
  bit-exact (integer work), on quadtrees and octrees, an L-shaped coarse
  grid and periodic domains, for random refine / derefine flags and buffer
  widths 0, 1 and 2;
* afmg_tree_transfer: every leaf value of the target equals the oracle's
  transfer to 1e-14 of the largest value (copies bitwise), with boundary
  values in the prolongation ghosts; a linear field is carried exactly;
* the adapted tree solves, with the transferred solution as initial guess;
* the entry points' checks.
"""

import sys

import numpy as np
import pytest

from oracle import adapt as AD
from oracle import oracle as O
from paper_1701_04329_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D_, N_, P_ = "dirichlet", "neumann", "periodic"


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def grids():
    """name -> (dim, (level, idx), side types, periodic axes)"""
    c = (0.3, 0.62, 0.41)
    return {
        "a2": (2, W.ball_leaves(2, 8, 6, c, 0.0, 1), None, None),
        "a3": (3, W.ball_leaves(3, 8, 4, c, 0.0, 1), None, None),
        "L2": (2, W.domain_leaves(2, 8, [(1, 1), (2, 1), (1, 2)], 5, (0.97, 0.97)), [D_, N_, N_, D_], None),
        "p2": (2, W.domain_leaves(2, 8, [(1, 1), (2, 1)], 5, (1.97, 0.5), periodic=(True, False, False)),
               [P_, P_, D_, N_], (True, False)),
        "p3": (3, W.domain_leaves(3, 8, [(1, 1, 1), (2, 1, 1)], 4, (1.98, 0.4, 0.6), periodic=(True, True, True)),
               P_, (True, True, True)),
        # boxes of 16^D cells
        "a2x16": (2, W.ball_leaves(2, 16, 5, c, 0.0, 1), None, None),
        "a3x16": (3, W.ball_leaves(3, 16, 3, c, 0.0, 1), None, None),
    }


def box_n(name):
    return 16 if name.endswith("x16") else 8


_G = None


def grid(name):
    global _G
    if _G is None:
        _G = grids()
    return _G[name]


def random_flags(n, C, rng, p_ref=0.2, p_der=0.4):
    f = np.zeros((n, C), np.int8)
    for q in range(n):
        r = rng.random()
        if r < p_ref:
            f[q, rng.integers(0, C, size=2)] = 1
        elif r < p_ref + p_der:
            f[q] = -1
            if rng.random() < 0.2:
                f[q, rng.integers(0, C)] = 0
    return f


def keys_of(level, idx, dim):
    return [(int(l),) + tuple(int(v) for v in i[:dim]) for l, i in zip(level, np.asarray(idx).reshape(-1, 3))]


def gpu_tree(name):
    from paper_1701_04329_amd import afmg as A
    dim, (lev, idx), types, _ = grid(name)
    return A.Tree(dim, lev, idx, box_n=box_n(name), bc_type=types)


NAMES = ["a2", "a3", "L2", "p2", "p3", "a2x16", "a3x16"]


@pytest.mark.parametrize("name", NAMES)
def test_adapt_matches_oracle(name):
    from paper_1701_04329_amd import afmg as A
    dim, (lev, idx), types, periodic = grid(name)
    t = gpu_tree(name)
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(sorted(NAMES).index(name) + 11)
    n = box_n(name)
    for trial, n_buf in enumerate((2, 1, 0, 2)):
        f = random_flags(len(lev), n ** dim, rng)
        announce(f"adapt {name} trial {trial} n_buf {n_buf}")
        nt, counts = A.adapt(t, t.leaf_to_boxes(torch.tensor(f, device=dev)).contiguous(), n_buf=n_buf)
        ol, oi = AD.adapt(dim, n, lev, idx, f, n_buf=n_buf, periodic=periodic)
        gl, gi = nt.leaves()
        assert sorted(keys_of(gl, gi, dim)) == sorted(keys_of(ol, oi, dim)), (name, trial)
        assert nt.n_leaves == len(ol)
        assert counts[0] > 0 or counts[1] > 0


@pytest.mark.parametrize("name", NAMES)
def test_transfer_matches_oracle(name):
    from paper_1701_04329_amd import afmg as A
    dim, (lev, idx), types, periodic = grid(name)
    t = gpu_tree(name)
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(31 + sorted(NAMES).index(name))
    n = box_n(name)
    f = random_flags(len(lev), n ** dim, rng)
    nt, _ = A.adapt(t, t.leaf_to_boxes(torch.tensor(f, device=dev)).contiguous())
    u = rng.standard_normal((len(lev), n ** dim))
    bc = rng.standard_normal((len(lev), 2 * dim, n ** (dim - 1)))
    bc *= W.domain_side_mask(dim, lev, idx, types)[:, :, None]
    for with_bc in (True, False):
        announce(f"transfer {name} bc {with_bc}")
        ug = A.transfer(t, nt, t.leaf_to_boxes(torch.tensor(u, device=dev)),
                        t.bc_rows(torch.tensor(bc, device=dev)) if (with_bc and t.n_bfaces) else None)
        torch.cuda.synchronize()
        gl, gi = nt.leaves()
        got = dict(zip(keys_of(gl, gi, dim), nt.boxes_to_leaf(ug).cpu().numpy()))
        ol, oi = AD.adapt(dim, n, lev, idx, f, periodic=periodic)
        ot = O.Tree(dim, n, lev, idx, bc_type=types)
        uo = AD.transfer(ot, ol, oi, u, bc if with_bc else None)
        scale = np.abs(uo).max()
        old_keys = dict(zip(keys_of(lev, idx, dim), u))
        for k, row in zip(keys_of(ol, oi, dim), uo):
            assert np.abs(got[k] - row).max() <= 1e-14 * scale, (name, k)
            if k in old_keys:
                assert np.array_equal(got[k], old_keys[k])


@pytest.mark.parametrize("dim", [2, 3])
def test_transfer_linear_field_exact(dim):
    from paper_1701_04329_amd import afmg as A
    name = "a2" if dim == 2 else "a3"
    _, (lev, idx), _, _ = grid(name)
    t = gpu_tree(name)
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    f = random_flags(len(lev), 8 ** dim, rng)

    def lin(x):
        return 0.3 - 0.8 * x[..., 0] + 1.1 * x[..., 1] + (0.5 * x[..., 2] if dim == 3 else 0.0)

    bc = np.zeros((len(lev), 2 * dim, 8 ** (dim - 1)))
    for s in range(2 * dim):
        bc[:, s, :] = lin(W.face_centres(dim, 8, lev, idx, s))
    bc *= W.physical_side_mask(dim, lev, idx)[:, :, None]
    nt, _ = A.adapt(t, t.leaf_to_boxes(torch.tensor(f, device=dev)).contiguous())
    announce(f"transfer linear {dim}D")
    ug = A.transfer(t, nt, t.leaf_to_boxes(torch.tensor(lin(W.cell_centres(dim, 8, lev, idx)), device=dev)),
                    t.bc_rows(torch.tensor(bc, device=dev)))
    gl, gi = nt.leaves()
    want = lin(W.cell_centres(dim, 8, gl, gi))
    assert np.abs(nt.boxes_to_leaf(ug).cpu().numpy() - want).max() <= 1e-13


def test_adapted_tree_solves_from_transferred_guess():
    """Time-stepping use: adapt to a moved source, carry the solution over,
    solve again from it; the guess starts closer than zero."""
    from paper_1701_04329_amd import afmg as A
    dev = torch.device("cuda", 0)
    w = W.adaptive_small(2, 8, 6, 1e-3, 5, n_src=2, sigma_range=(0.03, 0.06))
    t = A.Tree(2, w.level, w.idx)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    u, st = A.solve(t, rho, bc, None, cycle="FMG", tol=1e-10)
    assert st["status"] == 0
    # refine where |rho| h^2 is largest, derefine where it is tiny
    h = W.box_h(w.level, 8)[:, None]
    crit = np.abs(w.rho) * h ** 2
    f = np.where(crit > 3e-4, 1, np.where(crit < 1e-6, -1, 0)).astype(np.int8)
    nt, counts = A.adapt(t, t.leaf_to_boxes(torch.tensor(f, device=dev)).contiguous())
    announce(f"adapt + transfer + solve, refined {counts[0]} removed {counts[1]}")
    assert counts[0] > 0
    u2 = A.transfer(t, nt, u, bc)
    nl, ni = nt.leaves()
    w2 = W.sample_workload("moved", 2, 8, nl, ni, w.mix)
    rho2 = nt.leaf_to_boxes(torch.tensor(w2.rho, device=dev))
    bc2 = nt.bc_rows(torch.tensor(w2.bc, device=dev))
    _, s_guess = A.solve(nt, rho2, bc2, u2.clone(), cycle="V", tol=1e-10, use_guess=True)
    _, s_zero = A.solve(nt, rho2, bc2, None, cycle="V", tol=1e-10)
    assert s_guess["status"] == 0 and s_zero["status"] == 0
    assert s_guess["r0_max"] < s_zero["r0_max"]


def test_full_size_adaptation():
    """The benchmark's adaptation at full size (the adaptive octree of about
    2.3e7 unknowns, sources moved by 0.02, refine above 1e-4 and derefine
    below 1e-6 of |lap u| h^2): the adapted leaves equal the oracle's, bit
    for bit; the transferred field keeps every surviving leaf bitwise, and a
    leaf whose children were removed holds their mean (restriction, §2.5)."""
    from paper_1701_04329_amd import afmg as A
    dev = torch.device("cuda", 0)
    w = W.config3()
    moved = W.GaussMix(w.mix.centres + np.array([0.02, 0.0, 0.0]), w.mix.sigmas, w.mix.amps)
    crit = np.abs(moved.laplacian(W.cell_centres(w.dim, w.N, w.level, w.idx))) * (W.box_h(w.level, w.N)[:, None] ** 2)
    fine = (w.level < w.lmax)[:, None]
    flags = np.where((crit > 1e-4) & fine, 1, np.where(crit < 1e-6, -1, 0)).astype(np.int8)
    del crit
    t = A.Tree(w.dim, w.level, w.idx)
    announce(f"full-size adaptation leaves={w.n_leaves}")
    nt, counts = A.adapt(t, t.leaf_to_boxes(torch.tensor(flags, device=dev)).contiguous(), n_buf=2)
    ol, oi = AD.adapt(3, 8, w.level, w.idx, flags, n_buf=2)
    gl, gi = nt.leaves()
    assert sorted(keys_of(gl, gi, 3)) == sorted(keys_of(ol, oi, 3))
    assert counts[0] > 0 and counts[1] > 0
    # a field with distinct values per cell, carried over
    rng = np.random.default_rng(7)
    u = rng.standard_normal((w.n_leaves, 512))
    ug = nt.boxes_to_leaf(A.transfer(t, nt, t.leaf_to_boxes(torch.tensor(u, device=dev)))).cpu().numpy()
    old = {k: q for q, k in enumerate(keys_of(w.level, w.idx, 3))}
    new_keys = keys_of(gl, gi, 3)
    n_same = n_coarse = 0
    for q, k in enumerate(new_keys):
        if k in old:
            assert np.array_equal(ug[q], u[old[k]]), k
            n_same += 1
            continue
        kids = [(k[0] + 1, 2 * k[1] - 1 + a, 2 * k[2] - 1 + b, 2 * k[3] - 1 + c)
                for c in (0, 1) for b in (0, 1) for a in (0, 1)]
        if all(c in old for c in kids):
            # the parent's cell (I, J, K) is the mean of the 2x2x2 block of its child's cells
            want = np.zeros((8, 8, 8))
            for kid in kids:
                v = u[old[kid]].reshape(8, 8, 8)  # (z, y, x)
                blk = v.reshape(4, 2, 4, 2, 4, 2).mean(axis=(1, 3, 5))
                ox, oy, oz = (kid[1] - 1) % 2 * 4, (kid[2] - 1) % 2 * 4, (kid[3] - 1) % 2 * 4
                want[oz:oz + 4, oy:oy + 4, ox:ox + 4] = blk
            np.testing.assert_allclose(ug[q].reshape(8, 8, 8), want, rtol=0, atol=1e-14 * np.abs(u).max())
            n_coarse += 1
    print(f"kept {n_same}, coarsened {n_coarse}, refined {len(new_keys) - n_same - n_coarse}", flush=True)
    assert n_coarse == counts[1]


def test_adapt_and_transfer_checks():
    from paper_1701_04329_amd import afmg as A
    dev = torch.device("cuda", 0)
    t = gpu_tree("a2")
    f = torch.zeros((t.n_boxes, 64), dtype=torch.int8, device=dev)
    with pytest.raises(A.AfmgError):
        A.adapt(t, f, n_buf=9)
    nt, counts = A.adapt(t, f)
    assert counts == (0, 0) and nt.n_leaves == t.n_leaves
    other = A.Tree(2, *W.uniform_leaves(2, 2))
    u = torch.zeros((t.n_boxes, 64), dtype=torch.float64, device=dev)
    with pytest.raises(A.AfmgError):
        # leaves of t two levels and more below other's leaves
        A.transfer(other, t, torch.zeros((other.n_boxes, 64), dtype=torch.float64, device=dev))
    with pytest.raises(A.AfmgError):
        A.transfer(t, gpu_tree("L2"), u)  # another domain
