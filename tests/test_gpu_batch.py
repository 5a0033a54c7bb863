"""Batched solves on the GPU (afmg_batch_*): every tree of a batch against
its own unbatched GPU solve and against the FP64 oracle.

A batch runs each tree through exactly the iteration afmg_solve runs on it
alone, so the bar against the unbatched solve is bitwise: equal leaf
solutions, cycle counts, statuses and max-norm histories (the max-norm is
exact in any reduction order; the L2 norm is summed in another order and
agrees to 1e-12).  Against the oracle the single-tree bar applies: relative
L2 difference <= 1e-12 at equal cycle counts."""

import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W
from parity import assert_leaf_parity, assert_norms_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-12
DEV = None


def dev():
    return torch.device("cuda", 0)


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def single(w, **kw):
    from paper_1701_04329_amd import afmg as A
    t = A.Tree(w.dim, w.level, w.idx, box_n=w.N)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev()))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev()))
    u0 = kw.pop("u0", None)
    u = t.leaf_to_boxes(torch.tensor(u0, device=dev())) if u0 is not None else None
    u, st = A.solve(t, rho, bc, u, **kw)
    torch.cuda.synchronize()
    return t.boxes_to_leaf(u).cpu().numpy(), st


def batched(ws, u0s=None, **kw):
    from paper_1701_04329_amd import afmg as A
    trees = [A.Tree(w.dim, w.level, w.idx, box_n=w.N) for w in ws]
    b = A.Batch(trees)
    rho = b.concat([t.leaf_to_boxes(torch.tensor(w.rho, device=dev())) for t, w in zip(trees, ws)])
    bc = b.concat_bc([t.bc_rows(torch.tensor(w.bc, device=dev())) for t, w in zip(trees, ws)])
    u = None
    if u0s is not None:
        u = b.concat([t.leaf_to_boxes(torch.tensor(x, device=dev())) for t, x in zip(trees, u0s)])
    u, sts = A.solve_batch(b, rho, bc, u, **kw)
    torch.cuda.synchronize()
    return [t.boxes_to_leaf(x).cpu().numpy() for t, x in zip(trees, b.split(u))], sts


def zero_tree(dim):
    w = W.random_fields(dim, 8, *W.uniform_leaves(dim, 2), 13)
    w.rho[:] = 0.0
    w.bc[:] = 0.0
    w.name = f"zero_{dim}d"
    return w


def bag(dim):
    """Trees of unequal shape: the root alone (lmax 1), refinement boundaries
    at several levels with random rho and Dirichlet values, Gaussian sources,
    a tree whose zero data converge before the first cycle, trees of the
    batch workload recipe at reduced size, and a uniform two-level tree."""
    c = (0.3, 0.62, 0.41)
    ws = [
        W.random_fields(dim, 8, *W.uniform_leaves(dim, 1), 11),
        W.random_fields(dim, 8, *W.ball_leaves(dim, 8, 4 if dim == 3 else 6, c, 0.0, 1), 12),
        W.adaptive_small(dim, 8, 5 if dim == 3 else 7, 1e-3, 6, n_src=2,
                         sigma_range=(0.04, 0.08) if dim == 3 else (0.03, 0.06)),
        zero_tree(dim),
    ]
    js = [j for j in range(40) if (j % 2 == 0) == (dim == 2)][:3]
    ws += [W.config4_tree(j, box_range=(64, 400 if dim == 3 else 1500), seed_base=4100) for j in js]
    # uniform level 2 with data: its V-cycles start at level 2 while deeper
    # trees of the batch arrive there from level 3
    ws.append(W.random_fields(dim, 8, *W.uniform_leaves(dim, 2), 14))
    return ws


def assert_same(ub, sb, us, ss, name):
    assert np.array_equal(ub, us), (name, np.abs(ub - us).max())
    assert sb["status"] == ss["status"] and sb["cycles"] == ss["cycles"], (name, sb, ss)
    assert sb["r0_max"] == ss["r0_max"], name
    assert np.array_equal(sb["hist_max"], ss["hist_max"]), name
    np.testing.assert_allclose(sb["hist_l2"], ss["hist_l2"], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("cycle", ["V", "FMG"])
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_equals_unbatched(dim, cycle, precision):
    ws = bag(dim)
    announce(f"batch vs unbatched dim={dim} {cycle} {precision} trees={len(ws)}")
    ub, sb = batched(ws, cycle=cycle, precision=precision, tol=1e-10)
    cyc = []
    for w, u, s in zip(ws, ub, sb):
        us, ss = single(w, cycle=cycle, precision=precision, tol=1e-10)
        assert_same(u, s, us, ss, w.name)
        cyc.append(s["cycles"])
    print(f"cycles per tree {cyc}", flush=True)
    # the zero tree stops before its first cycle while the others iterate
    assert cyc[3] == 0 and max(cyc) >= 5


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_matches_oracle(dim):
    ws = bag(dim)
    announce(f"batch vs oracle dim={dim}")
    ub, sb = batched(ws, cycle="FMG", fixed_cycles=3)
    for w, u, s in zip(ws, ub, sb):
        uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="FMG", fixed_cycles=3)
        nrm = np.linalg.norm(uo)
        if nrm == 0.0:
            assert not u.any(), w.name
            continue
        assert_leaf_parity(u, uo, REL, w.name)
        np.testing.assert_allclose(s["r0_max"], so["r0_max"], rtol=1e-12)
        np.testing.assert_allclose(s["r0_l2"], so["r0_l2"], rtol=1e-12)
        floor = 16 * np.finfo(float).eps * 2 * w.dim * (w.N * 2.0 ** (w.lmax - 1)) ** 2 * np.abs(uo).max()
        assert_norms_close(s["hist_max"], so["hist_max"], floor, what=w.name)
        assert_norms_close(s["hist_l2"], so["hist_l2"], floor, what=w.name)
        assert s["cycles"] == so["cycles"] == 3


def bag16(dim):
    """Trees of 16^D-cell boxes (2D: forest kernels with 16 boxes per
    workgroup; 3D: one box per workgroup, level 2 box by box and levels
    <= 1 in the coarse kernel): the root alone, refinement boundaries at
    several levels, Gaussian sources, zero data, a uniform two-level tree."""
    c = (0.3, 0.62, 0.41)
    ws = [
        W.random_fields(dim, 16, *W.uniform_leaves(dim, 1), 21),
        W.random_fields(dim, 16, *W.ball_leaves(dim, 16, 5 if dim == 2 else 3, c, 0.0, 1), 22),
        W.adaptive_small(dim, 16, 6 if dim == 2 else 4, 1e-3, 6, n_src=2,
                         sigma_range=(0.03, 0.06) if dim == 2 else (0.04, 0.08)),
        W.random_fields(dim, 16, *W.uniform_leaves(dim, 2), 23),
    ]
    ws[3].rho[:] = 0.0
    ws[3].bc[:] = 0.0
    ws.append(W.random_fields(dim, 16, *W.uniform_leaves(dim, 2), 24))
    return ws


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_of_16_cell_boxes(dim, precision):
    """Boxes of 16^D cells: each tree bitwise as solved alone, and FP64
    against the oracle at a fixed cycle count."""
    ws = bag16(dim)
    announce(f"batch of 16^D-cell boxes dim={dim} {precision} trees={len(ws)}")
    ub, sb = batched(ws, cycle="FMG", precision=precision, tol=1e-10)
    for w, u, s in zip(ws, ub, sb):
        us, ss = single(w, cycle="FMG", precision=precision, tol=1e-10)
        assert_same(u, s, us, ss, w.name)
    assert sb[3]["cycles"] == 0 and max(s["cycles"] for s in sb) >= 5
    if precision == "fp64":
        ub, sb = batched(ws, cycle="FMG", fixed_cycles=3)
        for w, u, s in zip(ws, ub, sb):
            uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="FMG", fixed_cycles=3)
            if np.linalg.norm(uo) == 0.0:
                assert not u.any(), w.name
                continue
            assert_leaf_parity(u, uo, REL, w.name)


def test_batch_use_guess_and_single_tree_batch():
    ws = bag(3)[:3]
    rng = np.random.default_rng(5)
    u0s = [rng.standard_normal(w.rho.shape) for w in ws]
    announce("batch with initial guess")
    ub, sb = batched(ws, u0s=u0s, cycle="V", tol=1e-10)
    for w, u0, u, s in zip(ws, u0s, ub, sb):
        us, ss = single(w, u0=u0, cycle="V", tol=1e-10)
        assert_same(u, s, us, ss, w.name)
    announce("batch of one tree")
    w = ws[2]
    ub, sb = batched([w], cycle="FMG", tol=1e-10)
    us, ss = single(w, cycle="FMG", tol=1e-10)
    assert_same(ub[0], sb[0], us, ss, w.name)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(precision):
    """The recorded cycle replayed many times, with eager work between the
    replays and between solves: every solve equals the unrecorded one."""
    from paper_1701_04329_amd import afmg as A
    w = W.adaptive_small(3, 8, 5, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    t = A.Tree(w.dim, w.level, w.idx)
    rng = np.random.default_rng(9)
    bc = t.bc_rows(torch.tensor(w.bc, device=dev()))
    ws_bytes = t.workspace_bytes(A.make_opts(precision=precision))
    work = torch.empty(ws_bytes, dtype=torch.uint8, device=dev())
    u = torch.empty((t.n_boxes, t.cells_per_box), dtype=torch.float64, device=dev())
    for rep in range(3):
        announce(f"graph replay {precision} solve {rep}")
        rho = t.leaf_to_boxes(torch.tensor(w.rho * (1.0 + rep) + rng.standard_normal(w.rho.shape), device=dev()))
        u_ref, s_ref = A.solve(t, rho, bc, None, cycle="FMG", precision=precision, use_guess=False)
        junk = torch.randn(1 << 20, device=dev(), dtype=torch.float64)
        junk.mul_(2.0).sum().item()  # eager work between solves
        u, s = A.solve(t, rho, bc, u, cycle="FMG", precision=precision, use_guess=False, graph=True,
                       workspace=work)
        torch.cuda.synchronize()
        assert torch.equal(u, u_ref), rep
        assert s["cycles"] == s_ref["cycles"] >= 5
        assert np.array_equal(s["hist_max"], s_ref["hist_max"])
    announce(f"graph requested while profiling {precision}")
    u_e, s_e = A.solve(t, rho, bc, None, cycle="FMG", precision=precision, use_guess=False, profile=True)
    u_g, s_g = A.solve(t, rho, bc, u, cycle="FMG", precision=precision, use_guess=False, graph=True,
                       profile=True, workspace=work)
    torch.cuda.synchronize()
    assert torch.equal(u_e, u_g)
    assert s_g["prof_n"] == s_e["prof_n"] and s_e["prof_n"][0] > 0
    assert all(x > 0.0 for x, n in zip(s_g["prof_ms"], s_g["prof_n"]) if n)
    announce(f"graph replay batch {precision}")
    ws = bag(2)
    ub, sb = batched(ws, cycle="V", precision=precision, tol=1e-10)
    ug, sg = batched(ws, cycle="V", precision=precision, tol=1e-10, graph=True)
    for w, a, sa, b_, sb_ in zip(ws, ub, sb, ug, sg):
        assert_same(b_, sb_, a, sa, w.name)


def test_full_batch_workload_sampled():
    """The full batch workload (256 trees of 64-8192 boxes, D alternating),
    in the configuration the benchmark times (FMG then V-cycles to 1e-10,
    mixed precision, recorded cycles).  Sampled trees are compared with their
    unbatched solves bitwise and the smallest with the oracle."""
    from paper_1701_04329_amd import afmg as A
    workers = min(16, os.cpu_count() or 1)
    announce(f"full batch workload: generating 256 trees with {workers} workers")
    ws = W.config4(256, workers=workers)
    for dim in (2, 3):
        sub = [w for w in ws if w.dim == dim]
        announce(f"full batch dim={dim} trees={len(sub)} unknowns={sum(w.n_unknowns for w in sub)}")
        ub, sb = batched(sub, cycle="FMG", precision="mixed", tol=1e-10, graph=True)
        assert all(s["status"] == 0 for s in sb)
        order = np.argsort([w.n_unknowns for w in sub])
        for q in (order[0], order[len(order) // 2], order[-1]):
            us, ss = single(sub[q], cycle="FMG", precision="mixed", tol=1e-10)
            assert_same(ub[q], sb[q], us, ss, sub[q].name)
        w = sub[order[0]]
        uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="FMG", tol=1e-10)
        err = np.linalg.norm(ub[order[0]] - uo) / np.linalg.norm(uo)
        print(f"dim={dim} smallest tree {w.name}: mixed batch vs FP64 oracle {err:.2e}", flush=True)
        assert err <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_check_every(precision):
    """Reading the norms every k cycles runs the same cycles: at equal cycle
    counts the solution is bitwise that of checking every cycle, the checked
    history entries are equal and the others NaN, and a tolerance stop lands
    on the first check at or after the cycle where every-cycle checking
    stops.  Batches check every tree on the device after every cycle."""
    w = W.adaptive_small(3, 8, 5, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    announce(f"check_every {precision}")
    u1, s1 = single(w, cycle="FMG", precision=precision, fixed_cycles=6)
    u3, s3 = single(w, cycle="FMG", precision=precision, fixed_cycles=6, check_every=3)
    assert np.array_equal(u1, u3) and s3["cycles"] == 6
    assert np.isnan(s3["hist_max"][[0, 1, 3, 4]]).all()
    assert np.array_equal(s3["hist_max"][[2, 5]], s1["hist_max"][[2, 5]])
    ut, st = single(w, cycle="FMG", precision=precision, tol=1e-10)
    u2, s2 = single(w, cycle="FMG", precision=precision, tol=1e-10, check_every=4)
    expect = -(-st["cycles"] // 4) * 4
    assert s2["status"] == 0 and s2["cycles"] == expect, (st["cycles"], s2["cycles"])
    uf, sf = single(w, cycle="FMG", precision=precision, fixed_cycles=expect)
    assert np.array_equal(u2, uf)
    # batches apply every tree's stop test on the device after every cycle:
    # whatever the interval of host synchronisations, each tree runs the
    # cycles of its own solve with per-cycle checking, full history included
    ws = bag(3)
    ref = [single(x, cycle="V", precision=precision, tol=1e-10) for x in ws]
    for every in (1, 2, 5):
        ub, sb = batched(ws, cycle="V", precision=precision, tol=1e-10, check_every=every, graph=True)
        for x, ux, sx, (us, ss) in zip(ws, ub, sb, ref):
            assert np.array_equal(ux, us) and sx["cycles"] == ss["cycles"], (x.name, every)
            assert np.array_equal(sx["hist_max"], ss["hist_max"]), (x.name, every)
            assert not np.isnan(sx["hist_max"]).any()
