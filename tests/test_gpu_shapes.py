"""Launch shapes on the GPU: every workgroup size (64, 128, 256 threads) and
box order (XCD runs or launch order) of the per-level kernels computes
bitwise the same solve, so the autotuner may pick any of them; autotuned
trees and batches reproduce the default solves bitwise."""

import sys

import numpy as np
import pytest

from paper_1701_04329_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def grid(dim):
    if dim == 3:
        return W.random_fields(3, 8, *W.ball_leaves(3, 8, 5, (0.3, 0.62, 0.41), 0.0, 1), 21)
    return W.random_fields(2, 8, *W.ball_leaves(2, 8, 7, (0.3, 0.62, 0.41), 0.0, 1), 22)


def solve(t, w, **kw):
    from paper_1701_04329_amd import afmg as A
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    u, st = A.solve(t, rho, bc, None, **kw)
    torch.cuda.synchronize()
    return u, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_every_shape_gives_identical_solves(dim, precision):
    from paper_1701_04329_amd import afmg as A
    w = grid(dim)
    t = A.Tree(w.dim, w.level, w.idx)
    announce(f"shapes dim={dim} {precision} default")
    u0, s0 = solve(t, w, cycle="FMG", precision=precision, tol=1e-10)
    assert s0["cycles"] >= 5
    for wg in (64, 128, 256):
        for nr in (0, 1):
            announce(f"shapes dim={dim} {precision} wg={wg} no_remap={nr}")
            t.set_shape(wg, nr)
            u, s = solve(t, w, cycle="FMG", precision=precision, tol=1e-10)
            assert torch.equal(u, u0), (wg, nr)
            assert s["cycles"] == s0["cycles"]
            assert np.array_equal(s["hist_max"], s0["hist_max"])


@pytest.mark.parametrize("dim", [2, 3])
def test_shapes_of_16_cell_boxes(dim):
    """Boxes of 16^D cells: in 2D (16 threads per box) every shape gives the
    default solve bitwise; in 3D a box fills a 256-thread workgroup, so the
    smaller workgroups are refused and the autotuner keeps 256."""
    from paper_1701_04329_amd import afmg as A
    c = (0.3, 0.62, 0.41)
    w = W.random_fields(dim, 16, *W.ball_leaves(dim, 16, 4 if dim == 3 else 6, c, 0.0, 1), 25)
    t = A.Tree(w.dim, w.level, w.idx, box_n=16)
    announce(f"16-cell boxes shapes dim={dim} default")
    ref = {p: solve(t, w, cycle="FMG", precision=p, tol=1e-10) for p in ("fp64", "mixed")}
    wgs = (64, 128, 256) if dim == 2 else (256,)
    for p in ("fp64", "mixed"):
        for wg in wgs:
            for nr in (0, 1):
                announce(f"16-cell boxes dim={dim} {p} wg={wg} no_remap={nr}")
                t.set_shape(wg, nr)
                u, s = solve(t, w, cycle="FMG", precision=p, tol=1e-10)
                assert torch.equal(u, ref[p][0]), (p, wg, nr)
                assert np.array_equal(s["hist_max"], ref[p][1]["hist_max"])
    if dim == 3:
        for wg in (64, 128):
            with pytest.raises(A.AfmgError):
                t.set_shape(wg, 0)
    t.set_shape(256, 0)
    shapes = t.autotune()
    for vals in shapes.values():
        assert all(wg in wgs and nr in (0, 1) for wg, nr in vals)
    for p in ("fp64", "mixed"):
        u, s = solve(t, w, cycle="FMG", precision=p, tol=1e-10, graph=True)
        assert torch.equal(u, ref[p][0]), p


@pytest.mark.parametrize("dim", [2, 3])
def test_autotuned_tree_and_batch_reproduce_default(dim):
    from paper_1701_04329_amd import afmg as A
    w = grid(dim)
    t = A.Tree(w.dim, w.level, w.idx)
    ref = {p: solve(t, w, cycle="FMG", precision=p, tol=1e-10) for p in ("fp64", "mixed")}
    announce(f"autotune tree dim={dim}")
    shapes = t.autotune()
    print(f"tuned shapes: {shapes}", flush=True)
    for vals in shapes.values():
        assert all(wg in (64, 128, 256) and nr in (0, 1) for wg, nr in vals)
    for p in ("fp64", "mixed"):
        u, s = solve(t, w, cycle="FMG", precision=p, tol=1e-10, graph=True)
        assert torch.equal(u, ref[p][0]), p
        assert np.array_equal(s["hist_max"], ref[p][1]["hist_max"])
    announce(f"autotune batch dim={dim}")
    ws = [w, W.random_fields(dim, 8, *W.uniform_leaves(dim, 3), 23)]
    trees = [A.Tree(x.dim, x.level, x.idx) for x in ws]
    b = A.Batch(trees)
    dev = torch.device("cuda", 0)
    rho = b.concat([tr.leaf_to_boxes(torch.tensor(x.rho, device=dev)) for tr, x in zip(trees, ws)])
    bc = b.concat_bc([tr.bc_rows(torch.tensor(x.bc, device=dev)) for tr, x in zip(trees, ws)])
    u_def, _ = A.solve_batch(b, rho, bc, None, cycle="FMG", precision="mixed", tol=1e-10)
    b.autotune()
    u_tun, _ = A.solve_batch(b, rho, bc, None, cycle="FMG", precision="mixed", tol=1e-10, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(u_def, u_tun)
