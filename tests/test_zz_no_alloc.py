"""The allocation-free entry point afmg_solve_noalloc (workspace in the
library's scratch array) against afmg_solve with a caller workspace: bitwise
the same solution and statistics, on two calls in a row with the second on a
smaller tree, in FP64 and mixed precision, and against the oracle."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W
from parity import REL, assert_leaf_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def setup(w):
    from paper_1701_04329_amd import afmg as A
    t = A.Tree(w.dim, w.level, w.idx)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev)) if t.n_bfaces else None
    return t, rho, bc


def cases():
    big = W.adaptive_small(3, 8, 5, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    small = W.adaptive_small(2, 8, 6, 1e-3, 5, n_src=2, sigma_range=(0.03, 0.06))
    return [big, small]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("cycle,kw", [("FMG", dict(tol=1e-10)), ("V", dict(fixed_cycles=3))])
def test_noalloc_equals_solve_on_two_calls(precision, cycle, kw):
    from paper_1701_04329_amd import afmg as A
    ws = cases()
    assert ws[1].n_unknowns < ws[0].n_unknowns
    for call, w in enumerate(ws):
        announce(f"noalloc call {call} {w.name} unknowns={w.n_unknowns} {precision} {cycle} {kw}")
        t, rho, bc = setup(w)
        t.finalize()
        assert t.workspace_bytes(A.make_opts(precision=precision)) <= A.SCRATCH_BYTES
        u_ref, s_ref = A.solve(t, rho, bc, cycle=cycle, precision=precision, **kw)
        u = torch.full_like(rho, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        rc, st = A.solve_noalloc(t, rho, bc, u, cycle=cycle, precision=precision, **kw)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        if call > 0:
            # the scratch array is in place after the first call on the device
            assert free1 == free0, (free0, free1)
        assert rc == s_ref["rc"] == A.AFMG_OK
        assert torch.equal(u, u_ref), float((u - u_ref).abs().max())
        assert st["cycles"] == s_ref["cycles"] and st["status"] == s_ref["status"]
        assert np.array_equal(st["hist_max"], s_ref["hist_max"])
        assert st["r0_max"] == s_ref["r0_max"] and st["r_max"] == s_ref["r_max"]
        if precision == "fp64":
            uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle=cycle, **kw)
            assert_leaf_parity(t.boxes_to_leaf(u).cpu().numpy(), uo, REL, w.name)


def test_noalloc_argument_errors():
    from paper_1701_04329_amd import afmg as A
    w = cases()[1]
    t, rho, bc = setup(w)
    u = torch.zeros_like(rho)
    announce("noalloc: unprepared tree")
    rc, _ = A.solve_noalloc(t, rho, bc, u, check=False)
    assert rc == A.AFMG_ERR_ARG and "afmg_tree_finalize" in A.last_error()
    t.finalize()
    announce("noalloc: graph / profile")
    o = A.make_opts(graph=True)
    st = A.Stats()
    import ctypes as C
    s = torch.cuda.current_stream()
    rc = A.lib().afmg_solve_noalloc(t.handle, C.c_void_p(s.cuda_stream), C.c_void_p(rho.data_ptr()),
                                    C.c_void_p(bc.data_ptr()), C.c_void_p(u.data_ptr()), C.byref(o), C.byref(st))
    assert rc == A.AFMG_ERR_ARG
    announce("noalloc: tree larger than the scratch array")
    lev, idx = W.uniform_leaves(3, 6)
    big = A.Tree(3, lev, idx)
    assert big.workspace_bytes(A.make_opts()) > A.SCRATCH_BYTES
    big.finalize()
    rb = torch.zeros((big.n_boxes, big.cells_per_box), dtype=torch.float64, device=rho.device)
    rc, _ = A.solve_noalloc(big, rb, None, torch.zeros_like(rb), check=False)
    assert rc == A.AFMG_ERR_ARG and "scratch" in A.last_error()
    # the tree still solves through the workspace entry point, and a small
    # tree through the scratch array afterwards
    announce("noalloc: small tree after the rejected one")
    u_ref, _ = A.solve(t, rho, bc, fixed_cycles=2)
    rc, _ = A.solve_noalloc(t, rho, bc, u, fixed_cycles=2)
    assert rc == A.AFMG_OK and torch.equal(u, u_ref)


def test_noalloc_box16_and_operator_trees():
    """Boxes of 16^D cells, then a smaller tree with the paper's cylindrical
    variable-coefficient operator (§3.4, §3.5; its general coarse kernel keeps
    its grids in the workspace when they leave LDS) through the scratch
    array: bitwise afmg_solve's solution and statistics on both calls."""
    from paper_1701_04329_amd import afmg as A
    dev = torch.device("cuda", 0)
    a = W.adaptive_small(3, 16, 4, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    c = W.case2_workload(lmax=7)
    assert c.n_unknowns < a.n_unknowns
    t1 = A.Tree(3, a.level, a.idx, box_n=16)
    t2 = A.Tree(2, c.level, c.idx)
    t2.set_operator("cyl_eps", t2.leaf_to_boxes(torch.tensor(c.eps, device=dev)).contiguous())
    for call, (t, w) in enumerate(((t1, a), (t2, c))):
        announce(f"noalloc call {call} {w.name} box_n={t.box_n} unknowns={w.n_unknowns}")
        t.finalize()
        assert t.workspace_bytes(A.make_opts()) <= A.SCRATCH_BYTES
        rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
        bc = t.bc_rows(torch.tensor(w.bc, device=dev)) if t.n_bfaces else None
        u_ref, s_ref = A.solve(t, rho, bc, cycle="FMG", tol=1e-10)
        u = torch.full_like(rho, float("nan"))
        rc, st = A.solve_noalloc(t, rho, bc, u, cycle="FMG", tol=1e-10)
        torch.cuda.synchronize()
        assert rc == s_ref["rc"] == A.AFMG_OK
        assert torch.equal(u, u_ref), float((u - u_ref).abs().max())
        assert st["cycles"] == s_ref["cycles"] and st["status"] == s_ref["status"]
        assert np.array_equal(st["hist_max"], s_ref["hist_max"])
        assert st["r0_max"] == s_ref["r0_max"] and st["r_max"] == s_ref["r_max"]
