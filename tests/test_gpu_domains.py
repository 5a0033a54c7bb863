"""GPU parity on general domains (paper §2.2, §3, §3.2): coarse grids of
several level-1 boxes (rectangles, an L shape), Neumann and periodic sides,
refinement boundaries also across a periodic side.  The HIP path (through the
C-ABI) against the FP64 oracle on the same seeded inputs: every leaf cell to
1e-12 of the largest value at equal cycle counts, residual norms per cycle,
and equal cycle counts when solving to a tolerance.  Problems without a
Dirichlet side are singular: their rho is made compatible and both sides run
the same iteration, so the iterates (constant included) still agree."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W
from parity import REL, assert_leaf_parity, assert_norms_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D_, N_, P_ = "dirichlet", "neumann", "periodic"


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def cases():
    out = {}
    lev, idx = W.domain_leaves(2, 8, [(1, 1), (2, 1), (1, 2)], 6, (0.97, 0.97))
    out["L2"] = (lev, idx, 2, [D_, N_, N_, D_])
    lev, idx = W.domain_leaves(2, 8, [(1, 1), (2, 1)], 6, (1.98, 0.3), periodic=(True, False, False))
    out["px2"] = (lev, idx, 2, [P_, P_, D_, N_])
    lev, idx = W.domain_leaves(2, 8, [(1, 1), (2, 1), (3, 1)], 5, (0.1, 0.8))
    out["n2"] = (lev, idx, 2, N_)
    lev, idx = W.domain_leaves(3, 8, [(1, 1, 1), (2, 1, 1)], 4, (1.0, 0.4, 0.6))
    out["n3"] = (lev, idx, 3, [N_, D_, D_, D_, N_, N_])
    lev, idx = W.domain_leaves(3, 8, [(1, 1, 1), (2, 1, 1)], 4, (1.95, 0.5, 0.02), periodic=(True, True, True))
    out["p3"] = (lev, idx, 3, P_)
    lev, idx = W.uniform_leaves(3, 4)
    out["u3n"] = (lev, idx, 3, [N_, N_, N_, N_, D_, D_])
    return out


CASES = None


def get(name, seed=None):
    global CASES
    if CASES is None:
        CASES = cases()
    lev, idx, dim, types = CASES[name]
    w = W.domain_fields(dim, 8, lev, idx, 700 + sorted(CASES).index(name) if seed is None else seed, types)
    return w, types


def gpu_solve(w, types, **kw):
    from paper_1701_04329_amd import afmg as A
    t = A.Tree(w.dim, w.level, w.idx, bc_type=types)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev)) if t.n_bfaces else None
    u, st = A.solve(t, rho, bc, None, **kw)
    torch.cuda.synchronize()
    return t.boxes_to_leaf(u).cpu().numpy(), st, t


def check_pair(name, **kw):
    w, types = get(name)
    announce(f"{name} {types} n_leaves={w.n_leaves} opts={kw}")
    ug, sg, t = gpu_solve(w, types, **kw)
    uo, so = O.Tree(w.dim, w.N, w.level, w.idx, bc_type=types).solve(w.rho, w.bc, **kw)
    assert_leaf_parity(ug, uo, REL, (name, kw))
    np.testing.assert_allclose(sg["r0_max"], so["r0_max"], rtol=1e-12)
    np.testing.assert_allclose(sg["r0_l2"], so["r0_l2"], rtol=1e-12)
    h_min = 1.0 / (w.N * 2.0 ** (w.lmax - 1))
    floor = 16 * np.finfo(float).eps * 2 * w.dim / h_min ** 2 * np.abs(uo).max()
    if kw.get("fixed_cycles", 0) == 0:
        tol = kw.get("tol", 1e-10)
        assert sg["status"] == so["status"] == 0, (sg["status"], so["status"])
        if sg["cycles"] != so["cycles"]:
            ratio = so["r_max"] / (tol * so["r0_max"])
            assert abs(sg["cycles"] - so["cycles"]) == 1 and 0.99 < ratio < 1.01, (sg["cycles"], so["cycles"])
        floor = max(floor, 1e-2 * tol * so["r0_max"])
    n = min(sg["cycles"], so["cycles"])
    assert_norms_close(sg["hist_max"][:n], so["hist_max"][:n], floor, what=(name, "history max"))
    assert_norms_close(sg["hist_l2"][:n], so["hist_l2"][:n], floor, what=(name, "history L2"))
    return ug, sg, uo, so, t


NAMES = ["L2", "px2", "n2", "n3", "p3", "u3n"]


@pytest.mark.parametrize("name", NAMES)
def test_domain_fixed_cycles_match_oracle(name):
    check_pair(name, fixed_cycles=3, n_base=16)
    check_pair(name, cycle="FMG", fixed_cycles=1, n_base=16)


@pytest.mark.parametrize("name", NAMES)
def test_domain_solve_to_tolerance_matches_oracle(name):
    ug, sg, uo, so, t = check_pair(name, cycle="FMG", tol=1e-10, n_base=32, max_cycles=60)
    assert t.singular == (name in ("n2", "p3"))


def test_domain_default_n_base_converges_on_square_ends():
    """the default N_base = 4 on a 2x1 coarse grid with mixed sides"""
    check_pair("L2", tol=1e-10)


@pytest.mark.parametrize("name", ["L2", "n3", "u3n"])
def test_domain_mixed_precision(name):
    """FP32 V-cycles inside FP64 refinement on general domains, against the
    oracle's FP64 solve (the mixed bound, about 1e-10 relative)."""
    from paper_1701_04329_amd import afmg as A
    w, types = get(name)
    announce(f"mixed {name} {types}")
    t = A.Tree(w.dim, w.level, w.idx, bc_type=types)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    u, st = A.solve(t, rho, bc, cycle="FMG", tol=1e-10, precision="mixed", n_base=32)
    um = t.boxes_to_leaf(u).cpu().numpy()
    uo, so = O.Tree(w.dim, w.N, w.level, w.idx, bc_type=types).solve(w.rho, w.bc, cycle="FMG", tol=1e-10,
                                                                       n_base=32)
    err = np.linalg.norm(um - uo) / np.linalg.norm(uo)
    print(f"mixed {name}: outer={st['cycles']} oracle cycles={so['cycles']} rel-L2 {err:.2e}", flush=True)
    assert st["status"] == 0 and st["r_max"] <= 1e-10 * st["r0_max"]
    assert err <= 1e-8


@pytest.mark.parametrize("name", ["L2", "n3"])
def test_domain_adjoint_matches_oracle(name):
    """Gradients with Neumann sides (dl/dq = -lambda / h on Neumann rows,
    -2 lambda / h^2 on Dirichlet ones) against the oracle's sparse L^T
    solve."""
    from paper_1701_04329_amd import afmg as A
    w, types = get(name)
    announce(f"adjoint {name} {types}")
    t = A.Tree(w.dim, w.level, w.idx, bc_type=types)
    dev = torch.device("cuda", 0)
    ot = O.Tree(w.dim, w.N, w.level, w.idx, bc_type=types)
    rng = np.random.default_rng(9)
    ubar = rng.standard_normal(w.rho.shape)
    lam_o, gb_o = O.adjoint(ot, ubar)
    rho_bar, bc_bar, st = A.adjoint(t, t.leaf_to_boxes(torch.tensor(ubar, device=dev)), tol=1e-12, max_cycles=400)
    assert st["status"] == 0, st
    lam = t.boxes_to_leaf(rho_bar).cpu().numpy()
    assert np.abs(lam - lam_o).max() <= 1e-9 * np.abs(lam_o).max()
    bcb = bc_bar.cpu().numpy()
    leaf_of_box = {int(b): q for q, b in enumerate(t.leaf_boxes)}
    gb_rows = gb_o[[leaf_of_box[int(b)] for b in t.bfaces[:, 0]], t.bfaces[:, 1]]
    assert np.abs(bcb - gb_rows).max() <= 1e-9 * np.abs(gb_rows).max()


def test_singular_domain_rejects_adjoint():
    from paper_1701_04329_amd import afmg as A
    w, types = get("p3")
    t = A.Tree(w.dim, w.level, w.idx, bc_type=types)
    dev = torch.device("cuda", 0)
    with pytest.raises(A.AfmgError):
        A.adjoint(t, torch.zeros((t.n_boxes, t.cells_per_box), dtype=torch.float64, device=dev))


def test_periodic_solution_is_periodic_shift_invariant():
    """A fully periodic uniform grid over a 2x1 coarse grid: shifting rho by
    one level-1 box along the periodic axis shifts the solution (up to its
    free constant), a property that holds at any size."""
    from paper_1701_04329_amd import afmg as A
    lev, idx = W.uniform_leaves(3, 3)
    idx2 = np.concatenate([idx, idx + np.array([4, 0, 0], np.int32)])
    lev2 = np.concatenate([lev, lev])
    w = W.domain_fields(3, 8, lev2, idx2, 77, P_)
    n = len(lev)
    rho_shift = np.concatenate([w.rho[n:], w.rho[:n]])
    dev = torch.device("cuda", 0)
    t = A.Tree(3, lev2, idx2, bc_type=P_)
    announce("periodic shift")
    sols = []
    for rho in (w.rho, rho_shift):
        r = t.leaf_to_boxes(torch.tensor(rho, device=dev))
        u, st = A.solve(t, r, None, cycle="FMG", tol=1e-11, n_base=32)
        assert st["status"] == 0
        x = t.boxes_to_leaf(u).cpu().numpy()
        sols.append(x - x.mean())
    back = np.concatenate([sols[1][n:], sols[1][:n]])
    assert np.abs(back - sols[0]).max() <= 1e-9 * np.abs(sols[0]).max()
