"""Mixed precision on the GPU: FP32 V-cycles inside FP64 iterative
refinement (residual, correction update and coarsest grids in FP64).

There is no FP32 oracle: the mixed solution is compared with the FP64
oracle's solution at the same 1e-10 residual reduction, and the difference is
printed per case.  Both stop at a residual 1e-10 below the initial one, so
their difference is of the order of 1e-10 relative; the bound asserted here
is 1e-8.  Refinement with an FP64 residual converges at the rate of the
inner V-cycle, so the outer iteration count may exceed the FP64 cycle count
by at most two."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W
from parity import assert_leaf_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOUND = 1e-8


def run_mixed(w, **kw):
    from paper_1701_04329_amd import afmg as A
    t = A.Tree(w.dim, w.level, w.idx, box_n=w.N)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev)) if t.n_bfaces else None
    u, st = A.solve(t, rho, bc, precision="mixed", **kw)
    torch.cuda.synchronize()
    return t.boxes_to_leaf(u).cpu().numpy(), st


CASES = {
    "u3_64": lambda: W.config2(res=64),
    "c1": lambda: W.config1(),
    "a3": lambda: W.adaptive_small(3, 8, 5, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08)),
    "a2": lambda: W.adaptive_small(2, 8, 7, 1e-3, 5, n_src=2, sigma_range=(0.03, 0.06)),
    "b3_rand": lambda: W.random_fields(3, 8, *W.ball_leaves(3, 8, 5, (0.3, 0.62, 0.41), 0.0, 2), 77),
    "single_3d": lambda: W.random_fields(3, 8, *W.uniform_leaves(3, 1), 93),
    # boxes of 16^D cells: a complete finest level (the fused refinement
    # update), an adaptive octree (general coarse kernel), a quadtree
    "u3x16_64": lambda: W.config2(N=16, res=64),
    "a3x16": lambda: W.adaptive_small(3, 16, 4, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08)),
    "a2x16": lambda: W.adaptive_small(2, 16, 6, 1e-3, 5, n_src=2, sigma_range=(0.03, 0.06)),
}


@pytest.mark.parametrize("cycle", ["V", "FMG"])
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_matches_fp64_oracle(name, cycle):
    w = CASES[name]()
    print(f"[case] mixed {name} {cycle} leaves={w.n_leaves}", flush=True)
    um, sm = run_mixed(w, cycle=cycle, tol=1e-10)
    uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle=cycle, tol=1e-10)
    assert sm["status"] == 0, sm
    assert sm["r_max"] <= 1e-10 * sm["r0_max"]
    err = np.linalg.norm(um - uo) / np.linalg.norm(uo)
    print(f"mixed {name} {cycle}: outer={sm['cycles']} fp64 cycles={so['cycles']} "
          f"rel-L2 vs FP64 oracle {err:.2e}", flush=True)
    sys.stdout.flush()
    assert err <= BOUND
    assert sm["cycles"] <= so["cycles"] + 2
    np.testing.assert_allclose(sm["r0_max"], so["r0_max"], rtol=1e-12)


def test_full_size_adaptive_fp64_and_mixed_against_oracle():
    """The adaptive benchmark octree at full size (about 2.3e7 unknowns on
    leaves of levels 3-8): FP64 at a fixed cycle count against the oracle to
    1e-12, and the mixed refinement at a 1e-10 residual reduction against the
    oracle's FP64 solve to the mixed bound."""
    from paper_1701_04329_amd import afmg as A
    w = W.config3()
    print(f"[case] full-size adaptive {w.name} unknowns={w.n_unknowns}", flush=True)
    t = A.Tree(w.dim, w.level, w.idx)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    ot = O.Tree(w.dim, w.N, w.level, w.idx)
    u, s = A.solve(t, rho, bc, cycle="FMG", fixed_cycles=2)
    ug = t.boxes_to_leaf(u).cpu().numpy()
    uo, so = ot.solve(w.rho, w.bc, cycle="FMG", fixed_cycles=2)
    err, emax = assert_leaf_parity(ug, uo, 1e-12, "FP64 FMG+2V")
    print(f"FP64 FMG+2V vs oracle: rel-L2 {err:.2e}, max per cell {emax:.2e}", flush=True)
    np.testing.assert_allclose(s["r0_max"], so["r0_max"], rtol=1e-12)
    np.testing.assert_allclose(s["r0_l2"], so["r0_l2"], rtol=1e-12)
    u, s = A.solve(t, rho, bc, cycle="FMG", tol=1e-10, precision="mixed")
    um = t.boxes_to_leaf(u).cpu().numpy()
    uo, so = ot.solve(w.rho, w.bc, cycle="FMG", tol=1e-10)
    err = np.linalg.norm(um - uo) / np.linalg.norm(uo)
    print(f"mixed to 1e-10: outer={s['cycles']} fp64 oracle cycles={so['cycles']} rel-L2 {err:.2e}", flush=True)
    assert s["status"] == 0 and s["r_max"] <= 1e-10 * s["r0_max"]
    assert err <= BOUND
    assert s["cycles"] <= so["cycles"] + 2


def test_full_size_uniform_256_mixed_tuned_against_oracle():
    """The benchmark workload (uniform 256^3) in the mixed path as the
    benchmark runs it: autotuned launch shapes, FMG then refinement to a
    1e-10 residual reduction, the refinement update riding on the last half
    sweep of each correction.  The whole leaf solution against the oracle's
    FP64 solve to the mixed bound, and bitwise against the same solve with
    the default shapes."""
    from paper_1701_04329_amd import afmg as A
    w = W.config2()
    print(f"[case] full-size uniform mixed {w.name} unknowns={w.n_unknowns}", flush=True)
    dev = torch.device("cuda", 0)
    t = A.Tree(w.dim, w.level, w.idx)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    u_def, s_def = A.solve(t, rho, bc, cycle="FMG", tol=1e-10, precision="mixed")
    t.autotune(dev)
    u, s = A.solve(t, rho, bc, cycle="FMG", tol=1e-10, precision="mixed")
    torch.cuda.synchronize()
    assert torch.equal(u, u_def) and s["cycles"] == s_def["cycles"]
    um = t.boxes_to_leaf(u).cpu().numpy()
    uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="FMG", tol=1e-10)
    err = np.linalg.norm(um - uo) / np.linalg.norm(uo)
    print(f"mixed 256^3: outer={s['cycles']} fp64 oracle cycles={so['cycles']} rel-L2 {err:.2e}", flush=True)
    assert s["status"] == 0 and s["r_max"] <= 1e-10 * s["r0_max"]
    assert err <= BOUND
    assert s["cycles"] <= so["cycles"] + 2


@pytest.mark.parametrize("cycle", ["V", "FMG"])
def test_mixed_solution_independent_of_workspace_contents(cycle):
    """Every correction solve starts from e = 0 whatever the workspace held
    before: the solve itself zeroes e before the first V-cycle (FMG zeroes it
    on its own), and the refinement update clears e on the leaves it adds.
    A workspace filled with NaN bytes, and one left by a previous solve of
    other data, give bitwise the solution of a fresh zeroed workspace."""
    from paper_1701_04329_amd import afmg as A
    w = CASES["a3"]()
    print(f"[case] mixed workspace reuse {cycle} leaves={w.n_leaves}", flush=True)
    dev = torch.device("cuda", 0)
    t = A.Tree(w.dim, w.level, w.idx)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    nbytes = t.workspace_bytes(A.make_opts(cycle, 2, 2, 4, 1e-10, 100, 0, False, "mixed", False, False, 1))
    results = []
    for fill in ("zero", "nan", "reused"):
        ws = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=dev)
        if fill == "nan":
            ws.fill_(0xFF)  # every FP32 and FP64 word a NaN
        elif fill == "reused":
            A.solve(t, 3.0 * rho + 1.0, bc, cycle=cycle, precision="mixed", tol=1e-10, workspace=ws)
        u, st = A.solve(t, rho, bc, cycle=cycle, precision="mixed", tol=1e-10, workspace=ws)
        torch.cuda.synchronize()
        assert st["status"] == 0, (fill, st)
        results.append((fill, u.clone(), st["cycles"]))
    for fill, u, cycles in results[1:]:
        print(f"{fill}: cycles {cycles} vs {results[0][2]}", flush=True)
        assert cycles == results[0][2], fill
        assert torch.equal(u, results[0][1]), fill


@pytest.mark.parametrize("name,n_down,n_up", [("u3_64", 1, 3), ("u3_64", 0, 2), ("u3_64", 2, 0),
                                              ("u2_5", 1, 1)])
def test_mixed_fused_update_smoothing_counts(name, n_down, n_up):
    """On a tree whose leaves all lie on its complete finest level the
    refinement update rides on the last half sweep of each correction, and
    the next correction's first half sweep takes its colour's old values as
    zero; without post- or pre-smoothing steps on that level the separate
    update runs instead.  Each case against the FP64 oracle with the same
    smoothing counts, at a 1e-8 residual reduction with the bound 1e-6 (the
    margin of 100 of the cases above)."""
    w = W.random_fields(2, 8, *W.uniform_leaves(2, 5), 95) if name == "u2_5" else CASES[name]()
    print(f"[case] mixed {name} V({n_down},{n_up})", flush=True)
    um, sm = run_mixed(w, cycle="V", tol=1e-8, n_down=n_down, n_up=n_up, max_cycles=200)
    uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="V", tol=1e-8, n_down=n_down,
                                                       n_up=n_up, max_cycles=200)
    assert sm["status"] == 0, sm
    err = np.linalg.norm(um - uo) / np.linalg.norm(uo)
    print(f"mixed {name} V({n_down},{n_up}): outer={sm['cycles']} fp64 cycles={so['cycles']} "
          f"rel-L2 vs FP64 oracle {err:.2e}", flush=True)
    assert err <= 1e-6
    assert sm["cycles"] <= so["cycles"] + 2
