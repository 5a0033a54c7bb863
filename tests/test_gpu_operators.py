"""GPU parity of the variable-coefficient and cylindrical operators (paper
§3.4, §3.5, §4.1 case 2): the HIP path through the C-ABI against the FP64
oracle on the same seeded inputs.

* steps (afmg_step): one half sweep, residual + restriction, FAS right-hand
  side + copy, prolongation (default and eps-weighted) and the coarse-grid
  V-cycle, each once on the GPU and once by the oracle on the same random
  state; bar 1e-13 of the output's max-norm (rounding order only: the GPU
  forms ghosts from interior values and contracts multiply-adds);
* solves: every leaf cell to 1e-12 of the largest value at equal cycle
  counts, the residual history per cycle, and equal cycle counts when
  solving to a tolerance;
* the paper's case 2 at its own configuration (N_down = N_up = 2,
  N_base = 4, boxes of 8^2, refinement h^2 |rho| / eps > 1e-3): parity, one
  FMG cycle within twice the discretisation error, every V-cycle reducing the
  residual;
* the entry point's checks: eps not positive, mixed precision, the adjoint,
  batches, a 3D cylindrical form; restoring the Laplacian.
"""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W
from parity import REL, assert_leaf_parity, assert_norms_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STEP_REL = 1e-13
D_, N_, P_ = "dirichlet", "neumann", "periodic"


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def cases():
    """name -> (dim, (level, idx), side types, operator, eps recipe)"""
    c = (0.3, 0.62, 0.41)
    return {
        "e2": (2, W.ball_leaves(2, 8, 5, c, 0.0, 1), None, "eps", "random"),
        "e3": (3, W.ball_leaves(3, 8, 4, c, 0.0, 1), None, "eps", "random"),
        "c2": (2, W.ball_leaves(2, 8, 5, (0.1, 0.4), 0.05, 1), [N_, D_, D_, N_], "cyl", None),
        "ce2": (2, W.ball_leaves(2, 8, 5, (0.25, 0.25), 0.02, 1), None, "cyl_eps", "jump"),
        "eL2": (2, W.domain_leaves(2, 8, [(1, 1), (2, 1), (1, 2)], 5, (0.97, 0.97)), [D_, N_, N_, D_], "eps",
                "random"),
        "ep3": (3, W.domain_leaves(3, 8, [(1, 1, 1), (2, 1, 1)], 4, (1.98, 0.4, 0.6), periodic=(True, False, False)),
                [P_, P_, N_, D_, D_, N_], "eps", "random"),
        # a level of more than 1024 boxes (2048 at level 5), where the half
        # sweep takes its row form, with refinement, Neumann and periodic sides
        "ep3big": (3, W.domain_leaves(3, 8, [(1, 1, 1), (2, 1, 1)], 5, (1.0, 0.45, 0.55), 0.4,
                                      periodic=(True, False, False)),
                   [P_, P_, N_, D_, D_, N_], "eps", "random"),
        # boxes of 16^D cells
        "e3x16": (3, W.ball_leaves(3, 16, 3, c, 0.0, 1), None, "eps", "random"),
        "ce2x16": (2, W.ball_leaves(2, 16, 4, (0.25, 0.25), 0.02, 1), None, "cyl_eps", "jump"),
    }


def box_n(name):
    return 16 if name.endswith("x16") else 8


_CASES = None


def get_case(name):
    global _CASES
    if _CASES is None:
        _CASES = cases()
    return _CASES[name]


def make_eps(recipe, dim, lev, idx, seed, n=8):
    if recipe is None:
        return None
    if recipe == "random":
        return W.random_eps(len(lev), n, dim, seed)
    return W.eps_sampled(W.case2_eps, dim, n, lev, idx)


def gpu_tree(dim, lev, idx, types, kind, eps_leaf, prolong, n=8):
    from paper_1701_04329_amd import afmg as A
    t = A.Tree(dim, lev, idx, box_n=n, bc_type=types)
    dev = torch.device("cuda", 0)
    e = None if eps_leaf is None else t.leaf_to_boxes(torch.tensor(eps_leaf, device=dev)).contiguous()
    t.set_operator(kind, e, prolong)
    return t


def oracle_tree(dim, lev, idx, types, kind, eps_leaf, prolong, n=8):
    o = O.Tree(dim, n, lev, idx, bc_type=types)
    o.set_operator(kind, eps_leaf, prolong)
    return o


# ---------------------------------------------------------------------------
# steps
# ---------------------------------------------------------------------------
class Pair:
    def __init__(self, name, seed, prolong="default"):
        from paper_1701_04329_amd import afmg as A
        self.A = A
        dim, (lev, idx), types, kind, recipe = get_case(name)
        self.dim, self.n = dim, box_n(name)
        n = self.n
        eps = make_eps(recipe, dim, lev, idx, 90 + seed, n)
        if eps is None and prolong == "eps":
            pytest.skip("the eps prolongation needs eps")
        self.t = gpu_tree(dim, lev, idx, types, kind, eps, prolong, n)
        self.o = oracle_tree(dim, lev, idx, types, kind, eps, prolong, n)
        C = n ** dim
        key_o = {}
        for b in range(self.o.nbox):
            i = self.o.box_info(b)
            if i["level"] >= 1:
                key_o[(i["level"], i["ix"], i["iy"], i["iz"])] = b
        self.o_of = np.array([key_o[(self.t.box(b)["level"],) + self.t.box(b)["idx"]]
                              for b in range(self.t.n_boxes)])
        rng = np.random.default_rng(seed)
        self.u = rng.standard_normal((self.t.n_boxes, C))
        self.rho = rng.standard_normal((self.t.n_boxes, C))
        self.uold = rng.standard_normal((self.t.n_boxes, C))
        phys = W.domain_side_mask(dim, lev, idx, types)[:, :, None]
        self.bc_leaf = rng.standard_normal((len(lev), 2 * dim, n ** (dim - 1))) * phys
        self.levels = np.array([self.t.box(b)["level"] for b in range(self.t.n_boxes)])
        self.leaf = np.array([self.t.box(b)["leaf"] for b in range(self.t.n_boxes)])

    def gpu(self, op, level, colour=0, homog=False):
        dev = torch.device("cuda", 0)
        u = torch.tensor(self.u, device=dev)
        rho = torch.tensor(self.rho, device=dev)
        uold = torch.tensor(self.uold, device=dev)
        bc = self.t.bc_rows(torch.tensor(self.bc_leaf, device=dev))
        self.A.step(self.t, op, level, u, rho, uold, bc, colour=colour, homog=homog)
        torch.cuda.synchronize()
        return u.cpu().numpy(), rho.cpu().numpy(), uold.cpu().numpy()

    def _set(self, field, arr):
        n = self.n
        inner = tuple(slice(1, -1) for _ in range(self.dim))
        for b in range(self.t.n_boxes):
            ob = int(self.o_of[b])
            p = self.o.box_padded(ob, field)
            p[inner] = arr[b].reshape((n,) * self.dim)
            self.o.set_box_padded(ob, p, field)

    def _get(self, field):
        inner = tuple(slice(1, -1) for _ in range(self.dim))
        return np.stack([self.o.box_padded(int(self.o_of[b]), field)[inner].ravel()
                         for b in range(self.t.n_boxes)])

    def oracle_state(self):
        self.o.load(self.rho[self.t.leaf_boxes], self.bc_leaf)
        self._set("u", self.u)
        self._set("rho", self.rho)
        self._set("uold", self.uold)

    def boxes(self, level, parents=None):
        sel = self.levels == level
        if parents is not None:
            sel &= self.leaf != parents
        return np.nonzero(sel)[0]


def close(what, got, ref, rel=STEP_REL):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    print(f"  {what}: max rel diff {err:.2e}", flush=True)
    assert err <= rel, (what, err)


STEP_NAMES = ["e2", "e3", "c2", "ce2", "eL2", "ep3", "ep3big", "e3x16", "ce2x16"]


@pytest.mark.parametrize("name", STEP_NAMES)
def test_operator_steps(name):
    for homog in (False, True):
        P = Pair(name, 3)
        for level in range(1, P.t.lmax + 1):
            for colour in (0, 1):
                announce(f"op half sweep {name} level {level} colour {colour} homog {homog}")
                u, _, _ = P.gpu("half_sweep", level, colour, homog)
                P.oracle_state()
                P.o.half_sweep(level, colour, homog=homog)
                bs = P.boxes(level)
                close("u", u[bs], P._get("u")[bs])
        for level in range(2, P.t.lmax + 1):
            announce(f"op residual + restriction {name} level {level} homog {homog}")
            u, rho, _ = P.gpu("resid_restrict", level, homog=homog)
            P.oracle_state()
            P.o.resid_restrict_level(level, homog=homog)
            par = P.boxes(level - 1, parents=True)
            close("parent u", u[par], P._get("u")[par])
            close("parent restricted residual", rho[par], P._get("res")[par])
        for level in range(2, P.t.lmax):
            announce(f"op coarse rhs {name} level {level} homog {homog}")
            _, rho, uold = P.gpu("coarse_rhs", level, homog=homog)
            P.oracle_state()
            P._set("res", P.rho)
            P.o.coarse_rhs_level(level, homog=homog)
            bs, par = P.boxes(level), P.boxes(level, parents=True)
            close("uold", uold[bs], P._get("uold")[bs])
            close("parent rho", rho[par], P._get("rho")[par])
        announce(f"op coarse grids {name} homog {homog}")
        u, _, uold = P.gpu("coarse", 1, homog=homog)
        P.oracle_state()
        P._set("res", P.rho)
        P.o.coarse_rhs_level(1, homog=homog)
        P.o.vcycle_from(1, homog=homog)
        root = P.boxes(1)
        close("level-1 u", u[root], P._get("u")[root])
        close("level-1 uold", uold[root], P._get("uold")[root])


@pytest.mark.parametrize("prolong", ["default", "eps"])
@pytest.mark.parametrize("name", ["e2", "e3", "ce2", "eL2", "e3x16"])
def test_operator_prolong_steps(name, prolong):
    P = Pair(name, 4, prolong)
    for level in range(2, P.t.lmax + 1):
        announce(f"op prolongation {name} {prolong} level {level}")
        u, _, _ = P.gpu("prolong", level)
        P.oracle_state()
        P._set("u", P.uold)
        P.o.fill_gc(level - 1, "u")
        P.o.copy_uold(level - 1)
        P._set("u", P.u)
        P.o.fill_gc(level - 1, "u")
        P.o.prolong_level(level)
        bs = P.boxes(level)
        close("u", u[bs], P._get("u")[bs])


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------
def inputs(dim, lev, idx, types, seed, singular=False, n=8):
    rng = np.random.default_rng(seed)
    rho = rng.standard_normal((len(lev), n ** dim))
    bc = rng.standard_normal((len(lev), 2 * dim, n ** (dim - 1)))
    bc *= W.domain_side_mask(dim, lev, idx, types)[:, :, None]
    return rho, bc


def solve_pair(name, prolong, seed, **kw):
    dim, (lev, idx), types, kind, recipe = get_case(name)
    n = box_n(name)
    eps = make_eps(recipe, dim, lev, idx, seed + 1, n)
    rho, bc = inputs(dim, lev, idx, types, seed, n=n)
    t = gpu_tree(dim, lev, idx, types, kind, eps, prolong, n)
    o = oracle_tree(dim, lev, idx, types, kind, eps, prolong, n)
    from paper_1701_04329_amd import afmg as A
    dev = torch.device("cuda", 0)
    announce(f"op solve {name} {kind} {prolong} {kw}")
    u, sg = A.solve(t, t.leaf_to_boxes(torch.tensor(rho, device=dev)),
                    t.bc_rows(torch.tensor(bc, device=dev)) if t.n_bfaces else None, None, **kw)
    torch.cuda.synchronize()
    ug = t.boxes_to_leaf(u).cpu().numpy()
    uo, so = o.solve(rho, bc, **kw)
    return ug, sg, uo, so


@pytest.mark.parametrize("prolong", ["default", "eps"])
@pytest.mark.parametrize("name", STEP_NAMES)
def test_operator_fixed_cycles_match_oracle(name, prolong):
    if prolong == "eps" and get_case(name)[4] is None:
        pytest.skip("the eps prolongation needs eps")
    for kw in (dict(fixed_cycles=3, n_base=16), dict(cycle="FMG", fixed_cycles=1, n_base=16)):
        ug, sg, uo, so = solve_pair(name, prolong, 41, **kw)
        assert_leaf_parity(ug, uo, REL, (name, prolong, kw))
        floor = 1e-12 * so["r0_max"]
        assert_norms_close(sg["hist_max"], so["hist_max"], floor, what=(name, "history max"))
        assert_norms_close(sg["hist_l2"], so["hist_l2"], 1e-12 * so["r0_l2"], what=(name, "history L2"))


@pytest.mark.parametrize("name", ["e3", "ce2", "eL2", "ep3big", "e3x16", "ce2x16"])
def test_operator_solve_to_tolerance_matches_oracle(name):
    ug, sg, uo, so = solve_pair(name, "default", 51, cycle="FMG", tol=1e-10, n_base=16, max_cycles=80)
    assert sg["status"] == 0 and so["status"] == 0, (sg["status"], so["status"])
    if sg["cycles"] != so["cycles"]:
        ratio = so["r_max"] / (1e-10 * so["r0_max"])
        assert abs(sg["cycles"] - so["cycles"]) == 1 and 0.99 < ratio < 1.01
    assert_leaf_parity(ug, uo, 1e-9, name)


def test_case2_paper_configuration():
    """§4.1 case 2 on the GPU: parity with the oracle at equal cycles, one
    FMG cycle within twice the discretisation error, each V(2,2) cycle
    reducing the residual."""
    from paper_1701_04329_amd import afmg as A
    w = W.case2_workload(lmax=7)
    dev = torch.device("cuda", 0)
    t = A.Tree(2, w.level, w.idx)
    t.set_operator("cyl_eps", t.leaf_to_boxes(torch.tensor(w.eps, device=dev)).contiguous())
    o = O.Tree(2, 8, w.level, w.idx)
    o.set_operator("cyl_eps", w.eps)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    announce("case 2 FMG + 6 V-cycles")
    u, st = A.solve(t, rho, bc, None, cycle="FMG", fixed_cycles=6)
    torch.cuda.synchronize()
    uo, so = o.solve(w.rho, w.bc, cycle="FMG", fixed_cycles=6)
    assert_leaf_parity(t.boxes_to_leaf(u).cpu().numpy(), uo, REL, "case 2")
    announce("case 2 converged and one FMG cycle")
    uc, sc = A.solve(t, rho, bc, None, cycle="FMG", tol=1e-12, max_cycles=60)
    assert sc["status"] == 0
    disc = np.abs(t.boxes_to_leaf(uc).cpu().numpy() - w.u_exact).max()
    uf, _ = A.solve(t, rho, bc, None, cycle="FMG", fixed_cycles=0, max_cycles=0)
    assert np.abs(t.boxes_to_leaf(uf).cpu().numpy() - w.u_exact).max() <= 2.0 * disc
    h = np.concatenate([[sc["r0_max"]], sc["hist_max"]])
    assert np.all(h[1:] < 0.5 * h[:-1]), h


def test_full_size_eps_jump_matches_oracle():
    """The benchmark's variable-coefficient workload at its full size: the
    uniform 256^3 octree with eps = 100 in [0, 1/2)^3 and 1 elsewhere (a jump
    across three coarse-grid faces), FMG + 2 V-cycles on the GPU and in the
    oracle; every leaf cell to 1e-12 of the largest value, residual history
    to 1e-12 of the initial residual."""
    from paper_1701_04329_amd import afmg as A
    w = W.config2()
    eps = W.eps_sampled(lambda x: np.where(np.all(x < 0.5, axis=-1), 100.0, 1.0), w.dim, w.N, w.level, w.idx)
    dev = torch.device("cuda", 0)
    t = A.Tree(w.dim, w.level, w.idx)
    t.set_operator("eps", t.leaf_to_boxes(torch.tensor(eps, device=dev)).contiguous())
    announce(f"full-size eps jump unknowns={w.n_unknowns}")
    u, sg = A.solve(t, t.leaf_to_boxes(torch.tensor(w.rho, device=dev)), t.bc_rows(torch.tensor(w.bc, device=dev)),
                    None, cycle="FMG", fixed_cycles=2)
    ug = t.boxes_to_leaf(u).cpu().numpy()
    del u
    o = O.Tree(w.dim, w.N, w.level, w.idx)
    o.set_operator("eps", eps)
    uo, so = o.solve(w.rho, w.bc, cycle="FMG", fixed_cycles=2)
    assert_leaf_parity(ug, uo, REL, "eps3d full size")
    assert_norms_close(sg["hist_max"], so["hist_max"], 1e-12 * so["r0_max"], what="eps3d history")


# ---------------------------------------------------------------------------
# the entry point's checks
# ---------------------------------------------------------------------------
def test_operator_validation_and_reset():
    from paper_1701_04329_amd import afmg as A
    dim, (lev, idx), types, kind, recipe = get_case("e2")
    dev = torch.device("cuda", 0)
    t = A.Tree(dim, lev, idx)
    e = t.leaf_to_boxes(torch.tensor(W.random_eps(len(lev), 8, dim, 3), device=dev)).contiguous()
    bad = e.clone()
    bad[int(t.leaf_boxes[2]), 7] = -1.0
    announce("operator validation")
    with pytest.raises(A.AfmgError):
        t.set_operator("eps", bad)
    with pytest.raises(A.AfmgError):
        t.set_operator("eps", None)
    with pytest.raises(A.AfmgError):
        t.set_operator("cyl", None, "eps")
    t3 = A.Tree(3, *W.uniform_leaves(3, 2))
    with pytest.raises(A.AfmgError):
        t3.set_operator("cyl")
    rho_leaf, bc_leaf = inputs(dim, lev, idx, None, 5)
    rho = t.leaf_to_boxes(torch.tensor(rho_leaf, device=dev))
    bc = t.bc_rows(torch.tensor(bc_leaf, device=dev))
    u0, _ = A.solve(t, rho, bc, None, fixed_cycles=2)
    t.set_operator("eps", e)
    with pytest.raises(A.AfmgError):
        A.solve(t, rho, bc, None, fixed_cycles=2, precision="mixed")
    with pytest.raises(A.AfmgError):
        A.adjoint(t, torch.zeros_like(rho))
    with pytest.raises(A.AfmgError):
        A.Batch([t])
    ue, _ = A.solve(t, rho, bc, None, fixed_cycles=2)
    assert not torch.equal(ue, u0)
    t.set_operator("laplacian")
    u1, _ = A.solve(t, rho, bc, None, fixed_cycles=2)
    assert torch.equal(u1, u0)
    # the allocation-free entry point takes the operator too
    t.set_operator("eps", e)
    t.finalize()
    un = torch.zeros_like(rho)
    A.solve_noalloc(t, rho, bc, un, fixed_cycles=2)
    torch.cuda.synchronize()
    assert torch.equal(un, ue)
