"""Kernel-by-kernel parity: every step of the cycle (one half sweep, residual
+ restriction, FAS right-hand side + copy v', prolongation + correction, the
coarse-grid V-cycle of levels <= 1) run once through the C-ABI (afmg_step)
and once by the oracle on the same random state, with refinement boundaries
at the level under test and non-zero or zero boundary values; on the unit
square / cube with Dirichlet sides and on general domains (coarse grids of
several level-1 boxes, Neumann and periodic sides, paper §2.2, §3).

The GPU stores no ghost layers: it forms the ghosts from interior values
(and the ghosts of u - v' from interior differences) where the oracle fills
stored layers, so the two differ only in rounding order.  Bar: max-norm
difference <= 1e-14 of the output's max-norm."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-14


_G = {}


def grids(name):
    """name -> (dim, box size N, (level, idx), side types or None)"""
    if name in _G:
        return _G[name]
    c = (0.3, 0.62, 0.41)
    D_, N_, P_ = "dirichlet", "neumann", "periodic"
    make = {
        "a3": lambda: (3, 8, W.ball_leaves(3, 8, 5, c, 0.0, 1), None),
        "a2": lambda: (2, 8, W.ball_leaves(2, 8, 6, c, 0.0, 1), None),
        "u3": lambda: (3, 8, W.uniform_leaves(3, 3), None),
        # L-shaped coarse grid, refinement at the re-entrant corner, mixed sides
        "L2": lambda: (2, 8, W.domain_leaves(2, 8, [(1, 1), (2, 1), (1, 2)], 5, (0.97, 0.97)), [D_, N_, N_, D_]),
        # 2x1 coarse grid periodic in x, refinement across the periodic side
        "p3": lambda: (3, 8, W.domain_leaves(3, 8, [(1, 1, 1), (2, 1, 1)], 4, (1.98, 0.4, 0.6),
                                             periodic=(True, False, False)), [P_, P_, N_, D_, D_, N_]),
        # one level-1 box, Neumann sides along x and y
        "n3": lambda: (3, 8, W.ball_leaves(3, 8, 4, c, 0.0, 1), [N_, N_, N_, N_, D_, D_]),
        # boxes of 16^D cells (paper §2.1: N is a parameter): 3D trees take
        # the general coarse kernel, 2D trees the one-tree coarse kernel
        "a3x16": lambda: (3, 16, W.ball_leaves(3, 16, 4, c, 0.0, 1), None),
        "a2x16": lambda: (2, 16, W.ball_leaves(2, 16, 5, c, 0.0, 1), None),
        "u3x16": lambda: (3, 16, W.uniform_leaves(3, 2), None),
        "p3x16": lambda: (3, 16, W.domain_leaves(3, 16, [(1, 1, 1), (2, 1, 1)], 3, (1.98, 0.4, 0.6),
                                                 periodic=(True, False, False)), [P_, P_, N_, D_, D_, N_]),
    }
    _G[name] = make[name]()
    return _G[name]


NAMES = ["a3", "a2", "u3", "L2", "p3", "n3", "a3x16", "a2x16", "u3x16", "p3x16"]


class Pair:
    """The same tree in the library and in the oracle, with a random state."""

    def __init__(self, name, seed):
        from paper_1701_04329_amd import afmg as A
        self.A = A
        dim, n, (lev, idx), types = grids(name)
        self.dim, self.N = dim, n
        self.t = A.Tree(dim, lev, idx, box_n=n, bc_type=types)
        self.o = O.Tree(dim, n, lev, idx, bc_type=types)
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
        self.lev, self.idx = lev, idx

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
        n = self.N
        shape = (n + 2,) * self.dim
        for b in range(self.t.n_boxes):
            ob = int(self.o_of[b])
            p = self.o.box_padded(ob, field)
            inner = tuple(slice(1, -1) for _ in range(self.dim))
            p[inner] = arr[b].reshape((n,) * self.dim)
            self.o.set_box_padded(ob, p.reshape(shape), field)

    def _get(self, field):
        inner = tuple(slice(1, -1) for _ in range(self.dim))
        return np.stack([self.o.box_padded(int(self.o_of[b]), field)[inner].ravel()
                         for b in range(self.t.n_boxes)])

    def oracle_state(self):
        leaf_rho = self.rho[self.t.leaf_boxes]
        self.o.load(leaf_rho, self.bc_leaf)
        self._set("u", self.u)
        self._set("rho", self.rho)
        self._set("uold", self.uold)

    def boxes(self, level, parents=None):
        out = []
        for b in range(self.t.n_boxes):
            d = self.t.box(b)
            if d["level"] == level and (parents is None or parents != d["leaf"]):
                out.append(b)
        return np.array(out, dtype=np.int64)


def close(name, got, ref):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    print(f"  {name}: max rel diff {err:.2e}", flush=True)
    assert err <= REL, (name, err)


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("homog", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_half_sweep_steps(name, homog):
    P = Pair(name, 1)
    for level in range(1, P.t.lmax + 1):
        for colour in (0, 1):
            announce(f"half sweep {name} level {level} colour {colour} homog {homog}")
            u, _, _ = P.gpu("half_sweep", level, colour, homog)
            P.oracle_state()
            P.o.half_sweep(level, colour, homog=homog)
            bs = P.boxes(level)
            close("u", u[bs], P._get("u")[bs])
            others = np.setdiff1d(np.arange(P.t.n_boxes), bs)
            assert np.array_equal(u[others], P.u[others])


@pytest.mark.parametrize("homog", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_resid_restrict_steps(name, homog):
    P = Pair(name, 2)
    for level in range(2, P.t.lmax + 1):
        announce(f"residual + restriction {name} level {level} homog {homog}")
        u, rho, _ = P.gpu("resid_restrict", level, homog=homog)
        P.oracle_state()
        P.o.resid_restrict_level(level, homog=homog)
        par = P.boxes(level - 1, parents=True)
        close("parent u", u[par], P._get("u")[par])
        close("parent restricted residual", rho[par], P._get("res")[par])


@pytest.mark.parametrize("homog", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_coarse_rhs_steps(name, homog):
    P = Pair(name, 3)
    for level in range(2, P.t.lmax):
        announce(f"coarse rhs {name} level {level} homog {homog}")
        _, rho, uold = P.gpu("coarse_rhs", level, homog=homog)
        P.oracle_state()
        P._set("res", P.rho)  # the restricted residual, kept in rho on the GPU
        P.o.coarse_rhs_level(level, homog=homog)
        bs, par = P.boxes(level), P.boxes(level, parents=True)
        close("uold", uold[bs], P._get("uold")[bs])
        close("parent rho", rho[par], P._get("rho")[par])
        leaves = P.boxes(level, parents=False)
        assert np.array_equal(rho[leaves], P.rho[leaves])


@pytest.mark.parametrize("homog", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_prolong_steps(name, homog):
    P = Pair(name, 4)
    for level in range(2, P.t.lmax + 1):
        announce(f"prolongation {name} level {level} homog {homog}")
        u, _, _ = P.gpu("prolong", level, homog=homog)
        P.oracle_state()
        # the oracle's v' keeps the ghost layer of its copy: fill the ghosts
        # of v' (all levels) as the cycle did when it copied, then restore u
        P._set("u", P.uold)
        P.o.fill_gc(level - 1, "u", homog=homog)
        P.o.copy_uold(level - 1)
        P._set("u", P.u)
        P.o.fill_gc(level - 1, "u", homog=homog)
        P.o.prolong_level(level)
        bs = P.boxes(level)
        close("u", u[bs], P._get("u")[bs])


@pytest.mark.parametrize("homog", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_coarse_grid_step(name, homog):
    P = Pair(name, 5)
    announce(f"coarse grids {name} homog {homog}")
    u, _, uold = P.gpu("coarse", 1, homog=homog)
    P.oracle_state()
    P._set("res", P.rho)
    P.o.coarse_rhs_level(1, homog=homog)
    P.o.vcycle_from(1, homog=homog)
    root = P.boxes(1)
    close("level-1 u", u[root], P._get("u")[root])
    close("level-1 uold", uold[root], P._get("uold")[root])
