"""Pins of the oracle's alternative schemes (paper §2.4, §2.5, §3.3):

* bilinear-extrapolation refinement ghost: its 2D coefficients recovered by
  unit perturbations equal the printed ones; the printed conservation
  condition (eq. mg-gc-condition) holds for it and for the default scheme
  on random states, and its 3D analogue (the sum of the four ghosts of a
  coarse face, derived the same way) for both 3D schemes; the 3D scheme
  reduces to the printed 2D one on data constant along the second
  tangential axis; the converged solution solves the dense system
  assembled with these ghosts;
* bi/trilinear prolongation: exact for bilinear (trilinear) functions where
  the stencil stays inside the domain (diagonal neighbours copied); at a
  domain corner the extrapolated corner ghost b + c - a (printed) makes it
  equal to the 2-1-1 interpolation there, the property the paper states;
  the converged solution is unchanged (prolongation does not move the fixed
  point).
"""

import json
import os

import numpy as np
import pytest

import dense_ref
from oracle import oracle as O
from paper_1701_04329_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_coefficients.json")))


def cell_pos(dim, N, loc):
    p = 0
    for d in reversed(range(dim)):
        p = p * N + loc[d]
    return p


def find_refinement_side(t, dim):
    for b in range(t.nbox):
        bi = t.box_info(b)
        if bi["leaf"] and bi["level"] >= 2:
            for s in range(2 * dim):
                if bi["nbr"][s] == -2:
                    return b, s
    raise AssertionError("no refinement boundary")


class GhostProbe:
    """the ghost next to a face cell of a refinement side, as a function of
    unit values on the cells its formula may use"""

    def __init__(self, dim, scheme):
        self.dim, self.N = dim, 4
        self.lev, self.idx = W.ball_leaves(dim, 4, 4, (0.3, 0.62, 0.41), 0.0, 0)
        self.t = O.Tree(dim, 4, self.lev, self.idx)
        self.t.set_ghost_scheme(scheme)
        self.leaf_of_box = {b: q for q, b in enumerate(self.t.leaf_boxes())}
        self.b, self.s = find_refinement_side(self.t, dim)
        bi = self.t.box_info(self.b)
        self.l = bi["level"]
        self.d, self.hi = self.s // 2, self.s % 2
        self.q = self.leaf_of_box[self.b]
        self.tang = [e for e in range(dim) if e != self.d]

    def cell(self, depth, flips, tpos=None):
        """local cell of the box: `depth` cells inward from the face, at
        tangential position tpos (default 0), with the listed tangential
        axes flipped to the partner"""
        N = self.N
        c = [0] * self.dim if tpos is None else list(tpos)
        c[self.d] = (N - 1 - depth) if self.hi else depth
        for e in flips:
            c[e] ^= 1
        return c

    def coarse(self, tpos=None):
        N, dim = self.N, self.dim
        org = [(int(self.idx[self.q, e]) - 1) * N for e in range(dim)]
        face = self.cell(0, [], tpos)
        G = [org[e] + face[e] for e in range(dim)]
        G[self.d] += 1 if self.hi else -1
        GH = [g // 2 for g in G]
        key = (self.l - 1,) + tuple(g // N + 1 for g in GH) + ((1,) if dim == 2 else ())
        qH = [q for q, (lv, ix) in enumerate(zip(self.lev, self.idx))
              if (int(lv),) + tuple(int(v) for v in ix[:dim]) + ((1,) if dim == 2 else ()) == key][0]
        return qH, [g % N for g in GH]

    def ghosts(self, u, tpos_list):
        """ghost values next to the face cells at the given tangential positions"""
        self.t.load(np.zeros_like(u), None, u)
        self.t.fill_gc(self.l, "u", homog=True)
        P = self.t.box_padded(self.b)
        out = []
        for tp in tpos_list:
            g = [v + 1 for v in tp]
            g[self.d] = self.N + 1 if self.hi else 0
            out.append(P[tuple(reversed(g))])
        return out

    def unit(self, q, loc):
        u = np.zeros((len(self.lev), self.N ** self.dim))
        u[q, cell_pos(self.dim, self.N, loc)] = 1.0
        return u


def test_bilinear_ghost_matches_printed_coefficients_2d():
    G = GhostProbe(2, "bilinear")
    ref = GOLDEN["ghost_refinement_bilinear_2d"]["coef"]
    t0 = [[0, 0]]

    def gh(q, loc):
        return G.ghosts(G.unit(q, loc), t0)[0]

    e1 = G.tang[0]
    assert gh(*G.coarse()) == ref["u_H"]
    assert gh(G.q, G.cell(0, [])) == ref["u_31"]
    assert gh(G.q, G.cell(0, [e1])) == ref["u_32"]
    assert gh(G.q, G.cell(1, [])) == ref["u_41"]
    assert gh(G.q, G.cell(1, [e1])) == ref["u_42"]


@pytest.mark.parametrize("scheme", ["default", "bilinear"])
@pytest.mark.parametrize("dim", [2, 3])
def test_ghost_schemes_are_conservative(dim, scheme):
    """Sum of the ghosts over one coarse face (2 in 2D, 4 in 3D) equals
    2^(D-2) u_H + 3/4 sum(u_3) - 1/4 sum(u_4) (eq. mg-gc-condition in 2D; in
    3D the same flux balance with four fine fluxes), u_3 / u_4 the face and
    next-inward cells under that coarse face."""
    G = GhostProbe(dim, scheme)
    rng = np.random.default_rng(3 + dim)
    u = rng.standard_normal((len(G.lev), G.N ** dim))
    tps = []
    for flips in ([[]] if dim == 2 else [[], [G.tang[1]]]):
        for f1 in ([], [G.tang[0]]):
            tp = [0] * dim
            for e in f1 + flips:
                tp[e] ^= 1
            tps.append(tp)
    g = G.ghosts(u, tps)
    qH, lH = G.coarse()
    uH = u[qH, cell_pos(dim, G.N, lH)]
    u3 = sum(u[G.q, cell_pos(dim, G.N, G.cell(0, [], tp))] for tp in tps)
    u4 = sum(u[G.q, cell_pos(dim, G.N, G.cell(1, [], tp))] for tp in tps)
    ref = GOLDEN["ghost_conservation_2d"]["coef"]
    want = ref["u_H"] * 2 ** (dim - 2) * uH + ref["u_3"] * u3 + ref["u_4"] * u4
    assert abs(sum(g) - want) <= 1e-13 * max(1.0, abs(want))


def test_trilinear_ghost_reduces_to_printed_2d_scheme():
    """Data constant along the second tangential axis: the 3D bilinear-type
    ghost takes the printed 2D coefficients."""
    G = GhostProbe(3, "bilinear")
    ref = GOLDEN["ghost_refinement_bilinear_2d"]["coef"]
    e1, e2 = G.tang

    def gh_pair(q, loc):
        # the unit value on loc and on its partner along e2 (constant along e2)
        u = G.unit(q, loc)
        p = list(loc)
        p[e2] ^= 1
        u[q, cell_pos(3, G.N, p)] = 1.0
        return G.ghosts(u, [[0, 0, 0]])[0]

    qH, lH = G.coarse()
    # u_H is one coarse cell: constant along e2 already
    assert G.ghosts(G.unit(qH, lH), [[0, 0, 0]])[0] == ref["u_H"]
    assert gh_pair(G.q, G.cell(0, [])) == pytest.approx(ref["u_31"], abs=1e-15)
    assert gh_pair(G.q, G.cell(0, [e1])) == pytest.approx(ref["u_32"], abs=1e-15)
    assert gh_pair(G.q, G.cell(1, [])) == pytest.approx(ref["u_41"], abs=1e-15)
    assert gh_pair(G.q, G.cell(1, [e1])) == pytest.approx(ref["u_42"], abs=1e-15)


TREES = [
    (2, 4, W.ball_leaves(2, 4, 5, (0.3, 0.62), 0.0, 0)),
    (3, 4, W.ball_leaves(3, 4, 4, (0.3, 0.62, 0.41), 0.0, 0)),
    (2, 4, W.domain_leaves(2, 4, [(1, 1), (2, 1)], 4, (1.1, 0.4))),
]


@pytest.mark.parametrize("case", range(len(TREES)))
def test_bilinear_ghost_solution_solves_assembled_system(case):
    dim, N, (lev, idx) = TREES[case]
    rng = np.random.default_rng(40 + case)
    rho = rng.standard_normal((len(lev), N ** dim))
    bc = rng.standard_normal((len(lev), 2 * dim, N ** (dim - 1)))
    bc *= W.domain_side_mask(dim, lev, idx)[:, :, None]
    t = O.Tree(dim, N, lev, idx, bc_type="dirichlet" if case == 2 else None)
    t.set_ghost_scheme("bilinear")
    u, st = t.solve(rho, bc, tol=1e-13, max_cycles=300)
    assert st["status"] == 0
    A, g = dense_ref.assemble(dim, N, lev, idx, bc, ghost="bilinear")
    ud = np.linalg.solve(A, rho.ravel() - g).reshape(u.shape)
    assert np.abs(u - ud).max() <= 1e-9 * np.abs(ud).max()
    # the default ghosts give another discrete solution
    A0, g0 = dense_ref.assemble(dim, N, lev, idx, bc)
    u0 = np.linalg.solve(A0, rho.ravel() - g0).reshape(u.shape)
    assert np.abs(u0 - ud).max() > 1e-6 * np.abs(ud).max()


@pytest.mark.parametrize("case", range(len(TREES)))
def test_linear_prolongation_keeps_the_fixed_point(case):
    dim, N, (lev, idx) = TREES[case]
    rng = np.random.default_rng(50 + case)
    rho = rng.standard_normal((len(lev), N ** dim))
    bc = rng.standard_normal((len(lev), 2 * dim, N ** (dim - 1)))
    bc *= W.domain_side_mask(dim, lev, idx)[:, :, None]
    t = O.Tree(dim, N, lev, idx, bc_type="dirichlet" if case == 2 else None)
    t.set_operator("laplacian", None, "linear")
    u, st = t.solve(rho, bc, tol=1e-13, max_cycles=300)
    assert st["status"] == 0
    A, g = dense_ref.assemble(dim, N, lev, idx, bc)
    ud = np.linalg.solve(A, rho.ravel() - g).reshape(u.shape)
    assert np.abs(u - ud).max() <= 1e-9 * np.abs(ud).max()


def prolong_uniform(dim, f, prolong, N=8):
    """the oracle's prolongation of f's coarse cell values (level 2, uniform,
    Dirichlet values f at the faces) to level 3, v' = 0"""
    lev, idx = W.uniform_leaves(dim, 3)
    t = O.Tree(dim, N, lev, idx)
    t.set_operator("laplacian", None, prolong)
    xc = W.cell_centres(dim, N, lev, idx)
    bc = np.zeros((len(lev), 2 * dim, N ** (dim - 1)))
    for s in range(2 * dim):
        bc[:, s, :] = f(W.face_centres(dim, N, lev, idx, s))
    bc *= W.physical_side_mask(dim, lev, idx)[:, :, None]
    t.load(np.zeros((len(lev), N ** dim)), bc, np.zeros((len(lev), N ** dim)))
    inner = tuple(slice(1, -1) for _ in range(dim))
    for b in range(t.nbox):
        i = t.box_info(b)
        if i["level"] == 2:
            lv = np.array([2])
            ix = np.array([[i["ix"], i["iy"], i["iz"] if dim == 3 else 1]])
            P = t.box_padded(b)
            P[inner] = f(W.cell_centres(dim, N, lv, ix)[0]).reshape((N,) * dim)
            t.set_box_padded(b, P)
            t.set_box_padded(b, np.zeros_like(P), "uold")
    t.fill_gc(2, "u")
    t.prolong_level(3)
    return lev, idx, t.leaf_field("u"), xc


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_prolongation_exact_for_multilinear(dim):
    def f(x):
        v = 0.4 + 0.9 * x[..., 0] - 0.7 * x[..., 1] + 1.3 * x[..., 0] * x[..., 1]
        if dim == 3:
            v = v + 0.5 * x[..., 2] + 0.8 * x[..., 0] * x[..., 1] * x[..., 2]
        return v

    lev, idx, u, xc = prolong_uniform(dim, f, "linear")
    # fine cells whose coarse stencil stays inside the domain: parent coarse
    # cell not on the domain boundary
    hc = 1.0 / 16  # coarse (level 2) cell size with N = 8
    inside = np.all((xc > hc) & (xc < 1 - hc), axis=-1)
    err = np.abs(u - f(xc))[inside]
    assert inside.sum() > 0 and err.max() <= 1e-13
    _, _, u0, _ = prolong_uniform(dim, f, "default")
    assert np.abs(u0 - f(xc))[inside].max() > 1e-5  # 2-1-1 is only linear-exact


def test_corner_extrapolation_reduces_to_211_at_domain_corner():
    """At a domain corner the corner ghost is b + c - a (printed); bilinear
    interpolation with it equals the 2-1-1 value there, for any values."""
    def f(x):
        return np.sin(37.0 * x[..., 0] + 1.1) * np.cos(53.0 * x[..., 1] + 0.3) + x[..., 0] ** 2

    lev, idx, ul, xc = prolong_uniform(2, f, "linear")
    _, _, ud, _ = prolong_uniform(2, f, "default")
    # the fine cell at the lower-left domain corner
    q = [n for n, (l, i) in enumerate(zip(lev, idx)) if i[0] == 1 and i[1] == 1][0]
    assert abs(ul[q, 0] - ud[q, 0]) <= 1e-14 * max(1.0, abs(ud[q, 0]))
    ref = GOLDEN["corner_ghost_extrapolation_2d"]["coef"]
    assert (ref["a"], ref["b"], ref["c"]) == (-1.0, 1.0, 1.0)
