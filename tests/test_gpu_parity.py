"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the
same seeded inputs, element by element on the leaf cells.

Bar (FP64): at equal V-cycle counts the leaf solutions agree to a relative L2
difference of 1e-12 and in every cell to 1e-12 of the largest value; the
residual norms (max and volume-weighted L2) agree after every cycle; solves
to a 1e-10 residual reduction take the same number of cycles (one more or
less only when the last residual ratio lies within 1% of the tolerance)."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W
from parity import REL, assert_leaf_parity, assert_norms_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_solve(w, **kw):
    from paper_1701_04329_amd import afmg as A
    t = A.Tree(w.dim, w.level, w.idx, box_n=w.N)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev)) if t.n_bfaces else None
    u0 = kw.pop("u0", None)
    u = None
    if u0 is not None:
        u = t.leaf_to_boxes(torch.tensor(u0, device=dev))
    u, st = A.solve(t, rho, bc, u, **kw)
    torch.cuda.synchronize()
    return t.boxes_to_leaf(u).cpu().numpy(), st


def oracle_solve(w, **kw):
    t = O.Tree(w.dim, w.N, w.level, w.idx)
    kw = dict(kw)
    u0 = kw.pop("u0", None)
    return t.solve(w.rho, w.bc, u0=u0, **kw)


def check_pair(w, **kw):
    announce(f"{w.name} n_leaves={w.n_leaves} opts={kw}")
    ug, sg = gpu_solve(w, **dict(kw))
    uo, so = oracle_solve(w, **dict(kw))
    assert_leaf_parity(ug, uo, REL, (w.name, kw))
    if kw.get("fixed_cycles", 0) == 0:
        tol = kw.get("tol", 1e-10)
        if sg["cycles"] != so["cycles"]:
            ratio = so["r_max"] / (tol * so["r0_max"])
            assert abs(sg["cycles"] - so["cycles"]) == 1 and 0.99 < ratio < 1.01, (sg, so)
    # residual norms of the initial guess: max |r| and sqrt(sum r^2 h^D)
    np.testing.assert_allclose(sg["r0_max"], so["r0_max"], rtol=1e-12)
    np.testing.assert_allclose(sg["r0_l2"], so["r0_l2"], rtol=1e-12)
    # later residuals approach the rounding floor (about eps * 2D/h^2 * |u|
    # on the finest level), so they are compared to 1e-9 relative plus that
    # floor; a solve to a tolerance also allows 1% of tol * r0, within which
    # the two stop decisions agree.  The L2 norm is at most the max norm on
    # the unit domain, so one absolute allowance serves both.
    tol = kw.get("tol", 1e-10)
    h_min = 1.0 / (w.N * 2.0 ** (w.lmax - 1))
    floor = 16 * np.finfo(float).eps * 2 * w.dim / h_min ** 2 * np.abs(uo).max()
    atol = max(1e-2 * tol * so["r0_max"], floor) if kw.get("fixed_cycles", 0) == 0 else floor
    assert_norms_close([sg["r_max"], sg["r_l2"]], [so["r_max"], so["r_l2"]], atol, what=(w.name, "final norms"))
    n = min(sg["cycles"], so["cycles"])
    assert_norms_close(sg["hist_max"][:n], so["hist_max"][:n], atol, what=(w.name, "history max"))
    assert_norms_close(sg["hist_l2"][:n], so["hist_l2"][:n], atol, what=(w.name, "history L2"))
    return ug, sg, uo, so


def cases():
    out = {}
    out["c1"] = W.config1()
    out["u3_32"] = W.config2(res=32)
    out["u3_64"] = W.config2(res=64)
    out["a2"] = W.adaptive_small(2, 8, 7, 1e-3, 5, n_src=2, sigma_range=(0.03, 0.06))
    out["a3"] = W.adaptive_small(3, 8, 5, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    lev, idx = W.ball_leaves(3, 8, 5, (0.3, 0.62, 0.41), 0.0, 2)
    out["b3_rand"] = W.random_fields(3, 8, lev, idx, 77)
    lev, idx = W.ball_leaves(2, 8, 6, (0.71, 0.33), 0.0, 2)
    out["b2_rand"] = W.random_fields(2, 8, lev, idx, 78)
    for dim in (2, 3):
        for l in (1, 2):
            lev, idx = W.uniform_leaves(dim, l)
            out[f"single_{dim}d_l{l}"] = W.random_fields(dim, 8, lev, idx, 90 + 10 * dim + l)
    # boxes of 16^D cells (paper §2.1, §4.2): 3D trees take the general
    # coarse kernel for levels <= 1 and the box kernels from level 2 on
    out["u3x16_64"] = W.config2(N=16, res=64)
    out["a2x16"] = W.adaptive_small(2, 16, 6, 1e-3, 5, n_src=2, sigma_range=(0.03, 0.06))
    out["a3x16"] = W.adaptive_small(3, 16, 4, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    for dim in (2, 3):
        lev, idx = W.uniform_leaves(dim, 1)
        out[f"single_{dim}d_l1x16"] = W.random_fields(dim, 16, lev, idx, 190 + dim)
    return out


CASES = None


def get(name):
    global CASES
    if CASES is None:
        CASES = cases()
    return CASES[name]


@pytest.mark.parametrize("name", ["c1", "u3_32", "a2", "a3", "b3_rand", "b2_rand",
                                  "single_2d_l1", "single_2d_l2", "single_3d_l1", "single_3d_l2",
                                  "u3x16_64", "a2x16", "a3x16", "single_2d_l1x16", "single_3d_l1x16"])
@pytest.mark.parametrize("fixed", [1, 3])
def test_fixed_cycles_match_oracle(name, fixed):
    check_pair(get(name), fixed_cycles=fixed)


@pytest.mark.parametrize("name", ["c1", "u3_64", "a2", "a3", "b3_rand", "single_3d_l1", "u3x16_64", "a2x16",
                                  "a3x16"])
def test_solve_to_tolerance_matches_oracle(name):
    check_pair(get(name), tol=1e-10)


@pytest.mark.parametrize("name", ["c1", "u3_32", "a2", "a3", "single_2d_l1", "single_3d_l2", "u3x16_64", "a2x16",
                                  "a3x16", "single_3d_l1x16"])
def test_fmg_then_v_matches_oracle(name):
    check_pair(get(name), cycle="FMG", fixed_cycles=2)
    check_pair(get(name), cycle="FMG", tol=1e-10)


def test_box_sizes_give_the_same_uniform_solve():
    """On a uniform grid boxes of 8^3 and of 16^3 cells carry the same grids
    (64^3 down to 2^3), ghosts and red-black order: the two GPU solves agree
    cell by cell to rounding, with the same cycle counts."""
    w8, w16 = get("u3_64"), get("u3x16_64")
    out = []
    for w in (w8, w16):
        announce(f"uniform 64^3 with boxes of {w.N}^3")
        u, st = gpu_solve(w, cycle="FMG", tol=1e-10)
        n = w.N
        g = np.zeros((64, 64, 64))
        ub = u.reshape(-1, n, n, n)
        o = (w.idx[:, :3] - 1) * n
        for q in range(len(w.level)):
            g[o[q, 2]:o[q, 2] + n, o[q, 1]:o[q, 1] + n, o[q, 0]:o[q, 0] + n] = ub[q]
        out.append((g, st))
    (g8, s8), (g16, s16) = out
    assert s8["cycles"] == s16["cycles"]
    assert np.abs(g16 - g8).max() <= 1e-12 * np.abs(g8).max()


def test_stats_report_the_byte_model():
    """stats.bytes_model of an FP64 solve equals afmg_solve_bytes_model with
    the cycles run; mixed-precision solves report 0 (not modelled)."""
    from paper_1701_04329_amd import afmg as A
    w = get("a3")
    t = A.Tree(w.dim, w.level, w.idx)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = t.bc_rows(torch.tensor(w.bc, device=dev))
    for cyc in ("FMG", "V"):
        announce(f"byte model {cyc}")
        _, st = A.solve(t, rho, bc, None, cycle=cyc, tol=1e-10)
        assert st["bytes_model"] == t.bytes_model(st["cycles"], A.make_opts(cycle=cyc)) > 0
    _, st = A.solve(t, rho, bc, None, cycle="FMG", tol=1e-10, precision="mixed")
    assert st["bytes_model"] == 0.0


def test_warm_start_matches_oracle():
    w = get("a3")
    rng = np.random.default_rng(5)
    u0 = w.u_exact + 0.01 * rng.standard_normal(w.u_exact.shape)
    check_pair(w, fixed_cycles=2, u0=u0)


def test_zero_rhs_and_zero_bc_is_exact_immediately():
    w = get("u3_32")
    w0 = W.Workload("zero", 3, 8, w.level, w.idx, np.zeros_like(w.rho), np.zeros_like(w.bc))
    announce("zero problem")
    u, st = gpu_solve(w0, tol=1e-10)
    assert st["cycles"] == 0 and st["r0_max"] == 0.0
    assert np.all(u == 0.0)


def test_full_size_uniform_256():
    """The benchmark workload (uniform 256^3, FMG then V-cycles to 1e-10):
    the whole leaf solution against the oracle's."""
    w = W.config2()
    ug, sg, uo, so = check_pair(w, cycle="FMG", tol=1e-10)
    assert sg["status"] == 0 and sg["cycles"] <= 15


@pytest.mark.parametrize("dim,lmax", [(2, 14), (3, 10)])
def test_deep_point_refinement_matches_oracle(dim, lmax):
    """A grid refined around one point down to a deep level (cells of
    1/65536 in 2D, 1/4096 in 3D), refinement boundaries at every level:
    the solution at a fixed cycle count against the oracle."""
    c = (0.3, 0.62, 0.41)
    w = W.random_fields(dim, 8, *W.ball_leaves(dim, 8, lmax, c, 0.0, 1), 61 + dim)
    assert w.lmax == lmax
    check_pair(w, cycle="FMG", fixed_cycles=3)
    check_pair(w, cycle="V", tol=1e-10)


@pytest.mark.parametrize("n", [8, 16])
def test_maximum_size_uniform_512_residual(n):
    """The largest uniform grid the benchmark runs (512^3 = 134,217,728
    unknowns, lap(phi) = 1, phi = 0 on the boundary), solved to a 1e-8
    residual reduction (the FP64 rounding floor of this residual is about
    5e-11: |sum of neighbours - 6 u| ~ 0.3 carries ~1e-16 of rounding and is
    divided by h^2 = 3.8e-6).  The oracle does not run at this size, so the
    check is a property that holds at any size: the residual of the returned
    solution, recomputed here from the 7-point stencil with the Dirichlet
    ghost -u1 (plain numpy on the whole grid), is below 1e-8 of the initial
    one (max |rho| = 1), up to the rounding floor.  Boxes of 8^3 and of
    16^3 cells."""
    from paper_1701_04329_amd import afmg as A
    w = W.uniform_const_rhs(3, n, 512)
    announce(f"maximum size {w.name} box {n}^3 unknowns={w.n_unknowns}")
    t = A.Tree(3, w.level, w.idx, box_n=n)
    dev = torch.device("cuda", 0)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    u, st = A.solve(t, rho, None, cycle="FMG", tol=1e-8)
    assert st["status"] == 0 and st["r_max"] <= 1e-8 * st["r0_max"]
    assert st["r0_max"] == 1.0
    ul = t.boxes_to_leaf(u)
    del u, rho
    # leaves in box order -> one 512^3 array (z, y, x)
    lev, idx = w.level, w.idx
    g = np.zeros((512, 512, 512))
    ulh = ul.cpu().numpy().reshape(-1, n, n, n)
    del ul
    i0, j0, k0 = (idx[:, 0] - 1) * n, (idx[:, 1] - 1) * n, (idx[:, 2] - 1) * n
    for q in range(len(lev)):
        g[k0[q]:k0[q] + n, j0[q]:j0[q] + n, i0[q]:i0[q] + n] = ulh[q]
    del ulh
    p = np.pad(g, 1)
    for ax in range(3):  # Dirichlet ghosts 2b - u1 with b = 0
        sl_lo = [slice(None)] * 3
        sl_in = [slice(None)] * 3
        sl_lo[ax], sl_in[ax] = 0, 1
        p[tuple(sl_lo)] = -p[tuple(sl_in)]
        sl_lo[ax], sl_in[ax] = -1, -2
        p[tuple(sl_lo)] = -p[tuple(sl_in)]
    h = 1.0 / 512
    lap = (p[:-2, 1:-1, 1:-1] + p[2:, 1:-1, 1:-1] + p[1:-1, :-2, 1:-1] + p[1:-1, 2:, 1:-1]
           + p[1:-1, 1:-1, :-2] + p[1:-1, 1:-1, 2:] - 6.0 * g) / (h * h)
    r = np.abs(1.0 - lap).max()
    print(f"512^3: cycles={st['cycles']} library r_max={st['r_max']:.3e} numpy r_max={r:.3e}", flush=True)
    assert r <= 1e-8 + 2e-10
    assert abs(r - st["r_max"]) <= 2e-10
