"""Adjoint on the GPU: the operator and its transpose against the oracle's
sparse matrix, lambda = L^-T u_bar against the oracle's sparse direct solve,
the gradients against central finite differences of GPU solves (exact for a
quadratic loss up to the solver tolerance), and the torch.autograd path."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_04329_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = None


def dev():
    global DEV
    if DEV is None:
        DEV = torch.device("cuda", 0)
    return DEV


def grids(name):
    """name -> (dim, box size, (level, idx))"""
    return {
        "a2": lambda: (2, 8, W.ball_leaves(2, 8, 6, (0.71, 0.33), 0.0, 2)),
        "a3": lambda: (3, 8, W.ball_leaves(3, 8, 4, (0.3, 0.62, 0.41), 0.0, 1)),
        "u3": lambda: (3, 8, W.uniform_leaves(3, 3)),
        "u2": lambda: (2, 8, W.uniform_leaves(2, 4)),
        "b3": lambda: (3, 8, W.ball_leaves(3, 8, 5, (0.3, 0.62, 0.41), 0.0, 2)),
        # boxes of 16^D cells
        "a2x16": lambda: (2, 16, W.ball_leaves(2, 16, 5, (0.71, 0.33), 0.0, 2)),
        "a3x16": lambda: (3, 16, W.ball_leaves(3, 16, 3, (0.3, 0.62, 0.41), 0.0, 1)),
    }[name]()


def setup(name, seed):
    from paper_1701_04329_amd import afmg as A
    dim, n, (lev, idx) = grids(name)
    t = A.Tree(dim, lev, idx, box_n=n)
    o = O.Tree(dim, n, lev, idx)
    rng = np.random.default_rng(seed)
    return dim, lev, idx, t, o, rng


@pytest.mark.parametrize("name", ["a2", "a3", "u3", "b3", "a2x16", "a3x16"])
def test_apply_L_and_LT_match_oracle_matrix(name):
    dim, lev, idx, t, o, rng = setup(name, 11)
    print(f"[case] apply {name} leaves={len(lev)}", flush=True)
    A = O.assemble_L(o)
    from paper_1701_04329_amd import afmg as AF
    x = rng.standard_normal((len(lev), t.box_n ** dim))
    xd = t.leaf_to_boxes(torch.tensor(x, device=dev()))
    for op, M in (("L", A), ("LT", A.T.tocsr())):
        y = t.boxes_to_leaf(AF.apply(t, xd, op)).cpu().numpy().ravel()
        ref = M @ x.ravel()
        np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_transpose_dot_product_on_a_larger_grid():
    from paper_1701_04329_amd import afmg as AF
    w = W.adaptive_small(3, 8, 5, 1e-3, 6, n_src=2, sigma_range=(0.04, 0.08))
    t = AF.Tree(3, w.level, w.idx)
    rng = np.random.default_rng(3)
    x = t.leaf_to_boxes(torch.tensor(rng.standard_normal((w.n_leaves, 512)), device=dev()))
    y = t.leaf_to_boxes(torch.tensor(rng.standard_normal((w.n_leaves, 512)), device=dev()))
    lx = AF.apply(t, x, "L")
    lty = AF.apply(t, y, "LT")
    a = float((lx * y).sum())
    b = float((x * lty).sum())
    assert a == pytest.approx(b, rel=1e-12)


@pytest.mark.parametrize("name", ["a2", "a3", "u3", "u2", "a2x16", "a3x16"])
def test_adjoint_matches_oracle(name):
    from paper_1701_04329_amd import afmg as AF
    dim, lev, idx, t, o, rng = setup(name, 21)
    print(f"[case] adjoint {name} leaves={len(lev)}", flush=True)
    ubar = rng.standard_normal((len(lev), t.box_n ** dim))
    lam_o, gbc_o = O.adjoint(o, ubar)
    rb, bb, st = AF.adjoint(t, t.leaf_to_boxes(torch.tensor(ubar, device=dev())), tol=1e-12)
    lam = t.boxes_to_leaf(rb).cpu().numpy()
    err = np.linalg.norm(lam - lam_o) / np.linalg.norm(lam_o)
    print(f"adjoint {name}: iterations={st['cycles']} residual={st['r_max'] / st['r0_max']:.1e} "
          f"rel-L2 vs oracle {err:.2e}", flush=True)
    assert st["status"] == 0, st
    assert err <= 1e-9
    # Dirichlet gradient rows
    gref = t.bc_rows(gbc_o)
    np.testing.assert_allclose(bb.cpu().numpy(), gref, rtol=1e-8, atol=1e-9 * np.abs(gref).max())
    parents = np.ones(t.n_boxes, bool)
    parents[t.leaf_boxes] = False
    if parents.any():
        assert float(rb[torch.tensor(parents, device=rb.device)].abs().max()) == 0.0


@pytest.mark.parametrize("name", ["b3", "a2"])
def test_gradient_matches_central_differences_of_gpu_solves(name):
    """loss = sum over leaf cells (u - ut)^2; central differences are exact
    for a quadratic loss, up to the solves' tolerance."""
    from paper_1701_04329_amd import afmg as AF
    dim, lev, idx, t, o, rng = setup(name, 31)
    n = len(lev)
    print(f"[case] fd {name} leaves={n}", flush=True)
    rho = rng.standard_normal((n, 8 ** dim))
    phys = W.physical_side_mask(dim, lev, idx)[:, :, None]
    bcl = rng.standard_normal((n, 2 * dim, 8 ** (dim - 1))) * phys
    ut = rng.standard_normal((n, 8 ** dim))
    D = dev()
    utd = torch.tensor(ut, device=D)

    def loss(r, b):
        u, st = AF.solve(t, t.leaf_to_boxes(torch.tensor(r, device=D)), t.bc_rows(torch.tensor(b, device=D)),
                         tol=1e-13, max_cycles=200)
        return float(((t.boxes_to_leaf(u) - utd) ** 2).sum()), u

    l0, u = loss(rho, bcl)
    ubar = 2.0 * (t.boxes_to_leaf(u) - utd)
    rb, bb, st = AF.adjoint(t, t.leaf_to_boxes(ubar), tol=1e-13, max_cycles=400)
    g_rho = t.boxes_to_leaf(rb).cpu().numpy()
    g_bc = bb.cpu().numpy()
    for trial in range(2):
        dr = rng.standard_normal(rho.shape)
        db = rng.standard_normal(bcl.shape) * phys
        eps = 1.0  # the loss is quadratic: any step gives the exact derivative
        fd_r = (loss(rho + eps * dr, bcl)[0] - loss(rho - eps * dr, bcl)[0]) / (2 * eps)
        fd_b = (loss(rho, bcl + eps * db)[0] - loss(rho, bcl - eps * db)[0]) / (2 * eps)
        ad_r = float(np.sum(g_rho * dr))
        ad_b = float(np.sum(g_bc * t.bc_rows(db)))
        print(f"fd {name}: rho {ad_r:.10e} vs {fd_r:.10e}; bc {ad_b:.10e} vs {fd_b:.10e}", flush=True)
        assert ad_r == pytest.approx(fd_r, rel=1e-7)
        assert ad_b == pytest.approx(fd_b, rel=1e-7)


def test_autograd_through_poisson_solve():
    from paper_1701_04329_amd import afmg as AF
    dim, lev, idx, t, o, rng = setup("a3", 41)
    n = len(lev)
    D = dev()
    rho_l = rng.standard_normal((n, 512))
    phys = W.physical_side_mask(dim, lev, idx)[:, :, None]
    bc_l = rng.standard_normal((n, 6, 64)) * phys
    ut = torch.tensor(rng.standard_normal((n, 512)), device=D)
    rho = t.leaf_to_boxes(torch.tensor(rho_l, device=D)).requires_grad_(True)
    bc = t.bc_rows(torch.tensor(bc_l, device=D)).requires_grad_(True)
    u = AF.poisson_solve(t, rho, bc, tol=1e-12, max_cycles=200)
    loss = ((t.boxes_to_leaf(u) - ut) ** 2).sum()
    loss.backward()
    # oracle: the same gradients from the sparse direct solves
    A = O.assemble_L(o)
    import scipy.sparse.linalg as spla
    lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A")
    # boundary part of the rhs (L u = rho - B b): B b = apply_L(0) with the values b
    gb = o.apply_L(np.zeros((n, 512)), bc=bc_l, homog=False).ravel()
    us = lu.solve(rho_l.ravel() - gb)
    lam, gbc = O.adjoint(o, 2.0 * (us - ut.cpu().numpy().ravel()))
    g_rho = t.boxes_to_leaf(rho.grad).cpu().numpy()
    np.testing.assert_allclose(g_rho, lam, rtol=1e-8, atol=1e-9 * np.abs(lam).max())
    np.testing.assert_allclose(bc.grad.cpu().numpy(), t.bc_rows(gbc), rtol=1e-8,
                               atol=1e-9 * np.abs(gbc).max())


def test_full_size_adjoint_workload():
    """The adjoint benchmark octree at full size (about 4e6 unknowns): the
    transpose dot-product identity, and the gradients with respect to rho and
    the Dirichlet values against central differences of GPU solves (exact for
    the quadratic loss up to the solve tolerance)."""
    from paper_1701_04329_amd import afmg as AF
    w, u_t = W.config5()
    print(f"[case] full-size adjoint {w.name} unknowns={w.n_unknowns}", flush=True)
    t = AF.Tree(3, w.level, w.idx)
    D = dev()
    rng = np.random.default_rng(51)
    x = t.leaf_to_boxes(torch.tensor(rng.standard_normal((w.n_leaves, 512)), device=D))
    y = t.leaf_to_boxes(torch.tensor(rng.standard_normal((w.n_leaves, 512)), device=D))
    a = float((AF.apply(t, x, "L") * y).sum())
    b = float((x * AF.apply(t, y, "LT")).sum())
    assert a == pytest.approx(b, rel=1e-11)
    rho = t.leaf_to_boxes(torch.tensor(w.rho, device=D))
    bc = t.bc_rows(torch.tensor(w.bc, device=D))
    utd = t.leaf_to_boxes(torch.tensor(u_t, device=D))
    leaf = torch.zeros(t.n_boxes, dtype=torch.bool, device=D)
    leaf[torch.as_tensor(t.leaf_boxes, device=D).long()] = True

    def loss(r, bb):
        u, st = AF.solve(t, r, bb, cycle="FMG", tol=1e-12, max_cycles=200)
        assert st["status"] == 0
        return float(((u - utd)[leaf] ** 2).sum()), u

    _, u = loss(rho, bc)
    ubar = torch.where(leaf[:, None], 2.0 * (u - utd), torch.zeros_like(u))
    rb, bb, st = AF.adjoint(t, ubar, tol=1e-12, max_cycles=400)
    print(f"adjoint iterations {st['cycles']} residual ratio {st['r_max'] / st['r0_max']:.1e}", flush=True)
    assert st["status"] == 0
    dr = t.leaf_to_boxes(torch.tensor(rng.standard_normal((w.n_leaves, 512)), device=D))
    db = torch.tensor(rng.standard_normal(tuple(bc.shape)), device=D)
    fd_r = (loss(rho + dr, bc)[0] - loss(rho - dr, bc)[0]) / 2.0
    fd_b = (loss(rho, bc + db)[0] - loss(rho, bc - db)[0]) / 2.0
    ad_r = float((rb * dr).sum())
    ad_b = float((bb * db).sum())
    print(f"rho: adjoint {ad_r:.12e} fd {fd_r:.12e}; bc: adjoint {ad_b:.12e} fd {fd_b:.12e}", flush=True)
    assert ad_r == pytest.approx(fd_r, rel=1e-7)
    assert ad_b == pytest.approx(fd_b, rel=1e-7)
