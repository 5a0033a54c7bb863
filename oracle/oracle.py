"""ctypes wrapper of the FP64 CPU oracle (afmg_oracle.c).

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the CPU-baseline
leg of the benchmark use this module.  It imports nothing from the GPU
library; inputs come from the shared seeded generators.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "afmg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", "-Wall"]


def build(force=True):
    """Compile the oracle with gcc (plain C, OpenMP over boxes)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


class Opts(C.Structure):
    _fields_ = [
        ("cycle", C.c_int),
        ("n_down", C.c_int),
        ("n_up", C.c_int),
        ("n_base", C.c_int),
        ("tol", C.c_double),
        ("max_cycles", C.c_int),
        ("fixed_cycles", C.c_int),
        ("use_guess", C.c_int),
        ("homog", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("cycles", C.c_int),
        ("r0_max", C.c_double),
        ("r0_l2", C.c_double),
        ("r_max", C.c_double),
        ("r_l2", C.c_double),
        ("hist_max", C.c_double * 128),
        ("hist_l2", C.c_double * 128),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        vp, i32p, dp = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)
        L.or_tree_new.restype = vp
        L.or_tree_new.argtypes = [C.c_int, C.c_int, C.c_int64, i32p, i32p, C.c_char_p, C.c_int]
        L.or_tree_new_bc.restype = vp
        L.or_tree_new_bc.argtypes = [C.c_int, C.c_int, i32p, C.c_int64, i32p, i32p, C.c_char_p, C.c_int]
        L.or_tree_free.argtypes = [vp]
        L.or_last_error.restype = C.c_char_p
        L.or_tree_info.argtypes = [vp, C.POINTER(C.c_int64)]
        L.or_box_info.argtypes = [vp, C.c_int, i32p]
        L.or_leaf_boxes.argtypes = [vp, i32p]
        L.or_solve.argtypes = [vp, dp, dp, dp, C.POINTER(Opts), C.POINTER(Stats)]
        L.or_solve.restype = C.c_int
        L.or_apply_L.argtypes = [vp, dp, dp, dp, C.c_int]
        L.or_load.argtypes = [vp, dp, dp, dp]
        L.or_fill_gc.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.or_half_sweep.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.or_vcycle.argtypes = [vp, C.POINTER(Opts)]
        L.or_fmg.argtypes = [vp, C.POINTER(Opts)]
        L.or_finalize.argtypes = [vp, C.c_int, dp]
        L.or_restrict_level.argtypes = [vp, C.c_int, C.c_int]
        L.or_copy_uold.argtypes = [vp, C.c_int]
        L.or_prolong_level.argtypes = [vp, C.c_int]
        L.or_resid_restrict_level.argtypes = [vp, C.c_int, C.c_int]
        L.or_coarse_rhs_level.argtypes = [vp, C.c_int, C.c_int]
        L.or_vcycle_from.argtypes = [vp, C.c_int, C.POINTER(Opts)]
        L.or_get_box.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_set_box.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_get_leaf_field.argtypes = [vp, C.c_int, dp]
        L.or_get_bc.argtypes = [vp, C.c_int, C.c_int, dp]
        L.or_get_bc.restype = C.c_int
        L.or_num_threads.restype = C.c_int
        L.or_assemble_L.argtypes = [vp, i32p, i32p, dp]
        L.or_assemble_L.restype = C.c_int64
        L.or_set_operator.argtypes = [vp, C.c_int, dp, C.c_int]
        L.or_set_operator.restype = C.c_int
        L.or_set_ghost_scheme.argtypes = [vp, C.c_int]
        L.or_set_ghost_scheme.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


FIELD = {"u": 0, "rho": 1, "uold": 2, "res": 3, "eps": 4}

# operators (paper §3.4, §3.5): bit 1 a coefficient eps per cell with the
# harmonic mean on faces, bit 2 the cylindrical (r, z) form (2D, x = r)
OPERATORS = {"laplacian": 0, "eps": 1, "cyl": 2, "cyl_eps": 3}
# prolongations (paper §2.5 and §3.5) and refinement-boundary ghosts (§3.3)
PROLONGS = {"default": 0, "eps": 1, "linear": 2}
GHOSTS = {"default": 0, "bilinear": 1}


class OracleError(RuntimeError):
    pass


BC_TYPES = {"dirichlet": 0, "neumann": 1, "periodic": 2}


def bc_type_codes(bc_type, dim):
    """Side types per orientation (-x, +x, -y, +y, -z, +z): None (all
    Dirichlet), one name for all sides, or a sequence of 2D names / codes."""
    if bc_type is None:
        return np.zeros(6, np.int32)
    if isinstance(bc_type, str):
        bc_type = [bc_type] * (2 * dim)
    out = np.zeros(6, np.int32)
    for s, v in enumerate(bc_type):
        out[s] = BC_TYPES[v] if isinstance(v, str) else int(v)
    return out


class Tree:
    """Oracle tree built from a leaf list (level int32 [n], idx int32 [n,3]).
    The coarse grid is the set of level-1 boxes holding the leaves (one unit
    box at each 1-based lattice position); bc_type gives the side type of
    each orientation (see bc_type_codes)."""

    def __init__(self, dim, N, level, idx, bc_type=None):
        L = lib()
        self.dim, self.N = dim, N
        level = np.ascontiguousarray(level, dtype=np.int32)
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
        err = C.create_string_buffer(512)
        i32p = C.POINTER(C.c_int32)
        if bc_type is None:
            h = L.or_tree_new(dim, N, len(level), level.ctypes.data_as(i32p), idx.ctypes.data_as(i32p), err, 512)
        else:
            codes = bc_type_codes(bc_type, dim)
            h = L.or_tree_new_bc(dim, N, codes.ctypes.data_as(i32p), len(level), level.ctypes.data_as(i32p),
                                 idx.ctypes.data_as(i32p), err, 512)
        if not h:
            raise OracleError(err.value.decode())
        self.h = h
        info = (C.c_int64 * 10)()
        L.or_tree_info(h, info)
        self.nbox, self.lmin, self.lmax, self.n_leaves = info[0], info[1], info[2], info[3]
        self.nroot = info[6]
        self.ext = (info[7], info[8], info[9])
        self.bc_type = bc_type_codes(bc_type, dim)
        self.level = level
        self.idx = idx

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_tree_free(self.h)
            self.h = None

    @property
    def cells_per_box(self):
        return self.N ** self.dim

    def box_info(self, b):
        out = (C.c_int32 * 13)()
        lib().or_box_info(self.h, b, out)
        o = list(out)
        return dict(level=o[0], ix=o[1], iy=o[2], iz=o[3], n=o[4], parent=o[5], leaf=o[6],
                    nbr=o[7:13])

    def leaf_boxes(self):
        out = np.zeros(self.n_leaves, np.int32)
        lib().or_leaf_boxes(self.h, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def _leaf_arr(self, a, name):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.size != self.n_leaves * self.cells_per_box:
            raise ValueError(f"{name}: expected {self.n_leaves}x{self.cells_per_box} values")
        return a

    def _bc_arr(self, bc):
        if bc is None:
            return None
        bc = np.ascontiguousarray(bc, dtype=np.float64)
        if bc.size != self.n_leaves * 2 * self.dim * self.N ** (self.dim - 1):
            raise ValueError("bc has the wrong size")
        return bc

    def solve(self, rho, bc=None, u0=None, cycle="V", tol=1e-10, max_cycles=100,
              fixed_cycles=0, n_down=2, n_up=2, n_base=4, homog=False):
        rho = self._leaf_arr(rho, "rho")
        bc = self._bc_arr(bc)
        u = np.zeros(self.n_leaves * self.cells_per_box) if u0 is None else \
            self._leaf_arr(u0, "u0").copy()
        o = Opts(1 if cycle == "FMG" else 0, n_down, n_up, n_base, tol, max_cycles,
                 fixed_cycles, 0 if u0 is None else 1, 1 if homog else 0)
        st = Stats()
        rc = lib().or_solve(self.h, _dp(rho), _dp(bc), _dp(u), C.byref(o), C.byref(st))
        hist = np.array(st.hist_max[:min(st.cycles, 128)])
        return u.reshape(self.n_leaves, -1), dict(
            status=rc, cycles=st.cycles, r0_max=st.r0_max, r0_l2=st.r0_l2, r_max=st.r_max,
            r_l2=st.r_l2, hist_max=hist, hist_l2=np.array(st.hist_l2[:min(st.cycles, 128)]))

    def set_operator(self, kind="laplacian", eps=None, prolong="default"):
        """Operator of later solves and steps: "laplacian", "eps" (div(eps
        grad u)), "cyl" (cylindrical (r, z)) or "cyl_eps"; eps [n_leaves,
        N^D] > 0 per leaf cell; prolong "default" (2-1-1), "eps"
        (eps-weighted) or "linear" (bi/trilinear with edge and corner
        ghosts)."""
        code = OPERATORS[kind] if isinstance(kind, str) else int(kind)
        e = None if eps is None else self._leaf_arr(eps, "eps")
        rc = lib().or_set_operator(self.h, code, _dp(e), PROLONGS[prolong])
        if rc != 0:
            raise OracleError(lib().or_last_error().decode())
        self.operator = (code, prolong)

    def set_ghost_scheme(self, scheme="default"):
        """Refinement-boundary ghosts: "default" or "bilinear"."""
        if lib().or_set_ghost_scheme(self.h, GHOSTS[scheme]) != 0:
            raise OracleError(lib().or_last_error().decode())
        self.ghost_scheme = scheme

    def apply_L(self, u, bc=None, homog=True):
        u = self._leaf_arr(u, "u")
        bc = self._bc_arr(bc)
        out = np.zeros_like(u)
        lib().or_apply_L(self.h, _dp(u), _dp(bc), _dp(out), 1 if homog else 0)
        return out.reshape(self.n_leaves, -1)

    # ---- step-level access used by the pins -------------------------------
    def load(self, rho, bc=None, u=None):
        rho = self._leaf_arr(rho, "rho")
        bc = self._bc_arr(bc)
        u = None if u is None else self._leaf_arr(u, "u")
        lib().or_load(self.h, _dp(rho), _dp(bc), _dp(u))

    def fill_gc(self, level, field="u", homog=False):
        lib().or_fill_gc(self.h, level, FIELD[field], 1 if homog else 0)

    def half_sweep(self, level, colour, homog=False):
        lib().or_half_sweep(self.h, level, colour, 1 if homog else 0)

    def vcycle(self, n_down=2, n_up=2, n_base=4, homog=False):
        o = Opts(0, n_down, n_up, n_base, 0.0, 1, 1, 1, 1 if homog else 0)
        lib().or_vcycle(self.h, C.byref(o))

    def fmg(self, n_down=2, n_up=2, n_base=4, homog=False):
        o = Opts(1, n_down, n_up, n_base, 0.0, 1, 1, 0, 1 if homog else 0)
        lib().or_fmg(self.h, C.byref(o))

    def finalize(self, homog=False):
        out = np.zeros(2)
        lib().or_finalize(self.h, 1 if homog else 0, _dp(out))
        return out[0], out[1]

    def restrict_level(self, level, field="u"):
        lib().or_restrict_level(self.h, level, FIELD[field])

    def copy_uold(self, level):
        lib().or_copy_uold(self.h, level)

    def prolong_level(self, level):
        lib().or_prolong_level(self.h, level)

    def resid_restrict_level(self, level, homog=False):
        lib().or_resid_restrict_level(self.h, level, 1 if homog else 0)

    def coarse_rhs_level(self, level, homog=False):
        lib().or_coarse_rhs_level(self.h, level, 1 if homog else 0)

    def vcycle_from(self, top, n_down=2, n_up=2, n_base=4, homog=False):
        o = Opts(0, n_down, n_up, n_base, 0.0, 1, 1, 1, 1 if homog else 0)
        lib().or_vcycle_from(self.h, top, C.byref(o))

    def box_padded(self, b, field="u"):
        n = self.box_info(b)["n"]
        out = np.zeros((n + 2) ** self.dim)
        lib().or_get_box(self.h, b, FIELD[field], _dp(out))
        return out.reshape(((n + 2),) * self.dim)  # axes (z,) y, x

    def set_box_padded(self, b, arr, field="u"):
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        lib().or_set_box(self.h, b, FIELD[field], _dp(a))

    def leaf_field(self, field="u"):
        out = np.zeros(self.n_leaves * self.cells_per_box)
        lib().or_get_leaf_field(self.h, FIELD[field], _dp(out))
        return out.reshape(self.n_leaves, -1)

    def box_bc(self, b, side):
        n = self.box_info(b)["n"]
        out = np.zeros(n ** (self.dim - 1))
        ok = lib().or_get_bc(self.h, b, side, _dp(out))
        return out if ok else None


def _assemble(tree):
    L = lib()
    nnz = L.or_assemble_L(tree.h, None, None, None)
    r = np.zeros(nnz, np.int32)
    c = np.zeros(nnz, np.int32)
    v = np.zeros(nnz)
    L.or_assemble_L(tree.h, r.ctypes.data_as(C.POINTER(C.c_int32)), c.ctypes.data_as(C.POINTER(C.c_int32)),
                    _dp(v))
    return r, c, v


def assemble_L(tree):
    """Sparse matrix (scipy CSR) of the homogeneous composite operator on the
    leaf unknowns, numbered q * N^D + cell in the caller's leaf order."""
    import scipy.sparse as sp
    if getattr(tree, "operator", (0,))[0] or getattr(tree, "ghost_scheme", "default") != "default":
        raise OracleError("the sparse assembly covers the Laplacian with the default ghosts only")
    r, c, v = _assemble(tree)
    n = tree.n_leaves * tree.cells_per_box
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def adjoint(tree, ubar):
    """lambda = L^-T ubar on the leaf unknowns (sparse direct solve), and the
    gradient with respect to the boundary values, as [n_leaves, 2D, N^(D-1)]
    (zero on non-physical sides): -2 lambda / h^2 on the leaf cells next to a
    Dirichlet side, -lambda / h next to a Neumann side.  The derivation:
    u = L^-1 (rho - B b) with (B b)_c = sum over the physical sides of c of
    2 b / h^2 (Dirichlet ghost 2 b - u_c) or b / h (Neumann ghost u_c + h b)."""
    import scipy.sparse.linalg as spla
    A = assemble_L(tree)
    # minimum-degree ordering on A + A^T keeps the fill of 3D grids small
    lu = spla.splu(A.T.tocsc(), permc_spec="MMD_AT_PLUS_A")
    lam = lu.solve(np.ascontiguousarray(ubar, dtype=np.float64).ravel())
    return lam.reshape(tree.n_leaves, -1), boundary_gradient(tree, lam)


def boundary_gradient(tree, lam):
    dim, N = tree.dim, tree.N
    lam = np.asarray(lam).reshape((tree.n_leaves,) + (N,) * dim)
    h = 1.0 / (N * 2.0 ** (tree.level.astype(np.float64) - 1))
    out = np.zeros((tree.n_leaves, 2 * dim, N ** (dim - 1)))
    boxes = tree.leaf_boxes()
    for s in range(2 * dim):
        phys = np.array([tree.box_info(int(b))["nbr"][s] == -1 for b in boxes])
        ax = dim - 1 - s // 2
        sl = [slice(None)] * (dim + 1)
        sl[1 + ax] = N - 1 if s % 2 else 0
        face = lam[tuple(sl)].reshape(tree.n_leaves, -1)
        if tree.bc_type[s] == BC_TYPES["neumann"]:
            g = -face / h[:, None]
        else:
            g = -2.0 * face / (h[:, None] ** 2)
        out[:, s, :] = np.where(phys[:, None], g, 0.0)
    return out


def num_threads():
    return lib().or_num_threads()
