"""Python binding of the afmg C-ABI (include/afmg.h).

Argument marshalling only: every step of the solve runs in the HIP library
(libafmg.so next to this file).  Device memory and streams come from PyTorch.
There is no fallback: if the library is missing the import of this module's
entry points raises.
"""

from __future__ import annotations

import ctypes as C
import os
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafmg.so")

AFMG_OK = 0
AFMG_NOT_CONVERGED = 1
AFMG_ERR_ARG = -1
AFMG_ERR_TREE = -2
AFMG_ERR_HIP = -3
AFMG_ERR_OOM = -4
AFMG_ERR_NONFINITE = -5
AFMG_ERR_DIVERGED = -6
AFMG_HIST = 128

CYCLES = {"V": 0, "FMG": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}


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
        ("precision", C.c_int),
        ("profile", C.c_int),
        ("graph", C.c_int),
        ("check_every", C.c_int),
        ("prof_level", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("cycles", C.c_int),
        ("r0_max", C.c_double),
        ("r0_l2", C.c_double),
        ("r_max", C.c_double),
        ("r_l2", C.c_double),
        ("hist_max", C.c_double * AFMG_HIST),
        ("hist_l2", C.c_double * AFMG_HIST),
        ("t_ms", C.c_double),
        ("prof_ms", C.c_double * 4),
        ("prof_n", C.c_int * 4),
        ("bytes_model", C.c_double),
    ]

    def to_dict(self):
        n = min(self.cycles, AFMG_HIST)
        return dict(status=self.status, cycles=self.cycles, r0_max=self.r0_max, r0_l2=self.r0_l2,
                    r_max=self.r_max, r_l2=self.r_l2, hist_max=np.array(self.hist_max[:n]),
                    hist_l2=np.array(self.hist_l2[:n]), t_ms=self.t_ms,
                    prof_ms=list(self.prof_ms), prof_n=list(self.prof_n), bytes_model=self.bytes_model)


class TreeDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("box_n", C.c_int),
        ("n_boxes", C.c_int64),
        ("n_leaves", C.c_int64),
        ("n_bfaces", C.c_int64),
        ("lmin", C.c_int),
        ("lmax", C.c_int),
        ("cells_per_box", C.c_int64),
        ("n_unknowns", C.c_int64),
        ("n_roots", C.c_int),
        ("ext", C.c_int * 3),
        ("bc_type", C.c_int * 6),
        ("singular", C.c_int),
        ("op", C.c_int),
        ("prolong", C.c_int),
        ("ghost", C.c_int),
    ]


BC_TYPES = {"dirichlet": 0, "neumann": 1, "periodic": 2}


def bc_type_codes(bc_type, dim):
    """Side types per orientation (-x, +x, -y, +y, -z, +z): None (all
    Dirichlet), one name for all sides, or 2D names / codes."""
    out = np.zeros(6, np.int32)
    if bc_type is None:
        return out
    if isinstance(bc_type, str):
        bc_type = [bc_type] * (2 * dim)
    for s, v in enumerate(bc_type):
        out[s] = BC_TYPES[v] if isinstance(v, str) else int(v)
    return out


class BatchDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("box_n", C.c_int),
        ("n_trees", C.c_int),
        ("lmax", C.c_int),
        ("n_boxes", C.c_int64),
        ("n_bfaces", C.c_int64),
        ("n_unknowns", C.c_int64),
    ]


class BoxDesc(C.Structure):
    _fields_ = [
        ("level", C.c_int),
        ("idx", C.c_int * 3),
        ("parent", C.c_int),
        ("leaf", C.c_int),
        ("nbr", C.c_int * 6),
        ("children", C.c_int * 8),
        ("x_lo", C.c_double * 3),
        ("h", C.c_double),
    ]


EXPORTS = [
    "afmg_default_opts", "afmg_tree_create", "afmg_tree_destroy", "afmg_tree_info",
    "afmg_tree_leaf_boxes", "afmg_tree_bfaces", "afmg_tree_box", "afmg_workspace_bytes",
    "afmg_solve", "afmg_last_error", "afmg_adjoint_workspace_bytes", "afmg_apply", "afmg_adjoint",
    "afmg_batch_create", "afmg_batch_destroy", "afmg_batch_info", "afmg_batch_workspace_bytes",
    "afmg_batch_solve", "afmg_autotune_workspace_bytes", "afmg_tree_autotune", "afmg_tree_shape",
    "afmg_tree_set_shape", "afmg_batch_autotune_workspace_bytes", "afmg_batch_autotune", "afmg_batch_shape",
    "afmg_batch_set_shape", "afmg_tree_refine", "afmg_tree_finalize", "afmg_tree_level_list", "afmg_step",
    "afmg_solve_noalloc", "afmg_tree_create_domain", "afmg_tree_set_operator", "afmg_tree_adapt",
    "afmg_transfer_workspace_bytes", "afmg_tree_transfer", "afmg_tree_set_ghost_scheme",
    "afmg_solve_bytes_model",
]
# operators (paper §3.4, §3.5) and prolongations of afmg_tree_set_operator
OPERATORS = {"laplacian": 0, "eps": 1, "cyl": 2, "cyl_eps": 3}
PROLONGS = {"default": 0, "eps": 1, "linear": 2}
GHOSTS = {"default": 0, "bilinear": 1}
STEPS = {"half_sweep": 0, "resid_restrict": 1, "coarse_rhs": 2, "prolong": 3, "coarse": 4}
LISTS = {"all": 0, "parent": 1, "leaf": 2}
KINDS = {"gsrb": 0, "resid": 1, "coarse_rhs": 2, "prolong": 3, "final": 4}
OPS = {"L": 0, "LT": 1}

_lib = None


class AfmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"afmg error {code}: {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # PyTorch bundles its own HIP runtime.  Load it first so that the
        # library binds to that same runtime (matched by soname); two HIP
        # runtimes in one process cannot share the device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32p, i64 = C.c_void_p, C.POINTER(C.c_int32), C.c_int64
        L.afmg_default_opts.argtypes = [C.POINTER(Opts)]
        L.afmg_default_opts.restype = None
        L.afmg_tree_create.argtypes = [C.c_int, C.c_int, i64, i32p, i32p, C.POINTER(vp)]
        L.afmg_tree_create_domain.argtypes = [C.c_int, C.c_int, i32p, i64, i32p, i32p, C.POINTER(vp)]
        L.afmg_tree_destroy.argtypes = [vp]
        L.afmg_tree_destroy.restype = None
        L.afmg_tree_info.argtypes = [vp, C.POINTER(TreeDesc)]
        L.afmg_tree_leaf_boxes.argtypes = [vp, i32p]
        L.afmg_tree_bfaces.argtypes = [vp, i32p]
        L.afmg_tree_box.argtypes = [vp, i64, C.POINTER(BoxDesc)]
        L.afmg_workspace_bytes.argtypes = [vp, C.POINTER(Opts), C.POINTER(C.c_size_t)]
        L.afmg_solve_bytes_model.argtypes = [vp, C.POINTER(Opts), C.c_int, C.POINTER(C.c_double)]
        L.afmg_solve.argtypes = [vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(Opts), C.POINTER(Stats)]
        L.afmg_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, C.POINTER(Opts), C.POINTER(Stats)]
        L.afmg_last_error.restype = C.c_char_p
        L.afmg_adjoint_workspace_bytes.argtypes = [vp, C.POINTER(Opts), C.POINTER(C.c_size_t)]
        L.afmg_apply.argtypes = [vp, vp, C.c_int, vp, vp, vp, C.c_size_t]
        L.afmg_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(Opts), C.POINTER(Stats)]
        L.afmg_batch_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp)]
        L.afmg_batch_destroy.argtypes = [vp]
        L.afmg_batch_destroy.restype = None
        L.afmg_batch_info.argtypes = [vp, C.POINTER(BatchDesc)]
        L.afmg_batch_workspace_bytes.argtypes = [vp, C.POINTER(Opts), C.POINTER(C.c_size_t)]
        L.afmg_batch_solve.argtypes = [vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(Opts), C.POINTER(Stats)]
        ip = C.POINTER(C.c_int)
        for pre in ("tree", "batch"):
            getattr(L, f"afmg_{pre}_autotune").argtypes = [vp, vp, vp, C.c_size_t]
            getattr(L, f"afmg_{pre}_shape").argtypes = [vp, C.c_int, C.c_int, C.c_int, ip, ip]
            getattr(L, f"afmg_{pre}_set_shape").argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.afmg_autotune_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.afmg_tree_refine.argtypes = [vp, i32p, i64, C.c_int, C.POINTER(vp)]
        L.afmg_tree_finalize.argtypes = [vp, vp]
        L.afmg_tree_level_list.argtypes = [vp, C.c_int, C.c_int, i32p, C.POINTER(C.c_int64)]
        L.afmg_step.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, C.c_size_t,
                                C.POINTER(Opts)]
        L.afmg_batch_autotune_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.afmg_tree_set_operator.argtypes = [vp, vp, C.c_int, vp, C.c_int]
        L.afmg_tree_set_ghost_scheme.argtypes = [vp, vp, C.c_int]
        L.afmg_tree_adapt.argtypes = [vp, vp, vp, C.c_int, C.POINTER(vp), C.POINTER(C.c_int64)]
        L.afmg_transfer_workspace_bytes.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.afmg_tree_transfer.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_size_t]
        _lib = L
    return _lib


def last_error():
    return lib().afmg_last_error().decode()


def _check(rc, allow=(AFMG_OK,)):
    if rc not in allow:
        raise AfmgError(rc, last_error())
    return rc


def make_opts(cycle="V", n_down=2, n_up=2, n_base=4, tol=1e-10, max_cycles=100, fixed_cycles=0,
              use_guess=False, precision="fp64", profile=False, graph=False, check_every=1, prof_level=0):
    o = Opts()
    lib().afmg_default_opts(C.byref(o))
    o.cycle = CYCLES[cycle]
    o.n_down, o.n_up, o.n_base = n_down, n_up, n_base
    o.tol = tol
    o.max_cycles = max_cycles
    o.fixed_cycles = fixed_cycles
    o.use_guess = 1 if use_guess else 0
    o.precision = PRECISIONS[precision]
    o.profile = 1 if profile else 0
    o.graph = 1 if graph else 0
    o.check_every = check_every
    o.prof_level = prof_level
    return o


class _Shapes:
    """Launch shapes and the autotuner (shared by Tree and Batch)."""

    _pre = "tree"

    def shape(self, precision, kind, level):
        """(workgroup size, no_remap) of a kernel class on a level."""
        wg, nr = C.c_int(), C.c_int()
        _check(getattr(lib(), f"afmg_{self._pre}_shape")(self._h, PRECISIONS.get(precision, precision),
                                                          KINDS.get(kind, kind), level, C.byref(wg), C.byref(nr)))
        return wg.value, nr.value

    def shapes(self):
        out = {}
        for p in ("fp64", "mixed"):
            for k in KINDS:
                if k == "final" and p == "mixed":
                    continue
                out[(p, k)] = [self.shape(p, k, l) for l in range(1, self.lmax + 1)]
        return out

    def set_shape(self, wg, no_remap=0, precision=-1, kind=-1, level=-1):
        _check(getattr(lib(), f"afmg_{self._pre}_set_shape")(self._h, PRECISIONS.get(precision, precision),
                                                              KINDS.get(kind, kind), level, wg, no_remap))

    def autotune(self, device=None, stream=None):
        """Time every launch shape on this grid and keep the fastest."""
        import torch
        dev = device or torch.device("cuda", 0)
        n = C.c_size_t()
        _check(getattr(lib(), f"afmg_{'' if self._pre == 'tree' else 'batch_'}autotune_workspace_bytes")(
            self._h, C.byref(n)))
        ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        with torch.cuda.device(dev):
            _check(getattr(lib(), f"afmg_{self._pre}_autotune")(self._h, C.c_void_p(stream.cuda_stream),
                                                                 C.c_void_p(ws.data_ptr()), n.value))
        return self.shapes()


class Tree(_Shapes):
    """A quadtree/octree of 8^D-cell boxes built from its leaves.  With
    bc_type (see bc_type_codes) the domain is general: the level-1 boxes
    holding the leaves form the coarse grid on an integer lattice, and each
    side orientation is Dirichlet, Neumann or periodic
    (afmg_tree_create_domain)."""

    def __init__(self, dim, level=None, idx=None, box_n=8, _handle=None, bc_type=None):
        L = lib()
        if _handle is not None:
            h = _handle
        else:
            level = np.ascontiguousarray(level, dtype=np.int32)
            idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
            if len(level) != len(idx):
                raise ValueError("level and idx lengths differ")
            h = C.c_void_p()
            i32p = C.POINTER(C.c_int32)
            if bc_type is None:
                _check(L.afmg_tree_create(dim, box_n, len(level), level.ctypes.data_as(i32p),
                                          idx.ctypes.data_as(i32p), C.byref(h)))
            else:
                codes = bc_type_codes(bc_type, dim)
                _check(L.afmg_tree_create_domain(dim, box_n, codes.ctypes.data_as(i32p), len(level),
                                                 level.ctypes.data_as(i32p), idx.ctypes.data_as(i32p),
                                                 C.byref(h)))
        self._h = h
        d = TreeDesc()
        _check(L.afmg_tree_info(h, C.byref(d)))
        self.dim, self.box_n = d.dim, d.box_n
        self.n_boxes, self.n_leaves, self.n_bfaces = d.n_boxes, d.n_leaves, d.n_bfaces
        self.lmin, self.lmax = d.lmin, d.lmax
        self.cells_per_box = d.cells_per_box
        self.n_unknowns = d.n_unknowns
        self.n_roots = d.n_roots
        self.ext = tuple(d.ext)
        self.bc_type = tuple(d.bc_type[: 2 * self.dim])
        self.singular = bool(d.singular)
        self.leaf_boxes = np.zeros(self.n_leaves, np.int32)
        _check(L.afmg_tree_leaf_boxes(h, self.leaf_boxes.ctypes.data_as(C.POINTER(C.c_int32))))
        bf = np.zeros(2 * max(1, self.n_bfaces), np.int32)
        _check(L.afmg_tree_bfaces(h, bf.ctypes.data_as(C.POINTER(C.c_int32))))
        self.bfaces = bf[: 2 * self.n_bfaces].reshape(-1, 2)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.afmg_tree_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def box(self, b):
        d = BoxDesc()
        _check(lib().afmg_tree_box(self._h, b, C.byref(d)))
        return dict(level=d.level, idx=tuple(d.idx), parent=d.parent, leaf=bool(d.leaf), nbr=tuple(d.nbr),
                    children=tuple(d.children[: 2 ** self.dim]), x_lo=tuple(d.x_lo), h=d.h)

    def refine(self, box_ids, balance=1):
        """A new tree with the given leaf boxes refined (afmg_tree_refine)."""
        ids = np.ascontiguousarray(box_ids, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().afmg_tree_refine(self._h, ids.ctypes.data_as(C.POINTER(C.c_int32)), len(ids), balance,
                                      C.byref(h)))
        return Tree(self.dim, _handle=h)

    def finalize(self):
        _check(lib().afmg_tree_finalize(self._h, None))

    def set_operator(self, kind="laplacian", eps=None, prolong="default"):
        """Operator of later solves (afmg_tree_set_operator): "laplacian",
        "eps", "cyl" or "cyl_eps"; eps a float64 CUDA tensor [n_boxes, N^D]
        in box order (leaf boxes read); prolong "default", "eps" or
        "linear" (bi/trilinear)."""
        code = OPERATORS[kind] if isinstance(kind, str) else int(kind)
        pro = PROLONGS[prolong] if isinstance(prolong, str) else int(prolong)
        if eps is not None:
            if eps.dtype != __import__("torch").float64 or not eps.is_cuda or not eps.is_contiguous():
                raise ValueError("eps must be a contiguous float64 CUDA tensor")
            if eps.numel() != self.n_boxes * self.cells_per_box:
                raise ValueError("eps must hold n_boxes x N^D values")
        import torch
        dev = eps.device if eps is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(dev):
            stream = torch.cuda.current_stream(dev)
            _check(lib().afmg_tree_set_operator(self._h, C.c_void_p(stream.cuda_stream), code, _ptr(eps), pro))
        self.operator = (code, pro)

    def set_ghost_scheme(self, scheme="default"):
        """Refinement-boundary ghosts of later solves
        (afmg_tree_set_ghost_scheme): "default" or "bilinear"."""
        _check(lib().afmg_tree_set_ghost_scheme(self._h, None, GHOSTS[scheme] if isinstance(scheme, str)
                                                else int(scheme)))
        self.ghost_scheme = scheme

    def level_list(self, level, kind="all"):
        n = C.c_int64()
        L = lib()
        _check(L.afmg_tree_level_list(self._h, level, LISTS[kind], None, C.byref(n)))
        out = np.zeros(max(1, n.value), np.int32)
        _check(L.afmg_tree_level_list(self._h, level, LISTS[kind], out.ctypes.data_as(C.POINTER(C.c_int32)),
                                      C.byref(n)))
        return out[: n.value]

    def leaves(self):
        """(level, idx) of the leaves in the tree's input order."""
        boxes = [self.box(int(b)) for b in self.leaf_boxes]
        return (np.array([b["level"] for b in boxes], np.int32),
                np.array([b["idx"] for b in boxes], np.int32).reshape(-1, 3))

    def adjoint_workspace_bytes(self, opts=None):
        n = C.c_size_t()
        _check(lib().afmg_adjoint_workspace_bytes(self._h, C.byref(opts) if opts is not None else None,
                                                  C.byref(n)))
        return n.value

    def workspace_bytes(self, opts=None):
        n = C.c_size_t()
        _check(lib().afmg_workspace_bytes(self._h, C.byref(opts) if opts is not None else None, C.byref(n)))
        return n.value

    def bytes_model(self, v_cycles, opts=None):
        """Algorithmic HBM bytes of an FP64 solve with v_cycles V-cycles
        (after the FMG cycle when opts.cycle is FMG); host-only."""
        b = C.c_double()
        _check(lib().afmg_solve_bytes_model(self._h, C.byref(opts) if opts is not None else None, v_cycles,
                                            C.byref(b)))
        return b.value

    # ---- marshalling between the caller's leaf order and box order ---------
    def leaf_to_boxes(self, leaf_field):
        """[n_leaves, N^D] (leaf order) -> [n_boxes, N^D] (box order, zero on
        parents); works for numpy arrays and torch tensors."""
        if hasattr(leaf_field, "new_zeros"):
            import torch
            out = leaf_field.new_zeros((self.n_boxes, self.cells_per_box))
            out[torch.as_tensor(self.leaf_boxes, device=leaf_field.device).long()] = leaf_field.reshape(
                self.n_leaves, -1)
            return out
        out = np.zeros((self.n_boxes, self.cells_per_box), dtype=leaf_field.dtype)
        out[self.leaf_boxes] = leaf_field.reshape(self.n_leaves, -1)
        return out

    def boxes_to_leaf(self, box_field):
        if hasattr(box_field, "new_zeros"):
            import torch
            return box_field.reshape(self.n_boxes, -1)[torch.as_tensor(self.leaf_boxes, device=box_field.device).long()]
        return box_field.reshape(self.n_boxes, -1)[self.leaf_boxes]

    def bc_rows(self, bc_leaf):
        """Dirichlet values [n_leaves, 2D, N^(D-1)] (leaf order) -> the rows
        [n_bfaces, N^(D-1)] the library reads."""
        box_to_leaf = np.full(self.n_boxes, -1, np.int64)
        box_to_leaf[self.leaf_boxes] = np.arange(self.n_leaves)
        q = box_to_leaf[self.bfaces[:, 0]]
        s = self.bfaces[:, 1]
        if hasattr(bc_leaf, "new_zeros"):
            import torch
            dev = bc_leaf.device
            return bc_leaf[torch.as_tensor(q, device=dev), torch.as_tensor(s, device=dev)].contiguous()
        return np.ascontiguousarray(bc_leaf[q, s])


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def adapt(tree: Tree, flags, n_buf=2, stream=None):
    """afmg_tree_adapt: the tree after one mesh adaptation (paper §2.3).
    flags: int8 CUDA tensor [n_boxes, N^D] in box order (> 0 refine, < 0
    derefine, 0 keep; leaf boxes read).  Returns (new Tree, (boxes refined,
    boxes whose children were removed))."""
    import torch

    if flags.dtype != torch.int8 or not flags.is_cuda or not flags.is_contiguous() or \
            flags.numel() != tree.n_boxes * tree.cells_per_box:
        raise ValueError("flags must be a contiguous int8 CUDA tensor of n_boxes x N^D values")
    if stream is None:
        stream = torch.cuda.current_stream(flags.device)
    h = C.c_void_p()
    counts = (C.c_int64 * 2)()
    with torch.cuda.device(flags.device):
        _check(lib().afmg_tree_adapt(tree.handle, C.c_void_p(stream.cuda_stream), _ptr(flags), n_buf, C.byref(h),
                                     counts))
    return Tree(tree.dim, _handle=h), (counts[0], counts[1])


def transfer(src: Tree, dst: Tree, u, bc=None, out=None, workspace=None, stream=None):
    """afmg_tree_transfer: the cell field u (float64 CUDA tensor [n_boxes(src),
    N^D], box order) on tree dst; bc: src's boundary rows or None."""
    import torch

    _check_field(src, u, "u")
    if out is None:
        out = torch.empty((dst.n_boxes, dst.cells_per_box), dtype=torch.float64, device=u.device)
    _check_field(dst, out, "out")
    n = C.c_size_t()
    _check(lib().afmg_transfer_workspace_bytes(src.handle, dst.handle, C.byref(n)))
    if workspace is None or workspace.numel() * workspace.element_size() < n.value:
        workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=u.device)
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    with torch.cuda.device(u.device):
        _check(lib().afmg_tree_transfer(src.handle, dst.handle, C.c_void_p(stream.cuda_stream), _ptr(u), _ptr(bc),
                                        _ptr(out), _ptr(workspace), n.value))
    return out


def solve(tree: Tree, rho, bc=None, u=None, *, cycle="V", tol=1e-10, max_cycles=100, fixed_cycles=0,
          n_down=2, n_up=2, n_base=4, precision="fp64", workspace=None, stream=None, check=True,
          profile=False, use_guess=None, graph=False, check_every=1, prof_level=0):
    """Solve lap_h(u) = rho on `tree`.

    rho, u: torch float64 CUDA tensors [n_boxes, N^D] in box order; bc:
    [n_bfaces, N^(D-1)] Dirichlet rows or None (zero).  u (if given) is the
    initial guess (unless use_guess=False) and is overwritten; otherwise a
    new tensor is returned.  Returns (u, stats dict)."""
    import torch

    dev = rho.device
    if dev.type != "cuda":
        raise ValueError("rho must be a device tensor")
    shape = (tree.n_boxes, tree.cells_per_box)
    if rho.dtype != torch.float64 or tuple(rho.shape) != shape or not rho.is_contiguous():
        raise ValueError(f"rho must be contiguous float64 {shape}")
    if use_guess is None:
        use_guess = u is not None
    if u is None:
        u = torch.empty(shape, dtype=torch.float64, device=dev)
    elif u.dtype != torch.float64 or tuple(u.shape) != shape or not u.is_contiguous():
        raise ValueError(f"u must be contiguous float64 {shape}")
    if bc is not None:
        if bc.dtype != torch.float64 or bc.numel() != tree.n_bfaces * tree.box_n ** (tree.dim - 1):
            raise ValueError("bc has the wrong dtype or size")
        bc = bc.contiguous()
    opts = make_opts(cycle, n_down, n_up, n_base, tol, max_cycles, fixed_cycles, use_guess, precision,
                     profile, graph, check_every, prof_level)
    nbytes = tree.workspace_bytes(opts)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    st = Stats()
    with torch.cuda.device(dev):
        rc = lib().afmg_solve(tree.handle, C.c_void_p(stream.cuda_stream), _ptr(rho), _ptr(bc), _ptr(u),
                              _ptr(workspace), nbytes, C.byref(opts), C.byref(st))
    if check:
        _check(rc, allow=(AFMG_OK, AFMG_NOT_CONVERGED))
    d = st.to_dict()
    d["rc"] = rc
    return u, d


SCRATCH_BYTES = 128 << 20  # AFMG_SCRATCH_BYTES


def solve_noalloc(tree: Tree, rho, bc, u, *, cycle="V", tol=1e-10, max_cycles=100, fixed_cycles=0, n_down=2,
                  n_up=2, n_base=4, precision="fp64", stream=None, check=True, use_guess=False, check_every=1):
    """afmg_solve_noalloc: the solve with the library's own scratch array as
    its workspace (nothing is allocated; the tree must be finalized on the
    device).  rho, u: float64 device tensors [n_boxes, N^D] in box order, u
    overwritten; bc: Dirichlet rows or None.  Returns (rc, stats dict)."""
    import torch

    for t_, name in ((rho, "rho"), (u, "u")):
        _check_field(tree, t_, name)
    if bc is not None and (bc.dtype != torch.float64 or not bc.is_contiguous()
                           or bc.numel() != tree.n_bfaces * tree.box_n ** (tree.dim - 1)):
        raise ValueError("bc has the wrong dtype, layout or size")
    opts = make_opts(cycle, n_down, n_up, n_base, tol, max_cycles, fixed_cycles, use_guess, precision, False,
                     False, check_every)
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    st = Stats()
    with torch.cuda.device(u.device):
        rc = lib().afmg_solve_noalloc(tree.handle, C.c_void_p(stream.cuda_stream), _ptr(rho), _ptr(bc), _ptr(u),
                                      C.byref(opts), C.byref(st))
    if check:
        _check(rc, allow=(AFMG_OK, AFMG_NOT_CONVERGED))
    d = st.to_dict()
    d["rc"] = rc
    return rc, d


class Batch(_Shapes):
    """Independent trees of one dimension solved together (afmg_batch_*).

    Fields are the trees' [n_boxes, N^D] arrays one after the other (each in
    its tree's box order); `concat` and `split` convert from / to lists."""

    _pre = "batch"

    def __init__(self, trees):
        trees = list(trees)
        if not trees:
            raise ValueError("empty batch")
        L = lib()
        arr = (C.c_void_p * len(trees))(*[t.handle for t in trees])
        h = C.c_void_p()
        _check(L.afmg_batch_create(arr, len(trees), C.byref(h)))
        self._h = h
        d = BatchDesc()
        _check(L.afmg_batch_info(h, C.byref(d)))
        self.dim, self.box_n, self.n_trees, self.lmax = d.dim, d.box_n, d.n_trees, d.lmax
        self.n_boxes, self.n_bfaces, self.n_unknowns = d.n_boxes, d.n_bfaces, d.n_unknowns
        self.cells_per_box = trees[0].cells_per_box
        self.box_counts = [t.n_boxes for t in trees]
        self.bface_counts = [t.n_bfaces for t in trees]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.afmg_batch_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, opts=None):
        n = C.c_size_t()
        _check(lib().afmg_batch_workspace_bytes(self._h, C.byref(opts) if opts is not None else None,
                                                C.byref(n)))
        return n.value

    def concat(self, fields):
        import torch
        return torch.cat([f.reshape(n, -1) for f, n in zip(fields, self.box_counts)]).contiguous()

    def concat_bc(self, rows):
        import torch
        parts = [r.reshape(n, -1) for r, n in zip(rows, self.bface_counts) if n > 0]
        return torch.cat(parts).contiguous() if parts else None

    def split(self, field):
        return list(field.reshape(self.n_boxes, -1).split(self.box_counts))


def solve_batch(batch: Batch, rho, bc=None, u=None, *, cycle="V", tol=1e-10, max_cycles=100, fixed_cycles=0,
                n_down=2, n_up=2, n_base=4, precision="fp64", workspace=None, stream=None, check=True,
                profile=False, use_guess=None, graph=False, check_every=1, prof_level=0):
    """afmg_solve on every tree of the batch.  rho, u: float64 device tensors
    [batch.n_boxes, N^D] (the trees' arrays one after the other); bc: the
    trees' Dirichlet rows one after the other, or None.  Returns (u, list of
    per-tree stats dicts)."""
    import torch

    dev = rho.device
    shape = (batch.n_boxes, batch.cells_per_box)
    if dev.type != "cuda" or rho.dtype != torch.float64 or tuple(rho.shape) != shape or not rho.is_contiguous():
        raise ValueError(f"rho must be a contiguous float64 device tensor {shape}")
    if use_guess is None:
        use_guess = u is not None
    if u is None:
        u = torch.empty(shape, dtype=torch.float64, device=dev)
    elif u.dtype != torch.float64 or tuple(u.shape) != shape or not u.is_contiguous():
        raise ValueError(f"u must be contiguous float64 {shape}")
    if bc is not None:
        if bc.dtype != torch.float64 or bc.numel() != batch.n_bfaces * batch.box_n ** (batch.dim - 1):
            raise ValueError("bc has the wrong dtype or size")
        bc = bc.contiguous()
    opts = make_opts(cycle, n_down, n_up, n_base, tol, max_cycles, fixed_cycles, use_guess, precision,
                     profile, graph, check_every, prof_level)
    nbytes = batch.workspace_bytes(opts)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    sts = (Stats * batch.n_trees)()
    with torch.cuda.device(dev):
        rc = lib().afmg_batch_solve(batch.handle, C.c_void_p(stream.cuda_stream), _ptr(rho), _ptr(bc), _ptr(u),
                                    _ptr(workspace), nbytes, C.byref(opts), sts)
    if check:
        _check(rc, allow=(AFMG_OK, AFMG_NOT_CONVERGED))
    out = []
    for s in sts:
        d = s.to_dict()
        d["rc"] = rc
        out.append(d)
    return u, out


def step(tree: Tree, op, level, u, rho, uold, bc=None, colour=0, homog=False, n_down=2, n_up=2, n_base=4,
         workspace=None, stream=None):
    """One step of the cycle (afmg_step) in place on u, rho, uold: float64
    device tensors [n_boxes, N^D] in box order."""
    import torch
    for t_, name in ((u, "u"), (rho, "rho"), (uold, "uold")):
        _check_field(tree, t_, name)
    opts = make_opts("V", n_down, n_up, n_base)
    nbytes = tree.workspace_bytes(opts)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=u.device)
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    with torch.cuda.device(u.device):
        _check(lib().afmg_step(tree.handle, C.c_void_p(stream.cuda_stream), STEPS[op], level, colour,
                               1 if homog else 0, _ptr(u), _ptr(rho), _ptr(uold),
                               _ptr(bc.contiguous()) if bc is not None else None, _ptr(workspace), nbytes,
                               C.byref(opts)))


def _check_field(tree, t, name):
    import torch
    shape = (tree.n_boxes, tree.cells_per_box)
    if t.device.type != "cuda" or t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor {shape}")


def apply(tree: Tree, x, op="L", workspace=None, stream=None):
    """y = L x (op "L") or L^T x (op "LT") on the leaf cells, zero Dirichlet
    values; x, y: float64 device tensors [n_boxes, N^D]."""
    import torch
    _check_field(tree, x, "x")
    y = torch.empty_like(x)
    nbytes = tree.adjoint_workspace_bytes()
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=x.device)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    with torch.cuda.device(x.device):
        _check(lib().afmg_apply(tree.handle, C.c_void_p(stream.cuda_stream), OPS[op], _ptr(x), _ptr(y),
                                _ptr(workspace), nbytes))
    return y


def adjoint(tree: Tree, u_bar, *, tol=1e-10, max_cycles=200, n_down=2, n_up=2, n_base=4, workspace=None,
            stream=None, check=True):
    """Gradients of a loss with respect to rho and the Dirichlet rows given
    u_bar = dloss/du (float64 device [n_boxes, N^D]).  Returns (rho_bar,
    bc_bar, stats)."""
    import torch
    _check_field(tree, u_bar, "u_bar")
    dev = u_bar.device
    rho_bar = torch.empty_like(u_bar)
    bc_bar = torch.zeros((max(tree.n_bfaces, 1), tree.box_n ** (tree.dim - 1)), dtype=torch.float64, device=dev)
    opts = make_opts("V", n_down, n_up, n_base, tol, max_cycles, 0, False, "fp64")
    nbytes = tree.adjoint_workspace_bytes(opts)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    st = Stats()
    with torch.cuda.device(dev):
        rc = lib().afmg_adjoint(tree.handle, C.c_void_p(stream.cuda_stream), _ptr(u_bar.contiguous()),
                                _ptr(rho_bar), _ptr(bc_bar) if tree.n_bfaces else None, _ptr(workspace), nbytes,
                                C.byref(opts), C.byref(st))
    if check:
        _check(rc, allow=(AFMG_OK, AFMG_NOT_CONVERGED))
    d = st.to_dict()
    d["rc"] = rc
    return rho_bar, bc_bar[: tree.n_bfaces], d


def _autograd_function():
    import torch

    class PoissonSolve(torch.autograd.Function):
        """u = L^-1 (rho - B b): forward = afmg_solve, backward = afmg_adjoint."""

        @staticmethod
        def forward(ctx, rho, bc, tree, opts):
            u, st = solve(tree, rho.detach().contiguous(), None if bc is None else bc.detach().contiguous(),
                          **opts)
            if st["status"] != AFMG_OK:
                warnings.warn(f"poisson_solve: forward solve not converged (status {st['status']}, "
                              f"residual ratio {st['r_max'] / max(st['r0_max'], 1e-300):.2e})", RuntimeWarning)
            ctx.tree = tree
            ctx.opts = opts
            ctx.has_bc = bc is not None
            ctx.stats = st
            return u

        @staticmethod
        def backward(ctx, u_bar):
            o = ctx.opts
            rho_bar, bc_bar, st = adjoint(ctx.tree, u_bar.contiguous(), tol=o.get("tol", 1e-10),
                                          max_cycles=max(o.get("max_cycles", 100), 200),
                                          n_down=o.get("n_down", 2), n_up=o.get("n_up", 2),
                                          n_base=o.get("n_base", 4))
            if st["status"] != AFMG_OK:
                warnings.warn(f"poisson_solve: adjoint solve not converged (status {st['status']}, "
                              f"residual ratio {st['r_max'] / max(st['r0_max'], 1e-300):.2e})", RuntimeWarning)
            return rho_bar, (bc_bar if ctx.has_bc else None), None, None

    return PoissonSolve


_PS = None


def poisson_solve(tree: Tree, rho, bc=None, **opts):
    """Differentiable solve: gradients flow to rho (leaf boxes) and to the
    Dirichlet rows bc through the adjoint (one more multigrid solve on
    uniform grids, preconditioned BiCGSTAB on L^T otherwise)."""
    global _PS
    if _PS is None:
        _PS = _autograd_function()
    return _PS.apply(rho, bc, tree, opts)
