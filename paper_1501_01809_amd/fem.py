"""Thin ctypes binding of ``libfem.so`` (include/fem.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.
Function names are the C ABI's names.  Importing this module never falls back
to anything: if the HIP library is missing, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfem.so")

FEM_OK, FEM_E_ARG, FEM_E_RANGE, FEM_E_OVERFLOW, FEM_E_UNSUPPORTED, FEM_E_NOMEM, FEM_E_DEVICE = range(7)
STATUS_NAMES = {0: "FEM_OK", 1: "FEM_E_ARG", 2: "FEM_E_RANGE", 3: "FEM_E_OVERFLOW",
                4: "FEM_E_UNSUPPORTED", 5: "FEM_E_NOMEM", 6: "FEM_E_DEVICE"}
FEM_READ, FEM_WRITE, FEM_INC, FEM_SUM, FEM_MIN, FEM_MAX = 0, 1, 2, 3, 4, 5
FEM_SERVE_FIFO, FEM_SERVE_SHORTEST = 0, 1
FEM_TRIANGLE, FEM_TETRAHEDRON = 2, 3
FEM_FP64, FEM_FP32, FEM_BF16, FEM_FP16 = 0, 1, 2, 3
FEM_MASS, FEM_LAPLACE, FEM_HELMHOLTZ, FEM_SOURCE, FEM_NL_RESIDUAL, FEM_ELASTICITY = 0, 1, 2, 3, 4, 5

KINDS = {"mass": FEM_MASS, "laplace": FEM_LAPLACE, "helmholtz": FEM_HELMHOLTZ, "source": FEM_SOURCE,
         "nl_residual": FEM_NL_RESIDUAL, "elasticity": FEM_ELASTICITY}
PRECS = {"fp64": FEM_FP64, "fp32": FEM_FP32, "bf16": FEM_BF16, "fp16": FEM_FP16}


class FemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fem_set(C.Structure):
    _fields_ = [("size", C.c_int64)]


class fem_map(C.Structure):
    _fields_ = [("from_", C.POINTER(fem_set)), ("to", C.POINTER(fem_set)),
                ("arity", C.c_int32), ("values", C.c_void_p), ("version", C.c_uint64)]


class fem_dat(C.Structure):
    _fields_ = [("set", C.POINTER(fem_set)), ("dim", C.c_int32), ("data", C.c_void_p)]


class fem_sparsity(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class fem_mat(C.Structure):
    _fields_ = [("sp", C.POINTER(fem_sparsity)), ("values", C.c_void_p)]


class fem_global(C.Structure):
    _fields_ = [("data", C.c_void_p)]


class fem_facets(C.Structure):
    _fields_ = [("facets", C.POINTER(fem_set)), ("facet_vertex", C.POINTER(fem_map)),
                ("facet_node", C.POINTER(fem_map)), ("coords", C.POINTER(fem_dat)), ("g", C.POINTER(fem_dat))]


class fem_block(C.Structure):
    _fields_ = [("kind", C.c_int), ("scale", C.c_double), ("coeff", C.POINTER(fem_dat))]


class fem_form(C.Structure):
    _fields_ = [("kind", C.c_int), ("cell", C.c_int), ("degree", C.c_int32),
                ("dim", C.c_int32), ("prec", C.c_int), ("qdegree", C.c_int32)]


class fem_args(C.Structure):
    _fields_ = [("cells", C.POINTER(fem_set)), ("cell_vertex", C.POINTER(fem_map)),
                ("coords", C.POINTER(fem_dat)), ("cell_node", C.POINTER(fem_map)),
                ("coeff", C.POINTER(fem_dat) * 4), ("ncoeff", C.c_int32),
                ("cell_coord", C.POINTER(fem_map))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

EXPORTS = ["fem_ctx_create", "fem_ctx_destroy", "fem_ctx_set_stream", "fem_ctx_set_allocator", "fem_last_error",
           "fem_sync",
           "fem_build_sparsity", "fem_build_sparsity_noalloc", "fem_plan_create", "fem_plan_destroy", "fem_plan_info",
           "fem_par_loop_assemble_mat", "fem_par_loop_assemble_vec", "fem_apply_action",
           "fem_par_loop_assemble_adjoint", "fem_renumber", "fem_expand_sparsity",
           "fem_server_create", "fem_server_destroy", "fem_server_add_model", "fem_server_submit",
           "fem_server_poll", "fem_server_result", "fem_server_release", "fem_server_model_info",
           "fem_server_configure", "fem_server_set_batch", "fem_server_set_order", "fem_server_take_completed", "fem_par_loop_reduce",
           "fem_apply_dirichlet", "fem_par_loop_assemble_mixed", "fem_facet_plan_create",
           "fem_par_loop_assemble_facets"]
FEM_REQ_ASSEMBLE, FEM_REQ_ACTION = 0, 1

_lib = None


def lib():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.fem_ctx_create.argtypes = [C.c_int, P, C.POINTER(P)]
        L.fem_ctx_destroy.argtypes = [P]; L.fem_ctx_destroy.restype = None
        L.fem_ctx_set_stream.argtypes = [P, P]
        L.fem_ctx_set_allocator.argtypes = [P, ALLOC_FN, RELEASE_FN, P]
        L.fem_last_error.argtypes = [P]; L.fem_last_error.restype = C.c_char_p
        L.fem_sync.argtypes = [P]
        L.fem_build_sparsity.argtypes = [P, C.POINTER(fem_map), C.POINTER(fem_map), C.POINTER(fem_sparsity), P,
                                         C.POINTER(C.c_size_t)]
        L.fem_build_sparsity_noalloc.argtypes = [P, C.POINTER(fem_map), C.POINTER(fem_map),
                                                 C.POINTER(fem_sparsity)]
        L.fem_plan_create.argtypes = [P, C.POINTER(fem_form), C.POINTER(fem_args), C.POINTER(fem_sparsity),
                                      C.POINTER(P)]
        L.fem_plan_destroy.argtypes = [P]; L.fem_plan_destroy.restype = None
        L.fem_plan_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.fem_par_loop_assemble_mat.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_args),
                                                C.POINTER(fem_mat), C.c_int]
        L.fem_par_loop_assemble_vec.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_args),
                                                C.POINTER(fem_dat), C.c_int]
        L.fem_apply_action.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_args), C.POINTER(fem_dat),
                                       C.POINTER(fem_dat), C.c_int]
        L.fem_par_loop_assemble_adjoint.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_args),
                                                    C.POINTER(fem_dat), C.POINTER(fem_dat), C.POINTER(fem_dat),
                                                    C.c_int]
        L.fem_renumber.argtypes = [P, C.POINTER(fem_form), C.POINTER(fem_args), P, P, P]
        L.fem_facet_plan_create.argtypes = [P, C.POINTER(fem_form), C.POINTER(fem_facets), C.POINTER(P)]
        L.fem_par_loop_assemble_facets.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_facets),
                                                   C.POINTER(fem_dat), C.c_int]
        L.fem_par_loop_assemble_mixed.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_args), C.c_int32,
                                                  C.POINTER(fem_block), C.POINTER(fem_mat), C.c_int]
        L.fem_apply_dirichlet.argtypes = [P, C.POINTER(fem_sparsity), P, P, C.c_double, P, P]
        L.fem_par_loop_reduce.argtypes = [P, P, C.POINTER(fem_form), C.POINTER(fem_args), C.POINTER(fem_dat),
                                          C.POINTER(fem_global), C.c_int]
        L.fem_expand_sparsity.argtypes = [P, C.POINTER(fem_sparsity), C.c_int32, C.POINTER(fem_sparsity)]
        I64p = C.POINTER(C.c_int64)
        L.fem_server_create.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(P)]
        L.fem_server_destroy.argtypes = [P]; L.fem_server_destroy.restype = None
        L.fem_server_add_model.argtypes = [P, C.POINTER(fem_form), C.POINTER(fem_args), C.POINTER(C.c_int32), I64p]
        L.fem_server_submit.argtypes = [P, C.c_int32, C.c_int32, P, C.c_double, I64p]
        L.fem_server_poll.argtypes = [P, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
        L.fem_server_result.argtypes = [P, C.c_int64, C.POINTER(P), C.POINTER(P), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.fem_server_release.argtypes = [P, C.c_int64]
        L.fem_server_configure.argtypes = [P, C.c_int32, C.c_int32]
        L.fem_server_set_order.argtypes = [P, C.c_int32, C.c_double]
        L.fem_server_set_batch.argtypes = [P, C.c_int32, C.c_double]
        L.fem_server_take_completed.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32)]
        L.fem_server_model_info.argtypes = [P, C.c_int32, I64p, I64p, I64p, C.POINTER(P), C.POINTER(P)]
        for name in EXPORTS:
            if name not in ("fem_ctx_destroy", "fem_plan_destroy", "fem_last_error", "fem_server_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


class Context:
    """fem_ctx bound to a device and to torch's current stream on it.  With
    torch_memory (the default) the library's device memory (plans, setup
    temporaries) comes from torch's caching allocator on that stream, so it
    is visible to torch and reused by it; otherwise from the HIP runtime."""

    def __init__(self, device: int = 0, stream=None, torch_memory: bool = True):
        import torch
        L = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.h = C.c_void_p()
        st = L.fem_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(self.h))
        if st != FEM_OK:
            raise FemError(st, "fem_ctx_create failed")
        self._alloc = self._release = None
        self._callbacks = []   # every allocator installed: plans keep calling theirs
        if torch_memory:
            self.set_allocator(*torch_allocator(device, stream))

    def set_allocator(self, alloc, release):
        """alloc(nbytes) -> device address (int, 0 on failure) and
        release(address); both None restore the HIP runtime.  The callables
        are kept alive by the context."""
        if alloc is None:
            self._alloc = self._release = None
            self.check(lib().fem_ctx_set_allocator(self.h, ALLOC_FN(), RELEASE_FN(), None))
            return

        def _a(n, user):
            try:
                return alloc(n) or None
            except Exception:
                return None

        def _r(p, user):
            try:
                release(p)
            except Exception:
                pass

        self._alloc, self._release = ALLOC_FN(_a), RELEASE_FN(_r)
        self._callbacks.append((self._alloc, self._release))
        self.check(lib().fem_ctx_set_allocator(self.h, self._alloc, self._release, None))

    def check(self, st):
        if st != FEM_OK:
            raise FemError(st, lib().fem_last_error(self.h).decode())

    def set_stream(self, stream):
        self.check(lib().fem_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def close(self):
        if self.h:
            lib().fem_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def torch_allocator(device: int, stream):
    """(alloc, release) callables over torch's caching allocator on `stream`."""
    import torch

    def alloc(n):
        return torch.cuda.caching_allocator_alloc(max(int(n), 1), device, stream)

    def release(p):
        torch.cuda.caching_allocator_delete(p)

    return alloc, release


def form(kind="helmholtz", cell=3, degree=1, dim=1, prec=FEM_FP64, qdegree=0):
    """qdegree 0: exact integration (any degree at least the integrand's is
    the same); a lower positive degree is refused by the library."""
    return fem_form(KINDS.get(kind, kind) if isinstance(kind, str) else kind, cell, degree, dim, prec, qdegree)


class Args:
    """par_loop arguments over torch device tensors (references kept alive)."""

    def __init__(self, cell_vertex, coords, cell_node, nnodes, coeffs=(), nodal=False, cell_coord=None):
        """coeffs: float64 tensors, on the vertex Set (P1 fields read through
        cell_vertex) or, with nodal=True, on the node Set (the nonlinear
        residual's u, kappa, f).  cell_coord: optional int32 [cells][d+1]
        Map to the Set of coords' rows (a per-cell coordinate field for
        FEM_ELASTICITY); without it coords are read through cell_vertex."""
        import torch
        assert cell_vertex.dtype == torch.int32 and cell_node.dtype == torch.int32
        assert coords.dtype == torch.float64
        self.cell_vertex, self.coords, self.cell_node = cell_vertex, coords, cell_node
        self.coeffs = list(coeffs)
        self.nodal = nodal
        self.cells = fem_set(cell_vertex.shape[0])
        self.verts = fem_set(coords.shape[0])
        self.nodes = fem_set(nnodes)
        self.cv = fem_map(C.pointer(self.cells), C.pointer(self.verts), cell_vertex.shape[1], _ptr(cell_vertex))
        self.cn = fem_map(C.pointer(self.cells), C.pointer(self.nodes), cell_node.shape[1], _ptr(cell_node))
        self.cell_coord = cell_coord
        if cell_coord is not None:
            assert cell_coord.dtype == torch.int32
            self.cset = fem_set(coords.shape[0])
            self.cc = fem_map(C.pointer(self.cells), C.pointer(self.cset), cell_coord.shape[1], _ptr(cell_coord))
            self.X = fem_dat(C.pointer(self.cset), coords.shape[1], _ptr(coords))
        else:
            self.X = fem_dat(C.pointer(self.verts), coords.shape[1], _ptr(coords))
        cset = self.nodes if nodal else self.verts
        self.cdats = [fem_dat(C.pointer(cset), 1, _ptr(c)) for c in self.coeffs]
        self.c = fem_args()
        self.c.cells = C.pointer(self.cells)
        self.c.cell_vertex = C.pointer(self.cv)
        self.c.coords = C.pointer(self.X)
        self.c.cell_node = C.pointer(self.cn)
        for i, d in enumerate(self.cdats):
            self.c.coeff[i] = C.pointer(d)
        self.c.ncoeff = len(self.cdats)
        if cell_coord is not None:
            self.c.cell_coord = C.pointer(self.cc)

    def set_versions(self, cell_vertex=None, cell_node=None):
        """Declare that a Map's contents were rewritten in place (its version,
        fem_map.version): plans built at the older version are then refused."""
        if cell_vertex is not None:
            self.cv.version = cell_vertex
        if cell_node is not None:
            self.cn.version = cell_node

    def with_coeffs(self, *coeffs, nodal=False):
        return Args(self.cell_vertex, self.coords, self.cell_node, self.nodes.size, coeffs, nodal,
                    self.cell_coord)


class Sparsity:
    def __init__(self, row_ptr, col_idx, nrows, ncols):
        self.row_ptr, self.col_idx = row_ptr, col_idx
        self.c = fem_sparsity(nrows, ncols, int(col_idx.numel()), _ptr(row_ptr), _ptr(col_idx))


class Plan:
    def __init__(self, h, keep):
        self.h, self._keep = h, keep

    def info(self):
        nb, cv, by = C.c_int64(), C.c_int64(), C.c_int64()
        lib().fem_plan_info(self.h, C.byref(nb), C.byref(cv), C.byref(by))
        return {"blocks": nb.value, "cell_visits": cv.value, "device_bytes": by.value}

    def __del__(self):
        try:
            if self.h:
                lib().fem_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass


def fem_build_sparsity(ctx: Context, rmap, nrows: int, cmap=None, ncols: int | None = None,
                       work=None) -> Sparsity:
    """Two-pass CSR sparsity (count, then fill) of the Mat through rmap/cmap.
    work="torch": query the scratch size and pass a torch buffer of it (the
    library then allocates nothing); None: the library takes its scratch
    from the context's allocator."""
    import torch
    cmap = rmap if cmap is None else cmap
    ncols = nrows if ncols is None else ncols
    cells = fem_set(rmap.shape[0]); rs = fem_set(nrows); cs = fem_set(ncols)
    rm = fem_map(C.pointer(cells), C.pointer(rs), rmap.shape[1], _ptr(rmap))
    cm = fem_map(C.pointer(cells), C.pointer(cs), cmap.shape[1], _ptr(cmap))
    row_ptr = torch.empty(nrows + 1, dtype=torch.int64, device=rmap.device)
    sp = fem_sparsity(0, 0, 0, _ptr(row_ptr), None)
    if work == "torch":
        need = C.c_size_t(0)
        ctx.check(lib().fem_build_sparsity(ctx.h, C.byref(rm), C.byref(cm), C.byref(sp), None, C.byref(need)))
        buf = torch.empty(max(need.value, 1), dtype=torch.uint8, device=rmap.device)
        wp, wb = C.c_void_p(buf.data_ptr()), C.byref(need)
    else:
        buf, wp, wb = None, None, None
    ctx.check(lib().fem_build_sparsity(ctx.h, C.byref(rm), C.byref(cm), C.byref(sp), wp, wb))
    col_idx = torch.empty(max(sp.nnz, 1), dtype=torch.int32, device=rmap.device)
    sp.col_idx = C.c_void_p(col_idx.data_ptr())
    ctx.check(lib().fem_build_sparsity(ctx.h, C.byref(rm), C.byref(cm), C.byref(sp), wp, wb))
    if buf is not None:
        buf.record_stream(ctx.stream)   # in use until the queued fill pass has run
    return Sparsity(row_ptr, col_idx[:sp.nnz], nrows, ncols)


def fem_build_sparsity_noalloc(ctx: Context, rmap, nrows: int, row_ptr, col_idx=None):
    """The allocation-free sparsity build on caller tensors: with col_idx None
    the counting pass (fills row_ptr, returns nnz), else the fill pass into
    col_idx (its first nnz entries).  Scratch comes from the library's static
    array; the library allocates nothing."""
    cells = fem_set(rmap.shape[0]); rs = fem_set(nrows)
    rm = fem_map(C.pointer(cells), C.pointer(rs), rmap.shape[1], _ptr(rmap))
    sp = fem_sparsity(0, 0, 0, _ptr(row_ptr), None)
    if col_idx is not None:
        sp.nrows, sp.ncols = nrows, nrows
        sp.nnz = int(row_ptr[-1].item())
        sp.col_idx = C.c_void_p(col_idx.data_ptr())
    ctx.check(lib().fem_build_sparsity_noalloc(ctx.h, C.byref(rm), C.byref(rm), C.byref(sp)))
    return sp.nnz


def fem_expand_sparsity(ctx: Context, sp: Sparsity, bs: int) -> Sparsity:
    """The bs x bs block expansion of a node CSR (vector DOF bs*node + a)."""
    import torch
    row_ptr = torch.empty(bs * sp.c.nrows + 1, dtype=torch.int64, device=sp.row_ptr.device)
    out = fem_sparsity(0, 0, 0, _ptr(row_ptr), None)
    ctx.check(lib().fem_expand_sparsity(ctx.h, C.byref(sp.c), bs, C.byref(out)))
    col_idx = torch.empty(max(out.nnz, 1), dtype=torch.int32, device=sp.row_ptr.device)
    out.col_idx = C.c_void_p(col_idx.data_ptr())
    ctx.check(lib().fem_expand_sparsity(ctx.h, C.byref(sp.c), bs, C.byref(out)))
    return Sparsity(row_ptr, col_idx[:out.nnz], out.nrows, out.ncols)


def fem_plan_create(ctx: Context, frm: fem_form, args: Args, sp: Sparsity | None = None) -> Plan:
    h = C.c_void_p()
    ctx.check(lib().fem_plan_create(ctx.h, C.byref(frm), C.byref(args.c),
                                    C.byref(sp.c) if sp is not None else None, C.byref(h)))
    return Plan(h, (args, sp, ctx))   # the plan releases its memory through ctx's allocator


def fem_par_loop_assemble_mat(ctx: Context, plan: Plan, frm: fem_form, args: Args, values, sp: Sparsity,
                              acc: int = FEM_WRITE):
    m = fem_mat(C.pointer(sp.c), _ptr(values))
    ctx.check(lib().fem_par_loop_assemble_mat(ctx.h, plan.h, C.byref(frm), C.byref(args.c), C.byref(m), acc))


def fem_par_loop_assemble_vec(ctx: Context, plan: Plan, frm: fem_form, args: Args, b, acc: int = FEM_WRITE):
    d = fem_dat(C.pointer(args.nodes), 1, _ptr(b))
    ctx.check(lib().fem_par_loop_assemble_vec(ctx.h, plan.h, C.byref(frm), C.byref(args.c), C.byref(d), acc))


def fem_apply_action(ctx: Context, plan: Plan, frm: fem_form, args: Args, x, y, acc: int = FEM_WRITE):
    dx = fem_dat(C.pointer(args.nodes), 1, _ptr(x))
    dy = fem_dat(C.pointer(args.nodes), 1, _ptr(y))
    ctx.check(lib().fem_apply_action(ctx.h, plan.h, C.byref(frm), C.byref(args.c), C.byref(dx),
                                     C.byref(dy), acc))


def fem_par_loop_assemble_adjoint(ctx: Context, plan: Plan, frm: fem_form, args: Args, lam, g_u=None,
                                  g_kappa=None, acc: int = FEM_WRITE):
    dl = fem_dat(C.pointer(args.nodes), 1, _ptr(lam))
    du = fem_dat(C.pointer(args.nodes), 1, _ptr(g_u)) if g_u is not None else None
    dk = fem_dat(C.pointer(args.nodes), 1, _ptr(g_kappa)) if g_kappa is not None else None
    ctx.check(lib().fem_par_loop_assemble_adjoint(ctx.h, plan.h, C.byref(frm), C.byref(args.c), C.byref(dl),
                                                  C.byref(du) if du is not None else None,
                                                  C.byref(dk) if dk is not None else None, acc))


def fem_par_loop_reduce(ctx: Context, plan: Plan, frm: fem_form, args: Args, x, g, acc: int = FEM_SUM):
    """g: a one-element float64 device tensor (the Global)."""
    dx = fem_dat(C.pointer(args.nodes), 1, _ptr(x)) if x is not None else None
    gg = fem_global(_ptr(g))
    ctx.check(lib().fem_par_loop_reduce(ctx.h, plan.h, C.byref(frm), C.byref(args.c),
                                        C.byref(dx) if dx is not None else None, C.byref(gg), acc))


def fem_par_loop_assemble_mixed(ctx: Context, plan: Plan, frm: fem_form, args: Args, blocks, values, sp: Sparsity,
                                acc: int = FEM_WRITE):
    """blocks: nf x nf list of (kind name, scale, coefficient tensor or None), or None
    for a zero block; values: nf x nf list of float64 device tensors (None for zero
    blocks).  Every block shares sp and the Mat plan."""
    nf = len(blocks)
    bl = (fem_block * (nf * nf))()
    ms = (fem_mat * (nf * nf))()
    keep = []
    for a in range(nf):
        for b in range(nf):
            q = a * nf + b
            spec, vals = blocks[a][b], values[a][b]
            if spec is None or vals is None:
                ms[q] = fem_mat(C.pointer(sp.c), None)
                continue
            kind, scale, coeff = spec
            d = fem_dat(C.pointer(args.verts), 1, _ptr(coeff)) if coeff is not None else None
            keep.append(d)
            bl[q] = fem_block(KINDS[kind], scale, C.pointer(d) if d is not None else None)
            ms[q] = fem_mat(C.pointer(sp.c), _ptr(vals))
    ctx.check(lib().fem_par_loop_assemble_mixed(ctx.h, plan.h, C.byref(frm), C.byref(args.c), nf, bl, ms, acc))


class Facets:
    """Exterior facet arguments over torch device tensors (references kept)."""

    def __init__(self, facet_vertex, facet_node, coords, g, nnodes):
        self.t = (facet_vertex, facet_node, coords, g)
        self.fset = fem_set(facet_vertex.shape[0])
        self.verts = fem_set(coords.shape[0])
        self.nodes = fem_set(nnodes)
        self.fv = fem_map(C.pointer(self.fset), C.pointer(self.verts), facet_vertex.shape[1], _ptr(facet_vertex))
        self.fn = fem_map(C.pointer(self.fset), C.pointer(self.nodes), facet_node.shape[1], _ptr(facet_node))
        self.X = fem_dat(C.pointer(self.verts), coords.shape[1], _ptr(coords))
        self.g = fem_dat(C.pointer(self.verts), 1, _ptr(g))
        self.c = fem_facets(C.pointer(self.fset), C.pointer(self.fv), C.pointer(self.fn), C.pointer(self.X),
                            C.pointer(self.g))


def fem_facet_plan_create(ctx: Context, frm: fem_form, fa: Facets) -> Plan:
    h = C.c_void_p()
    ctx.check(lib().fem_facet_plan_create(ctx.h, C.byref(frm), C.byref(fa.c), C.byref(h)))
    return Plan(h, (fa, ctx))


def fem_par_loop_assemble_facets(ctx: Context, plan: Plan, frm: fem_form, fa: Facets, b, acc: int = FEM_WRITE):
    d = fem_dat(C.pointer(fa.nodes), 1, _ptr(b))
    ctx.check(lib().fem_par_loop_assemble_facets(ctx.h, plan.h, C.byref(frm), C.byref(fa.c), C.byref(d), acc))


def fem_apply_dirichlet(ctx: Context, sp: Sparsity, values, mask, diag: float = 1.0, b=None, g=None):
    """mask: uint8 device tensor over the rows; b, g: float64 device tensors or None."""
    ctx.check(lib().fem_apply_dirichlet(ctx.h, C.byref(sp.c), _ptr(values), _ptr(mask), diag,
                                        _ptr(b) if b is not None else None, _ptr(g) if g is not None else None))


def fem_renumber(ctx: Context, frm: fem_form, args: Args):
    """(cell_perm, vertex_perm, node_perm) as numpy int32: new -> old."""
    cp = np.empty(args.cells.size, dtype=np.int32)
    vp = np.empty(args.verts.size, dtype=np.int32)
    npm = np.empty(args.nodes.size, dtype=np.int32)
    ctx.check(lib().fem_renumber(ctx.h, C.byref(frm), C.byref(args.c), cp.ctypes.data_as(C.c_void_p),
                                 vp.ctypes.data_as(C.c_void_p), npm.ctypes.data_as(C.c_void_p)))
    return cp, vp, npm


def fem_sync(ctx: Context):
    ctx.check(lib().fem_sync(ctx.h))


class Server:
    """Request server over resident models (fem_server_*): argument
    marshalling only.  Models keep references to their device tensors."""

    def __init__(self, ctx: Context, slots: int = 8, hbm_budget: int = 64 << 30):
        self.ctx = ctx
        self.h = C.c_void_p()
        ctx.check(lib().fem_server_create(ctx.h, slots, hbm_budget, C.byref(self.h)))
        self.keep = []

    def add_model(self, frm: fem_form, args: Args) -> tuple[int, int]:
        mid, res = C.c_int32(), C.c_int64()
        self.ctx.check(lib().fem_server_add_model(self.h, C.byref(frm), C.byref(args.c), C.byref(mid), C.byref(res)))
        self.keep.append(args)
        return mid.value, res.value

    def model_info(self, mid: int):
        c, r, z = C.c_int64(), C.c_int64(), C.c_int64()
        rp, ci = C.c_void_p(), C.c_void_p()
        self.ctx.check(lib().fem_server_model_info(self.h, mid, C.byref(c), C.byref(r), C.byref(z), C.byref(rp),
                                                   C.byref(ci)))
        return {"cells": c.value, "nrows": r.value, "nnz": z.value, "row_ptr": rp.value, "col_idx": ci.value}

    def submit(self, mid: int, op: int, x=None, arrival: float = 0.0) -> int:
        rid = C.c_int64()
        self.ctx.check(lib().fem_server_submit(self.h, mid, op, _ptr(x) if x is not None else None, arrival,
                                               C.byref(rid)))
        return rid.value

    def poll(self, now: float):
        d, r, q = C.c_int32(), C.c_int32(), C.c_int32()
        self.ctx.check(lib().fem_server_poll(self.h, now, C.byref(d), C.byref(r), C.byref(q)))
        return d.value, r.value, q.value

    def result(self, rid: int):
        """(values device pointer or None, vector device pointer, t_admit, t_done)."""
        v, b = C.c_void_p(), C.c_void_p()
        ta, td = C.c_double(), C.c_double()
        self.ctx.check(lib().fem_server_result(self.h, rid, C.byref(v), C.byref(b), C.byref(ta), C.byref(td)))
        return v.value, b.value, ta.value, td.value

    def release(self, rid: int):
        self.ctx.check(lib().fem_server_release(self.h, rid))

    def take_completed(self, cap: int = 256) -> list[int]:
        buf = np.zeros(cap, dtype=np.int64)
        n = C.c_int32()
        self.ctx.check(lib().fem_server_take_completed(self.h, buf.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
        return buf[:n.value].tolist()

    def configure(self, slots: int, share_cus: bool = True):
        self.ctx.check(lib().fem_server_configure(self.h, slots, int(share_cus)))

    def set_batch(self, max_requests: int, max_work: float = 1e8):
        """Requests per batch (1: each request in launches of its own) and the
        estimated work a batch may hold (a larger request runs alone)."""
        self.ctx.check(lib().fem_server_set_batch(self.h, max_requests, max_work))

    def set_order(self, order: int, max_wait: float = 0.0):
        """FEM_SERVE_FIFO or FEM_SERVE_SHORTEST (least estimated work first; a
        queue head that has waited max_wait seconds goes first)."""
        self.ctx.check(lib().fem_server_set_order(self.h, order, max_wait))

    def close(self):
        if self.h:
            lib().fem_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_copy(ptr: int, n: int, dtype=None):
    """Copy n float64 values at a device address into a new torch tensor (for
    reading server outputs); a plain device-to-device copy."""
    import torch
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    if n:
        hip = C.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        rc = hip.hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), 8 * n, 3)
        if rc != 0:
            raise FemError(FEM_E_DEVICE, f"hipMemcpy failed ({rc})")
    return out
