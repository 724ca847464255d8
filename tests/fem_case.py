"""Shared helpers of the GPU tests: build seeded problems, run the HIP library
through its C ABI binding, run the oracle on the same inputs, compare."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import fem_inputs as fi

TOL = 1e-12   # FP64 bar: per entry vs the abs-sum of contributions, and Frobenius


@dataclass
class Case:
    dim: int
    degree: int
    cells: np.ndarray      # cell -> vertex
    coords: np.ndarray
    cell_node: np.ndarray
    nnodes: int
    kappa: np.ndarray
    f: np.ndarray
    x: np.ndarray


def make_case(kind: str, n: int, degree: int, seed: int = 1501, jitter: float = 0.2,
              shuffle: bool = False, local_perm: bool = False) -> Case:
    st = fi.spawn_streams(seed)
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    if jitter:
        m = fi.jitter_interior(m, jitter, st["mesh"])
    if local_perm:
        rng = np.random.default_rng(seed + 7)
        order = np.argsort(rng.random(m.cells.shape), axis=1)
        m = fi.Mesh(m.dim, m.coords, np.take_along_axis(m.cells, order, 1).astype(np.int32), m.n, m.vlat)
    cn, N = fi.node_map(m, degree)
    cells = m.cells
    coords = m.coords
    if shuffle:
        rng = np.random.default_rng(seed + 3)
        cp = rng.permutation(m.ncells)
        cells, cn = fi.permute_cells(cp, cells, cn)
        vp = rng.permutation(m.nverts)
        inv = np.empty_like(vp); inv[vp] = np.arange(vp.size)
        coords = coords[vp]
        cells = inv[cells].astype(np.int32)
        npn = rng.permutation(N)
        cn = fi.permute_nodes(cn, npn)
    kappa = fi.field(st["kappa"], m.nverts, 0.5, 1.5)
    f = fi.field(st["f"], m.nverts, -1.0, 1.0)
    x = fi.field(st["x"], N, -1.0, 1.0)
    return Case(m.dim, degree, np.ascontiguousarray(cells, dtype=np.int32), coords,
                np.ascontiguousarray(cn, dtype=np.int32), N, kappa, f, x)


EPS = 2.0 ** -52


def row_floor(absref, row_ptr):
    """64 eps times the largest term scale of each entry's row (CSR order)."""
    absref = np.asarray(absref); row_ptr = np.asarray(row_ptr)
    lens = np.diff(row_ptr)
    starts = row_ptr[:-1][lens > 0]
    mx = np.maximum.reduceat(absref, starts) if starts.size else np.zeros(0)
    return 64 * EPS * np.repeat(mx, lens[lens > 0])


def check_close(got, ref, absref, what="", cabs=None, row_ptr=None):
    """FP64 bar: |got - ref| <= TOL * S per entry, S the oracle's term-level
    scale, and the relative Frobenius error <= TOL.  For a matrix (row_ptr
    given) the bar of an entry also has a floor of 64 eps times its row's
    largest S: where a part of the integrand vanishes identically (the
    stiffness on an axis-aligned boundary cell) the oracle sums exact zeros
    while the kernels' metric-form contraction leaves rounding of the row's
    stiffness size.  With cabs (the contribution-level scale, sum over cells
    of |element entry|, which the term-level scale can exceed on
    near-cancelling entries) the worst error is also reported against it, so
    that the strength of the bar is visible; returns both worst ratios."""
    got = np.asarray(got); ref = np.asarray(ref); absref = np.asarray(absref)
    err = np.abs(got - ref)
    floor = row_floor(absref, row_ptr) if row_ptr is not None else 0.0
    bad = err > TOL * absref + floor + 1e-300
    w_term = float((err / np.maximum(absref, 1e-300)).max()) if err.size else 0.0
    assert not bad.any(), f"{what}: {bad.sum()} entries outside {TOL}*S; worst {w_term:.3e}"
    nref = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= TOL * nref + 1e-300, f"{what}: Frobenius error too large"
    w_con = None
    if cabs is not None and err.size:
        cabs = np.asarray(cabs)
        w_con = float((err / np.maximum(cabs, 1e-300)).max())
        print(f"{what}: worst error / term-level S = {w_term:.2e}, / contribution-level S = {w_con:.2e}",
              flush=True)
    return w_term, w_con


class GpuRun:
    """Runs the HIP library on a Case (device tensors kept alive)."""

    def __init__(self, case: Case, form_kind: str = "helmholtz"):
        import torch
        from paper_1501_01809_amd import fem as F
        self.F, self.torch = F, torch
        self.case = case
        dev = "cuda"
        self.cv = torch.from_numpy(case.cells).to(dev)
        self.X = torch.from_numpy(case.coords).to(dev)
        self.cn = torch.from_numpy(case.cell_node).to(dev)
        self.kappa = torch.from_numpy(case.kappa).to(dev)
        self.f = torch.from_numpy(case.f).to(dev)
        self.x = torch.from_numpy(case.x).to(dev)
        self.ctx = F.Context(0)
        self.args_k = F.Args(self.cv, self.X, self.cn, case.nnodes, [self.kappa])
        self.args_f = F.Args(self.cv, self.X, self.cn, case.nnodes, [self.f])
        self.kind = form_kind
        self.form = F.form(form_kind, case.dim, case.degree)
        self.src = F.form("source", case.dim, case.degree)
        self._sp = self._mplan = self._vplan = None

    def sparsity(self):
        if self._sp is None:
            self._sp = self.F.fem_build_sparsity(self.ctx, self.cn, self.case.nnodes)
        return self._sp

    def mat_plan(self):
        if self._mplan is None:
            self._mplan = self.F.fem_plan_create(self.ctx, self.form, self.args_k, self.sparsity())
        return self._mplan

    def vec_plan(self):
        if self._vplan is None:
            self._vplan = self.F.fem_plan_create(self.ctx, self.form, self.args_k, None)
        return self._vplan

    def mat(self, acc=None, init=None):
        sp = self.sparsity()
        vals = self.torch.zeros(max(sp.col_idx.numel(), 1), dtype=self.torch.float64, device="cuda")
        if init is not None:
            vals[: init.size] = self.torch.from_numpy(init).cuda()
        self.F.fem_par_loop_assemble_mat(self.ctx, self.mat_plan(), self.form, self.args_k, vals, sp,
                                         self.F.FEM_WRITE if acc is None else acc)
        self.F.fem_sync(self.ctx)
        return vals[: sp.col_idx.numel()].cpu().numpy()

    def vec(self, acc=None, init=None):
        b = self.torch.zeros(self.case.nnodes, dtype=self.torch.float64, device="cuda")
        if init is not None:
            b.copy_(self.torch.from_numpy(init))
        self.F.fem_par_loop_assemble_vec(self.ctx, self.vec_plan(), self.src, self.args_f, b,
                                         self.F.FEM_WRITE if acc is None else acc)
        self.F.fem_sync(self.ctx)
        return b.cpu().numpy()

    def action(self, acc=None, init=None):
        y = self.torch.zeros(self.case.nnodes, dtype=self.torch.float64, device="cuda")
        if init is not None:
            y.copy_(self.torch.from_numpy(init))
        self.F.fem_apply_action(self.ctx, self.vec_plan(), self.form, self.args_k, self.x, y,
                                self.F.FEM_WRITE if acc is None else acc)
        self.F.fem_sync(self.ctx)
        return y.cpu().numpy()

    def csr(self):
        sp = self.sparsity()
        return sp.row_ptr.cpu().numpy(), sp.col_idx.cpu().numpy()
