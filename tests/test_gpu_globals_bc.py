"""GPU Global reductions (SUM / MIN / MAX of cell energies and of integrals
of f) and Dirichlet rows, against the oracle."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle
from fem_case import check_close, make_case

pytestmark = pytest.mark.gpu


def _setup(case, form="helmholtz"):
    import torch
    from paper_1501_01809_amd import fem as F
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    g = dict(cv=t(case.cells), X=t(case.coords), cn=t(case.cell_node), kappa=t(case.kappa), f=t(case.f),
             x=t(case.x))
    ctx = F.Context(0)
    frm = F.form(form, case.dim, case.degree)
    args = F.Args(g["cv"], g["X"], g["cn"], case.nnodes, [g["kappa"]])
    plan = F.fem_plan_create(ctx, frm, args, None)
    return F, torch, ctx, frm, args, plan, g


def _reduce(F, torch, ctx, plan, frm, args, x, acc, init):
    g = torch.full((1,), init, dtype=torch.float64, device="cuda")
    F.fem_par_loop_reduce(ctx, plan, frm, args, x, g, acc)
    F.fem_sync(ctx)
    return float(g.cpu()[0])


# 16^3 x 6 (24,576 cells) spans 24 partials; P3 stays at small sizes for the oracle's sake
@pytest.mark.parametrize("kind,n,degree", [(k, n, d) for k, n in (("square", 9), ("cube", 3)) for d in (1, 2, 3)]
                         + [("cube", 16, 1), ("cube", 16, 2)])
def test_energy_sum_min_max(kind, n, degree):
    case = make_case(kind, n, degree, seed=77, shuffle=True)
    F, torch, ctx, frm, args, plan, g = _setup(case)
    q, qa, s, sa = oracle.cell_values("energy", case.dim, degree, case.cells, case.coords, case.cell_node,
                                      case.kappa, case.x)
    got = _reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_SUM, 0.0)
    assert abs(got - s) <= 1e-12 * sa
    again = _reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_SUM, 0.0)
    assert got == again                                   # fixed combination order
    assert _reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_SUM, 1.5) == 1.5 + got
    lo = _reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_MIN, np.inf)
    hi = _reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_MAX, -np.inf)
    assert abs(lo - q.min()) <= 1e-12 * qa.max() and abs(hi - q.max()) <= 1e-12 * qa.max()
    assert _reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_MIN, -1.0) == -1.0   # g takes part


def test_integral_of_f_and_config1_size():
    case = make_case("square", 64, 1, seed=1501, jitter=0.0)        # the 64x64x2 P1 workload
    F, torch, ctx, frm, args, plan, g = _setup(case)
    src = F.form("source", 2, 1)
    fargs = args.with_coeffs(g["f"])
    gi = torch.zeros(1, dtype=torch.float64, device="cuda")
    F.fem_par_loop_reduce(ctx, plan, src, fargs, None, gi, F.FEM_SUM)
    q, qa, s, sa = oracle.cell_values("integral", 2, 1, case.cells, case.coords, case.cell_node, case.f)
    assert abs(float(gi.cpu()[0]) - s) <= 1e-12 * sa
    q, qa, s, sa = oracle.cell_values("energy", 2, 1, case.cells, case.coords, case.cell_node, case.kappa, case.x)
    assert abs(_reduce(F, torch, ctx, plan, frm, args, g["x"], F.FEM_SUM, 0.0) - s) <= 1e-12 * sa
    with pytest.raises(F.FemError) as e:
        F.fem_par_loop_reduce(ctx, plan, frm, args, g["x"], gi, F.FEM_INC)
    assert e.value.status == F.FEM_E_ARG


def _laplace_system(F, torch, case):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ctx = F.Context(0)
    cv, X, cn = t(case.cells), t(case.coords), t(case.cell_node)
    args = F.Args(cv, X, cn, case.nnodes, [t(np.ones(case.coords.shape[0]))])
    sp = F.fem_build_sparsity(ctx, cn, case.nnodes)
    frm = F.form("laplace", case.dim, case.degree)
    plan = F.fem_plan_create(ctx, frm, args, sp)
    vals = torch.empty(int(sp.col_idx.numel()), dtype=torch.float64, device="cuda")
    F.fem_par_loop_assemble_mat(ctx, plan, frm, args, vals, sp)
    F.fem_sync(ctx)
    return ctx, sp, vals


@pytest.mark.parametrize("kind,n,degree", [("square", 6, 2), ("cube", 2, 3), ("square", 12, 1)])
def test_dirichlet_matches_oracle_and_patch_test(kind, n, degree):
    import torch
    from paper_1501_01809_amd import fem as F
    case = make_case(kind, n, degree, seed=31, shuffle=True)
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    ctx, sp, vals = _laplace_system(F, torch, case)
    rp = sp.row_ptr.cpu().numpy(); ci = sp.col_idx.cpu().numpy(); v0 = vals.cpu().numpy()
    # boundary nodes from the positions of the (shuffled) nodes
    W = fi.local_node_barycentrics(case.dim, degree) / degree
    pos = np.zeros((case.nnodes, case.dim))
    for c in range(case.cells.shape[0]):
        pos[case.cell_node[c]] = W @ case.coords[case.cells[c]]
    mask = np.any((pos <= 1e-12) | (pos >= 1 - 1e-12), axis=1).astype(np.uint8)
    a = np.array([0.75, -0.5, 0.25][:case.dim]); u = pos @ a + 0.125
    gvals = np.where(mask == 1, u, 0.0)
    b0 = np.zeros(case.nnodes)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    vb, bb = vals.clone(), t(b0)
    F.fem_apply_dirichlet(ctx, sp, vb, t(mask), 1.0, bb, t(gvals))
    F.fem_sync(ctx)
    rv, rb, rab = oracle.apply_dirichlet(rp, ci, v0, b0, mask, gvals, 1.0)
    assert np.array_equal(vb.cpu().numpy(), rv)
    assert np.all(np.abs(bb.cpu().numpy() - rb) <= 1e-12 * rab + 1e-300)
    # end to end: oracle assembly then oracle conditions, against the GPU's
    # assembly then the GPU's conditions (the matrix within the assembly bar;
    # the lifted right-hand side within the bar carried through the lifting)
    ov, oa = oracle.assemble_mat(case.dim, degree, case.cells, case.coords, case.cell_node,
                                 np.ones(case.coords.shape[0]), rp, ci, form="laplace")
    ev, eb, eab = oracle.apply_dirichlet(rp, ci, ov, b0, mask, gvals, 1.0)
    oa_bc = np.where(ev == ov, oa, 0.0)                   # kept entries keep their scale; set ones are exact
    check_close(vb.cpu().numpy(), ev, oa_bc, "assembly + Dirichlet, end to end", row_ptr=rp)
    lift = np.zeros(case.nnodes)                          # sum over kept columns of |a_rj g_j| per row
    rows = np.repeat(np.arange(case.nnodes), np.diff(rp))
    np.add.at(lift, rows, np.where(mask[ci] == 1, oa * np.abs(gvals[ci]), 0.0))
    assert np.all(np.abs(bb.cpu().numpy() - eb) <= 1e-12 * (eab + lift) + 1e-300)
    A = np.zeros((case.nnodes, case.nnodes))
    for r in range(case.nnodes):
        A[r, ci[rp[r]:rp[r + 1]]] = rv[rp[r]:rp[r + 1]]
    sol = np.linalg.solve(A, bb.cpu().numpy())            # linear u is reproduced exactly
    assert np.allclose(sol, u, rtol=0, atol=1e-9)
    # homogeneous conditions on A alone
    vh = vals.clone()
    F.fem_apply_dirichlet(ctx, sp, vh, t(mask), 2.0, None, None)
    F.fem_sync(ctx)
    rvh, _, _ = oracle.apply_dirichlet(rp, ci, v0, b0, mask, None, 2.0)
    assert np.array_equal(vh.cpu().numpy(), rvh)
    with pytest.raises(F.FemError) as e:
        F.fem_apply_dirichlet(ctx, sp, vh, t(mask), 1.0, None, t(gvals))
    assert e.value.status == F.FEM_E_ARG


@pytest.mark.parametrize("kind,n", [("square", 7), ("cube", 3)])
@pytest.mark.parametrize("degree", [1, 2, 3])
def test_exterior_facet_integrals(kind, n, degree):
    import torch
    from paper_1501_01809_amd import fem as F
    case = make_case(kind, n, degree, seed=61, shuffle=True)
    m = fi.Mesh(case.dim, case.coords, case.cells)
    fv, fn = fi.exterior_facets(m, case.cell_node, degree)
    g = case.f
    b_ref, ab = oracle.facet_vec(case.dim, degree, fv, case.coords, fn, g, case.nnodes)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ctx = F.Context(0)
    fa = F.Facets(t(fv), t(fn), t(case.coords), t(g), case.nnodes)
    frm = F.form("source", case.dim, degree)
    plan = F.fem_facet_plan_create(ctx, frm, fa)
    b = torch.full((case.nnodes,), 7.0, dtype=torch.float64, device="cuda")
    F.fem_par_loop_assemble_facets(ctx, plan, frm, fa, b)
    F.fem_sync(ctx)
    got = b.cpu().numpy()
    assert np.all(np.abs(got - b_ref) <= 1e-12 * ab + 1e-300)
    F.fem_par_loop_assemble_facets(ctx, plan, frm, fa, b, F.FEM_INC)
    F.fem_sync(ctx)
    assert np.array_equal(b.cpu().numpy(), got + got)       # INC adds the same sums, bitwise
    with pytest.raises(F.FemError) as e:
        F.fem_facet_plan_create(ctx, F.form("helmholtz", case.dim, degree), fa)
    assert e.value.status == F.FEM_E_UNSUPPORTED
