"""End-to-end Poisson convergence with the analytic solution (the paper's
Poisson example, "Experiments"): -div grad u = f on the unit square and cube,
u = 0 on the boundary, u = prod_i sin(pi x_i), f = d pi^2 u.  The Laplace Mat
and the source vector are assembled on the GPU, the Dirichlet rows are applied
on the GPU, and the sparse system is solved on the host (scipy).  f enters as
a P1 field (its vertex values), as every coefficient of the library does, so
the right-hand side carries an O(h^2) interpolation error: the nodal error
must fall at least like h^2 for P1 and P2 (P2's own h^3 is capped by that),
and P2 must beat P1 on the same mesh."""
import numpy as np
import pytest

import fem_inputs as fi

pytestmark = pytest.mark.gpu


def _solve(dim, n, degree):
    import scipy.sparse as sps
    import scipy.sparse.linalg as spl
    import torch
    from paper_1501_01809_amd import fem as F
    m = fi.unit_square(n) if dim == 2 else fi.unit_cube(n)
    cn, N = fi.node_map(m, degree)
    W = fi.local_node_barycentrics(dim, degree) / degree
    pos = np.zeros((N, dim))
    for l in range(cn.shape[1]):
        pos[cn[:, l]] = np.einsum("cv,cvd->cd", np.repeat(W[l][None], m.ncells, 0), m.coords[m.cells])
    exact = lambda x: np.prod(np.sin(np.pi * x), axis=1)
    f = dim * np.pi ** 2 * exact(m.coords)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx = F.Context(0)
    cv, X, cnd = t(m.cells.astype(np.int32)), t(m.coords), t(cn.astype(np.int32))
    args = F.Args(cv, X, cnd, N, [t(np.ones(m.nverts))])
    sp = F.fem_build_sparsity(ctx, cnd, N)
    lap = F.form("laplace", dim, degree)
    vals = torch.empty(int(sp.col_idx.numel()), dtype=torch.float64, device="cuda")
    F.fem_par_loop_assemble_mat(ctx, F.fem_plan_create(ctx, lap, args, sp), lap, args, vals, sp)
    src = F.form("source", dim, degree)
    fargs = args.with_coeffs(t(f))
    b = torch.zeros(N, dtype=torch.float64, device="cuda")
    F.fem_par_loop_assemble_vec(ctx, F.fem_plan_create(ctx, src, fargs, None), src, fargs, b)
    mask = np.any((pos <= 1e-12) | (pos >= 1 - 1e-12), axis=1).astype(np.uint8)
    F.fem_apply_dirichlet(ctx, sp, vals, t(mask), 1.0, b, t(np.zeros(N)))
    F.fem_sync(ctx)
    A = sps.csr_matrix((vals.cpu().numpy(), sp.col_idx.cpu().numpy(), sp.row_ptr.cpu().numpy()), shape=(N, N))
    u = spl.spsolve(A.tocsc(), b.cpu().numpy())
    assert np.all(u[mask == 1] == 0.0)
    return float(np.max(np.abs(u - exact(pos))))


# (the coarsest 3D meshes are still pre-asymptotic: 4 -> 8 gives rates 1.80)
@pytest.mark.parametrize("dim,sizes", [(2, (8, 16, 32)), (3, (8, 16))])
def test_poisson_nodal_error_converges(dim, sizes):
    errs = {k: [_solve(dim, n, k) for n in sizes] for k in (1, 2)}
    for k, e in errs.items():
        rates = [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
        print(f"d={dim} P{k}: nodal max errors {['%.3e' % x for x in e]}, rates {['%.2f' % r for r in rates]}")
        assert all(r > 1.85 for r in rates), (k, e, rates)
    assert all(p2 < p1 for p1, p2 in zip(errs[1], errs[2]))
