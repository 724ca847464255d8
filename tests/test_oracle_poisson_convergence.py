"""The oracle against an analytic solution: -div grad u = f on the unit
square (and cube, P1), u = 0 on the boundary, u = prod_i sin(pi x_i), f = d
pi^2 u as a P1 field.  The oracle's Laplace Mat, source vector and Dirichlet
rows, solved with scipy, must converge at the rate the method fixes (nodal
error ~ h^2 here, the P1 right-hand side capping P2), and P2 must beat P1.
A wrong sign, a dropped term or a transposed operand in the oracle's element
tensors breaks convergence; this pins them to the mathematics rather than to
the oracle's own formulas."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle


def _solve(dim, n, degree):
    import scipy.sparse as sps
    import scipy.sparse.linalg as spl
    m = fi.unit_square(n) if dim == 2 else fi.unit_cube(n)
    cn, N = fi.node_map(m, degree)
    W = fi.local_node_barycentrics(dim, degree) / degree
    pos = np.zeros((N, dim))
    for l in range(cn.shape[1]):
        pos[cn[:, l]] = np.einsum("cv,cvd->cd", np.repeat(W[l][None], m.ncells, 0), m.coords[m.cells])
    exact = lambda x: np.prod(np.sin(np.pi * x), axis=1)
    f = dim * np.pi ** 2 * exact(m.coords)
    rp, ci = oracle.sparsity(cn, N)
    v, _ = oracle.assemble_mat(dim, degree, m.cells, m.coords, cn, np.ones(m.nverts), rp, ci, form="laplace")
    b, _ = oracle.assemble_vec(dim, degree, m.cells, m.coords, cn, f, N)
    mask = np.any((pos <= 1e-12) | (pos >= 1 - 1e-12), axis=1).astype(np.uint8)
    vv, bb, _ = oracle.apply_dirichlet(rp, ci, v, b, mask, np.zeros(N), 1.0)
    u = spl.spsolve(sps.csr_matrix((vv, ci, rp), shape=(N, N)).tocsc(), bb)
    return float(np.max(np.abs(u - exact(pos))))


@pytest.mark.parametrize("dim,sizes,degrees", [(2, (8, 16, 32), (1, 2)), (3, (8, 16), (1,))])
def test_oracle_poisson_converges(dim, sizes, degrees):
    errs = {k: [_solve(dim, n, k) for n in sizes] for k in degrees}
    for k, e in errs.items():
        rates = [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
        assert all(r > 1.85 for r in rates), (k, e, rates)
    if 2 in errs:
        assert all(p2 < p1 for p1, p2 in zip(errs[1], errs[2]))
