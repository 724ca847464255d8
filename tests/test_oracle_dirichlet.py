"""Pins of the oracle's Dirichlet application: the patch test (a Laplace
problem whose exact solution is linear is solved exactly by P_k once the
boundary values are imposed and lifted), symmetry, and the boundary mask."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle


def _dense(rp, ci, v, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, ci[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
    return A


@pytest.mark.parametrize("kind,n", [("square", 4), ("cube", 2)])
@pytest.mark.parametrize("degree", [1, 2, 3])
def test_patch_test_with_lifted_boundary_values(kind, n, degree):
    st = fi.spawn_streams(21)
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    m = fi.jitter_interior(m, 0.2, st["mesh"])
    cn, N = fi.node_map(m, degree)
    kappa = np.ones(m.nverts)
    rp, ci = oracle.sparsity(cn, N)
    vals, _ = oracle.assemble_mat(m.dim, degree, m.cells, m.coords, cn, kappa, rp, ci, form="laplace")
    W = fi.local_node_barycentrics(m.dim, degree) / degree
    pos = np.zeros((N, m.dim))
    for c in range(m.ncells):
        pos[cn[c]] = W @ m.coords[m.cells[c]]
    a = np.array([0.75, -0.5, 0.25][:m.dim])
    u = pos @ a + 0.125                                   # harmonic: -div grad u = 0
    mask = fi.boundary_nodes(m, cn, degree)
    assert mask.sum() > 0 and mask.sum() < N
    g = np.where(mask == 1, u, 0.0)
    v2, b2, _ = oracle.apply_dirichlet(rp, ci, vals, np.zeros(N), mask, g, diag=1.0)
    A2 = _dense(rp, ci, v2, N)
    assert np.array_equal(A2, A2.T)
    sol = np.linalg.solve(A2, b2)
    assert np.allclose(sol, u, rtol=0, atol=1e-10)


def test_boundary_mask_counts():
    m = fi.unit_square(5)
    for k, expect in ((1, 4 * 5), (2, 4 * 10), (3, 4 * 15)):
        cn, N = fi.node_map(m, k)
        assert fi.boundary_nodes(m, cn, k).sum() == expect
    m = fi.unit_cube(3)
    cn, N = fi.node_map(m, 1)
    assert fi.boundary_nodes(m, cn, 1).sum() == 4 ** 3 - 2 ** 3
