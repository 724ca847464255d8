"""Pins of the oracle's exterior facet integrals b_i = sum_F integral_F g v_i ds:
facet counts, Simpson-type closed forms for g = 1, and the boundary
integral of a linear g (partition of unity) against its exact value."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle


@pytest.mark.parametrize("kind,n", [("square", 4), ("cube", 3)])
@pytest.mark.parametrize("degree", [1, 2, 3])
def test_boundary_integral_of_linear_g(kind, n, degree):
    st = fi.spawn_streams(8)
    m = fi.jitter_interior(fi.unit_square(n) if kind == "square" else fi.unit_cube(n), 0.2, st["mesh"])
    cn, N = fi.node_map(m, degree)
    fv, fn = fi.exterior_facets(m, cn, degree)
    assert fv.shape[0] == (4 * n if kind == "square" else 12 * n * n)
    a = np.array([0.75, -0.5, 0.25][:m.dim]); c = 0.125
    g = m.coords @ a + c
    b, ab = oracle.facet_vec(m.dim, degree, fv, m.coords, fn, g, N)
    exact = 2 * a.sum() + 4 * c if m.dim == 2 else 3 * a.sum() + 6 * c
    assert abs(b.sum() - exact) <= 1e-12 * ab.sum()


@pytest.mark.parametrize("degree,vertex,edge", [(1, 1.0, None), (2, 1.0 / 3, 2.0 / 3)])
def test_unit_g_on_the_square_boundary(degree, vertex, edge):
    """g = 1: a boundary vertex collects h (P1) or h/3 (P2, Simpson), an edge
    midpoint 2h/3; interior nodes nothing."""
    n = 5
    h = 1.0 / n
    m = fi.unit_square(n)
    cn, N = fi.node_map(m, degree)
    fv, fn = fi.exterior_facets(m, cn, degree)
    b, _ = oracle.facet_vec(2, degree, fv, m.coords, fn, np.ones(m.nverts), N)
    W = fi.local_node_barycentrics(2, degree) / degree
    pos = np.zeros((N, 2))
    for e in range(m.ncells):
        pos[cn[e]] = W @ m.coords[m.cells[e]]
    on = np.any((pos <= 1e-12) | (pos >= 1 - 1e-12), axis=1)
    grid = np.abs(pos * n - np.round(pos * n)).max(1) <= 1e-9
    assert np.all(np.abs(b[~on]) == 0.0)
    assert np.allclose(b[on & grid], vertex * h, rtol=1e-13)
    if edge is not None:
        assert np.allclose(b[on & ~grid], edge * h, rtol=1e-13)
