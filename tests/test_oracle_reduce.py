"""Pins of the oracle's per-cell Global contributions (energies
x_K^T A_K x_K of the Helmholtz form, integrals of f), used by the SUM, MIN and
MAX reductions: closed forms for linear fields, not the oracle's quadrature."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle


def _mesh(kind, n, jitter, seed):
    st = fi.spawn_streams(seed)
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    if jitter:
        m = fi.jitter_interior(m, jitter, st["mesh"])
    return m, st


def _volumes(m):
    X = m.coords[m.cells]
    J = np.stack([X[:, i + 1] - X[:, 0] for i in range(m.dim)], 2)
    return np.abs(np.linalg.det(J)) / (2 if m.dim == 2 else 6)


@pytest.mark.parametrize("kind,n", [("square", 6), ("cube", 3)])
@pytest.mark.parametrize("degree", [1, 2, 3])
def test_constant_field_energy_is_the_measure(kind, n, degree):
    m, st = _mesh(kind, n, 0.2, 3)
    cn, N = fi.node_map(m, degree)
    kappa = fi.field(st["kappa"], m.nverts, 0.5, 1.5)
    q, qa, s, sa = oracle.cell_values("energy", m.dim, degree, m.cells, m.coords, cn, kappa, np.ones(N))
    assert abs(s - 1.0) <= 1e-12 * sa                     # grad 1 = 0, integral of 1 = |Omega|
    assert np.allclose(q, _volumes(m), rtol=0, atol=1e-12 * qa.max())


@pytest.mark.parametrize("kind,n", [("square", 5), ("cube", 3)])
@pytest.mark.parametrize("degree", [1, 2, 3])
def test_linear_field_cell_energies(kind, n, degree):
    """u = a.x + c: q_K = |a|^2 |K| mean(kappa_K) + |K| (sum u_i^2 + (sum u_i)^2) / ((d+1)(d+2))."""
    m, st = _mesh(kind, n, 0.0, 4)
    d = m.dim
    cn, N = fi.node_map(m, degree)
    kappa = fi.field(st["kappa"], m.nverts, 0.5, 1.5)
    a = np.array([0.75, -0.5, 0.25][:d]); c = 0.125
    W = fi.local_node_barycentrics(d, degree) / degree
    pos = np.zeros((N, d))
    for e in range(m.ncells):
        pos[cn[e]] = W @ m.coords[m.cells[e]]
    u = pos @ a + c
    q, qa, s, sa = oracle.cell_values("energy", d, degree, m.cells, m.coords, cn, kappa, u)
    vol = _volumes(m)
    uv = m.coords[m.cells] @ a + c                         # u at the vertices of every cell
    ref = a @ a * vol * kappa[m.cells].mean(1) + vol * ((uv ** 2).sum(1) + uv.sum(1) ** 2) / ((d + 1) * (d + 2))
    assert np.all(np.abs(q - ref) <= 1e-12 * qa)
    assert q.min() == pytest.approx(ref.min(), rel=1e-12) and q.max() == pytest.approx(ref.max(), rel=1e-12)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_integral_of_a_linear_field(degree):
    m, st = _mesh("square", 6, 0.2, 5)
    cn, N = fi.node_map(m, degree)
    f = 0.5 * m.coords[:, 0] - 0.25 * m.coords[:, 1] + 1.0
    q, qa, s, sa = oracle.cell_values("integral", 2, degree, m.cells, m.coords, cn, f)
    assert abs(s - (0.25 - 0.125 + 1.0)) <= 1e-12 * sa      # integral over the unit square
    assert np.all(np.abs(q - _volumes(m) * f[m.cells].mean(1)) <= 1e-12 * qa)
