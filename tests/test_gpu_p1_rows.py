"""P1 matrices on meshes with long rows and with node Maps that differ from
the vertex Map: fans of 40, 63 and 100 triangles around one vertex (rows of
41 to 101 values, whose cells span several lanes' streams), and shuffled
meshes whose cell-to-node Map is a renumbering of the cell-to-vertex Map,
against the oracle and bitwise run to run."""
import numpy as np
import pytest

import oracle
from fem_case import GpuRun, Case, check_close, make_case

pytestmark = pytest.mark.gpu


def _fan(n, seed=3):
    """A disc of n triangles around vertex 0 (row 0 holds n + 1 values), the
    ring's vertices jittered in radius."""
    rng = np.random.default_rng(seed)
    th = 2 * np.pi * np.arange(n) / n
    rad = 1.0 + 0.1 * rng.uniform(-1, 1, n)
    X = np.concatenate([[[0.0, 0.0]], np.stack([rad * np.cos(th), rad * np.sin(th)], 1)])
    t = np.arange(n)
    cells = np.stack([np.zeros(n, np.int32), 1 + t, 1 + (t + 1) % n], 1).astype(np.int32)
    kappa = rng.uniform(0.5, 1.5, n + 1)
    return Case(2, 1, cells, X, cells.copy(), n + 1, kappa, rng.uniform(-1, 1, n + 1), rng.uniform(-1, 1, n + 1))


@pytest.mark.parametrize("n", [40, 63, 100])
def test_fan_rows_short_and_long(n):
    c = _fan(n)
    g = GpuRun(c)
    rp, ci = oracle.sparsity(c.cell_node, c.nnodes)
    assert rp[1] - rp[0] == n + 1
    v, va = oracle.assemble_mat(2, 1, c.cells, c.coords, c.cell_node, c.kappa, rp, ci)
    check_close(g.mat(), v, va, f"fan of {n}", row_ptr=rp)


@pytest.mark.parametrize("kind,n,shuffle", [("square", 40, True), ("cube", 10, True), ("square", 40, False),
                                            ("cube", 10, False)])
def test_node_and_vertex_maps(kind, n, shuffle):
    c = make_case(kind, n, 1, shuffle=shuffle)
    assert np.array_equal(c.cells, c.cell_node) != shuffle
    g = GpuRun(c)
    rp, ci = oracle.sparsity(c.cell_node, c.nnodes)
    v, va = oracle.assemble_mat(c.dim, 1, c.cells, c.coords, c.cell_node, c.kappa, rp, ci)
    got = g.mat()
    check_close(got, v, va, f"{kind} P1 shuffle={shuffle}", row_ptr=rp)
    np.testing.assert_array_equal(g.mat().view(np.uint64), got.view(np.uint64))
