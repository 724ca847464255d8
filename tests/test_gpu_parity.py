"""GPU parity of the HIP library against the CPU oracle (through the C ABI).

Sparsity and Maps bit-exact; values within 1e-12 of the oracle per entry
(relative to the sum of |contributions|) and in Frobenius norm; bitwise
run-to-run reproducibility; INC = initial + WRITE bitwise.
"""
import numpy as np
import pytest

import oracle
from fem_case import GpuRun, check_close, make_case

pytestmark = pytest.mark.gpu

SMALL = [("square", 5, 1), ("square", 4, 2), ("square", 3, 3),
         ("cube", 3, 1), ("cube", 2, 2), ("cube", 2, 3)]


def _oracle_all(c, kind="helmholtz"):
    rp, ci = oracle.sparsity(c.cell_node, c.nnodes)
    v, va = oracle.assemble_mat(c.dim, c.degree, c.cells, c.coords, c.cell_node, c.kappa, rp, ci, kind)
    b, ba = oracle.assemble_vec(c.dim, c.degree, c.cells, c.coords, c.cell_node, c.f, c.nnodes)
    y, ya = oracle.apply_action(c.dim, c.degree, c.cells, c.coords, c.cell_node, c.kappa, c.x,
                                c.nnodes, kind)
    return rp, ci, v, va, b, ba, y, ya


@pytest.mark.parametrize("kind,n,deg", SMALL)
@pytest.mark.parametrize("layout", ["lattice", "shuffled"])
def test_small_meshes_all_ops(kind, n, deg, layout):
    c = make_case(kind, n, deg, shuffle=layout == "shuffled", local_perm=layout == "shuffled")
    print(f"case {kind} n={n} P{deg} {layout}", flush=True)
    g = GpuRun(c)
    rp, ci, v, va, b, ba, y, ya = _oracle_all(c)
    grp, gci = g.csr()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gci, ci)
    check_close(g.mat(), v, va, "mat", row_ptr=rp)
    check_close(g.vec(), b, ba, "vec")
    check_close(g.action(), y, ya, "action")


@pytest.mark.parametrize("form", ["mass", "laplace"])
@pytest.mark.parametrize("kind,n,deg", [("square", 4, 2), ("cube", 2, 2)])
def test_other_forms(kind, n, deg, form):
    c = make_case(kind, n, deg)
    g = GpuRun(c, form)
    rp, ci, v, va, _, _, y, ya = _oracle_all(c, form)
    check_close(g.mat(), v, va, form, row_ptr=rp)
    check_close(g.action(), y, ya, form + " action")


def test_config1_square_p1():
    """64x64x2 triangles, P1 Helmholtz, kappa U[0.5,1.5], f U[-1,1] (no jitter)."""
    c = make_case("square", 64, 1, jitter=0.0)
    g = GpuRun(c)
    rp, ci, v, va, b, ba, y, ya = _oracle_all(c)
    grp, gci = g.csr()
    assert rp[-1] == 7 * 64 * 64 + 6 * 64 + 1
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gci, ci)
    check_close(g.mat(), v, va, "mat", row_ptr=rp)
    check_close(g.vec(), b, ba, "vec")
    check_close(g.action(), y, ya, "action")


@pytest.mark.parametrize("kind,n,deg", [("square", 6, 2), ("cube", 3, 2)])
def test_determinism_and_inc(kind, n, deg):
    c = make_case(kind, n, deg, shuffle=True)
    g = GpuRun(c)
    m1, m2 = g.mat(), g.mat()
    assert np.array_equal(m1.view(np.uint64), m2.view(np.uint64))
    b1, b2 = g.vec(), g.vec()
    assert np.array_equal(b1.view(np.uint64), b2.view(np.uint64))
    y1, y2 = g.action(), g.action()
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    rng = np.random.default_rng(0)
    init = rng.uniform(-1, 1, m1.size)
    mi = g.mat(acc=g.F.FEM_INC, init=init)
    assert np.array_equal(mi, init + m1)
    vi = rng.uniform(-1, 1, b1.size)
    assert np.array_equal(g.vec(acc=g.F.FEM_INC, init=vi), vi + b1)
    assert np.array_equal(g.action(acc=g.F.FEM_INC, init=vi), vi + y1)


def test_two_cell_meshes():
    import fem_inputs as fi
    for m in (fi.two_triangles(), fi.two_tets()):
        for deg in (1, 2, 3):
            cn, N = fi.node_map(m, deg)
            from fem_case import Case
            rng = np.random.default_rng(deg)
            c = Case(m.dim, deg, m.cells, m.coords, cn, N, rng.uniform(0.5, 1.5, m.nverts),
                     rng.uniform(-1, 1, m.nverts), rng.uniform(-1, 1, N))
            g = GpuRun(c)
            rp, ci, v, va, b, ba, y, ya = _oracle_all(c)
            grp, gci = g.csr()
            np.testing.assert_array_equal(gci, ci)
            check_close(g.mat(), v, va, "mat", row_ptr=rp)
            check_close(g.vec(), b, ba, "vec")
            check_close(g.action(), y, ya, "action")


def test_isolated_nodes_and_empty_rows():
    """Nodes no cell reaches give empty rows, zero vector entries."""
    import fem_inputs as fi
    from fem_case import Case
    m = fi.unit_square(3)
    cn, N = fi.node_map(m, 2)
    N2 = N + 5
    rng = np.random.default_rng(3)
    c = Case(2, 2, m.cells, m.coords, cn, N2, rng.uniform(0.5, 1.5, m.nverts),
             rng.uniform(-1, 1, m.nverts), rng.uniform(-1, 1, N2))
    g = GpuRun(c)
    rp, ci, v, va, b, ba, y, ya = _oracle_all(c)
    grp, gci = g.csr()
    np.testing.assert_array_equal(grp, rp)
    assert rp[-1] == rp[N]
    check_close(g.mat(), v, va, "mat", row_ptr=rp)
    bb = g.vec()
    check_close(bb, b, ba, "vec")
    assert np.all(bb[N:] == 0)
