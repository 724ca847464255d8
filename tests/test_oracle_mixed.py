"""Pins of the oracle's monolithic mixed-space matrix: each block of the
monolithic matrix equals the scalar assembly of that block's form (a
different code path of the oracle: per-block element matrices scattered
into the scalar CSR), the block structure of the sparsity, and the
Cahn-Hilliard-type system's mass blocks summing to |Omega|."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle


def _dense(rp, ci, v, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, ci[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
    return A


@pytest.mark.parametrize("kind,n,degree", [("square", 4, 1), ("square", 3, 2), ("cube", 2, 1)])
def test_blocks_of_the_monolithic_matrix(kind, n, degree):
    st = fi.spawn_streams(41)
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    m = fi.jitter_interior(m, 0.2, st["mesh"])
    cn, N = fi.node_map(m, degree)
    kap = fi.field(st["kappa"], m.nverts, 0.5, 1.5)
    dt, lam = 0.25, 0.01
    blocks = [[(0.0, 1.0, None), (dt, 0.0, kap)], [(-lam, 0.0, None), (0.0, 1.0, None)]]
    rp, ci, v, a = oracle.mixed_mat(m.dim, degree, m.cells, m.coords, cn, N, blocks)
    M = _dense(rp, ci, v, 2 * N)
    srp, sci = oracle.sparsity(cn, N)
    mass, _ = oracle.assemble_mat(m.dim, degree, m.cells, m.coords, cn, np.ones(m.nverts), srp, sci, form="mass")
    lapk, _ = oracle.assemble_mat(m.dim, degree, m.cells, m.coords, cn, kap, srp, sci, form="laplace")
    lap1, _ = oracle.assemble_mat(m.dim, degree, m.cells, m.coords, cn, np.ones(m.nverts), srp, sci, form="laplace")
    ref = [[_dense(srp, sci, mass, N), dt * _dense(srp, sci, lapk, N)],
           [-lam * _dense(srp, sci, lap1, N), _dense(srp, sci, mass, N)]]
    for i in range(2):
        for j in range(2):
            blk = M[i * N:(i + 1) * N, j * N:(j + 1) * N]
            assert np.allclose(blk, ref[i][j], rtol=0, atol=1e-14 * np.abs(ref[i][j]).max() + 1e-300)
    # every block has the scalar pattern
    for r in range(2 * N):
        cols = ci[rp[r]:rp[r + 1]]
        s = r % N
        scal = sci[srp[s]:srp[s + 1]]
        assert np.array_equal(cols, np.concatenate([scal, scal + N]))
    assert abs(M[:N, :N].sum() - 1.0) <= 1e-12 * np.abs(M[:N, :N]).sum()
