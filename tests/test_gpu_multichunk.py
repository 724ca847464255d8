"""GPU parity of Mat plans whose row blocks hold several chunks of cells.

A Mat block keeps its values in LDS while chunks of its cells pass through
(chunk sizes per dimension and degree below); the kernel pipelines the next
chunk's data behind the current one and the plan balances the lane streams
chunk by chunk.  The small parity cases fit in one chunk per block.  Here the
cells and nodes are numbered at random (a block's rows then share few cells)
and the meshes are sized so that the blocks hold several chunks (checked
from the plan: mean cells per block above one chunk); the whole CSR is
compared with the oracle, entry by entry (1e-12 of the term scale), plus
bitwise run-to-run reproducibility.
"""
import numpy as np
import pytest

import oracle
from fem_case import GpuRun, check_close, make_case

pytestmark = pytest.mark.gpu

# (mesh, n, degree, cells of one chunk)
CASES = [("square", 400, 1, 1024), ("cube", 40, 1, 1024), ("cube", 14, 2, 256),
         ("square", 80, 3, 128), ("cube", 8, 3, 64)]


@pytest.mark.parametrize("kind,n,deg,chunk", CASES)
def test_multichunk_blocks_match_oracle(kind, n, deg, chunk):
    print(f"case {kind} n={n} P{deg}", flush=True)
    c = make_case(kind, n, deg, shuffle=True, local_perm=True)
    g = GpuRun(c)
    got = g.mat()
    info = g.mat_plan().info()
    assert info["cell_visits"] / info["blocks"] > chunk, f"blocks fit one chunk: {info}"
    rp, ci = oracle.sparsity(c.cell_node, c.nnodes)
    grp, gci = g.csr()
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gci, ci)
    v, va = oracle.assemble_mat(c.dim, c.degree, c.cells, c.coords, c.cell_node, c.kappa, rp, ci, "helmholtz")
    check_close(got, v, va, "mat", row_ptr=rp)
    np.testing.assert_array_equal(g.mat(), got)
