"""Parity at the sizes whose Mat timings are reported beside the benchmark
workload: P1 on the 128^3 x 6 Kuhn cube (12.6 M cells), P1 on the 2048^2 x 2
square (8.4 M cells) and P3 on the 64^3 x 6 cube (345 M nonzeros), each with
the bench's inputs and launch configuration.  nnz against its closed form,
sampled rows against the oracle (Mat, vector, action), and the whole output's
invariants.  At the P1 sizes the Dat blocks hold more cells than the source
vector kernel has lanes (1024), so its cell loop runs more than one pass."""
import pytest

from fullsize import assemble_full, check_sampled_rows, check_whole_output, nnz_closed_form

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

CASES = [("cube", 128, 1), ("square", 2048, 1), ("cube", 64, 3)]


@pytest.mark.parametrize("mesh,n,deg", CASES)
def test_roofline_size_parity(mesh, n, deg):
    full = assemble_full(mesh, n, deg)
    assert full["rp"][-1] == nnz_closed_form(mesh, deg, n)
    vp = full["vplan"]
    if deg == 1:
        assert vp["cell_visits"] / vp["blocks"] > 1024, f"Dat blocks fit one pass: {vp}"
    check_sampled_rows(full)
    check_whole_output(full)
