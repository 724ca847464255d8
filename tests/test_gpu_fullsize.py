"""Full-size parity at the benchmark's workload and launch configuration:
P2 Helmholtz on the 64^3 x 6 jittered Kuhn cube (1,572,864 cells), shuffled
then renumbered exactly as bench.py does.  The whole CSR pattern is compared
with the oracle's bit by bit; the oracle computes sampled rows of the values
one by one; properties that hold at any size are checked on the whole output.
"""
import numpy as np
import pytest

import oracle
from fullsize import assemble_full, check_sampled_rows, check_whole_output, nnz_closed_form

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


@pytest.fixture(scope="module")
def full():
    return assemble_full("cube", 64, 2)


def test_whole_csr_matches_oracle(full):
    d = full["d"]
    assert full["rp"][-1] == nnz_closed_form("cube", 2, full["n"])
    rp, ci = oracle.sparsity(d["cn"], d["N"])
    np.testing.assert_array_equal(full["rp"], rp)
    np.testing.assert_array_equal(full["ci"], ci)


def test_sampled_rows_match_oracle(full):
    check_sampled_rows(full)


def test_whole_output_properties(full):
    check_whole_output(full)
