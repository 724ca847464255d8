"""Full-size parity at the benchmark's workload and launch configuration:
P2 Helmholtz on the 64^3 x 6 jittered Kuhn cube (1,572,864 cells), shuffled
then renumbered exactly as bench.py does.  The oracle computes sampled rows
one by one; properties that hold at any size are checked on the whole output.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from fem_case import check_close

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def full():
    import torch
    sys.path.insert(0, ROOT)
    import bench
    from paper_1501_01809_amd import fem as F
    n, deg = 64, 2
    print("building 64^3 P2 inputs", flush=True)
    d = bench.build_inputs(n, deg, 1501)
    ctx = F.Context(0)
    dev = "cuda"
    up = lambda dd: {k: torch.from_numpy(dd[k]).to(dev) for k in ("cells", "coords", "cn", "kappa", "f", "x")}
    g = up(d)
    form = F.form("helmholtz", 3, deg)
    cp, vp, npn = F.fem_renumber(ctx, form, F.Args(g["cells"], g["coords"], g["cn"], d["N"], [g["kappa"]]))
    for p, size in ((cp, d["cells"].shape[0]), (vp, d["coords"].shape[0]), (npn, d["N"])):
        assert np.array_equal(np.sort(p), np.arange(size)), "renumbering is not a permutation"
    d = bench.apply_perms(d, cp, vp, npn)
    g = up(d)
    args_k = F.Args(g["cells"], g["coords"], g["cn"], d["N"], [g["kappa"]])
    args_f = F.Args(g["cells"], g["coords"], g["cn"], d["N"], [g["f"]])
    print("sparsity + plans", flush=True)
    sp = F.fem_build_sparsity(ctx, g["cn"], d["N"])
    mplan = F.fem_plan_create(ctx, form, args_k, sp)
    vplan = F.fem_plan_create(ctx, form, args_k, None)
    vals = torch.empty(sp.col_idx.numel(), dtype=torch.float64, device=dev)
    b = torch.empty(d["N"], dtype=torch.float64, device=dev)
    y = torch.empty(d["N"], dtype=torch.float64, device=dev)
    F.fem_par_loop_assemble_mat(ctx, mplan, form, args_k, vals, sp)
    F.fem_par_loop_assemble_vec(ctx, vplan, F.form("source", 3, deg), args_f, b)
    F.fem_apply_action(ctx, vplan, form, args_k, g["x"], y)
    ones = torch.ones(d["N"], dtype=torch.float64, device=dev)
    y1 = torch.empty_like(y)
    F.fem_apply_action(ctx, vplan, form, args_k, ones, y1)
    vals2 = torch.empty_like(vals)
    F.fem_par_loop_assemble_mat(ctx, mplan, form, args_k, vals2, sp)
    F.fem_sync(ctx)
    print("assembled", flush=True)
    return dict(d=d, n=n, deg=deg, rp=sp.row_ptr.cpu().numpy(), ci=sp.col_idx.cpu().numpy(),
                vals=vals.cpu().numpy(), vals2=vals2.cpu().numpy(), b=b.cpu().numpy(),
                y=y.cpu().numpy(), y1=y1.cpu().numpy())


def test_nnz_closed_form(full):
    n = full["n"]
    assert full["rp"][-1] == 230 * n ** 3 + 138 * n * n + 24 * n + 1


def test_sampled_rows_match_oracle(full):
    d, rp, ci, vals = full["d"], full["rp"], full["ci"], full["vals"]
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([rng.choice(d["N"], 48, replace=False), [0, d["N"] - 1]]))
    ref = oracle.mat_rows(3, full["deg"], d["cells"], d["coords"], d["cn"], d["kappa"], d["N"], rows)
    for r, (cols, v, a) in zip(rows, ref):
        np.testing.assert_array_equal(ci[rp[r]:rp[r + 1]], cols)
        check_close(vals[rp[r]:rp[r + 1]], v, a, f"row {r}")
    bs, ba = oracle.vec_rows(3, full["deg"], d["cells"], d["coords"], d["cn"], d["f"], d["N"], rows)
    check_close(full["b"][rows], bs, ba, "vec")
    ys, ya = oracle.action_rows(3, full["deg"], d["cells"], d["coords"], d["cn"], d["kappa"], d["x"],
                                d["N"], rows)
    check_close(full["y"][rows], ys, ya, "action")


def test_whole_output_properties(full):
    vals, rp, ci = full["vals"], full["rp"], full["ci"]
    # bitwise reproducible run to run
    assert np.array_equal(vals.view(np.uint64), full["vals2"].view(np.uint64))
    # sum of the Helmholtz matrix = |Omega| (stiffness rows sum to zero)
    assert abs(vals.sum() - 1.0) < 1e-9
    # A 1 = M 1 >= 0 and sums to |Omega|
    assert abs(full["y1"].sum() - 1.0) < 1e-11
    # bitwise symmetry on sampled rows
    rng = np.random.default_rng(5)
    for r in rng.choice(rp.size - 1, 64, replace=False):
        for k in range(rp[r], rp[r + 1]):
            c = ci[k]
            kk = rp[c] + np.searchsorted(ci[rp[c]:rp[c + 1]], r)
            assert ci[kk] == r and vals[kk] == vals[k]
