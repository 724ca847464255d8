"""C-ABI checks.  CPU: the library loads and exports every function the header
declares.  GPU: argument, range, support and ownership errors come back as
status codes with a message, and nothing is queued."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fem.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1501_01809_amd import fem as F
    L = F.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
        assert n in F.EXPORTS, n
    # exported with C linkage (unmangled)
    sym = open(F.LIB_PATH, "rb").read()
    for n in names:
        assert n.encode() + b"\x00" in sym, n


def test_oracle_is_not_linked_into_the_library():
    from paper_1501_01809_amd import fem as F
    sym = open(F.LIB_PATH, "rb").read()
    assert b"oracle_" not in sym


@pytest.mark.gpu
def test_status_codes():
    import torch
    from paper_1501_01809_amd import fem as F
    from fem_case import make_case
    c = make_case("square", 3, 2)
    cv = torch.from_numpy(c.cells).cuda(); X = torch.from_numpy(c.coords).cuda()
    cn = torch.from_numpy(c.cell_node).cuda(); k = torch.from_numpy(c.kappa).cuda()
    ctx = F.Context(0)
    args = F.Args(cv, X, cn, c.nnodes, [k])
    frm = F.form("helmholtz", 2, 2)
    # out-of-range map entry -> FEM_E_RANGE
    bad = cn.clone(); bad[1, 2] = c.nnodes + 3
    with pytest.raises(F.FemError) as e:
        F.fem_build_sparsity(ctx, bad, c.nnodes)
    assert e.value.status == F.FEM_E_RANGE
    with pytest.raises(F.FemError) as e:
        F.fem_plan_create(ctx, frm, F.Args(cv, X, bad, c.nnodes, [k]), None)
    assert e.value.status == F.FEM_E_RANGE
    # arity mismatch -> FEM_E_ARG
    with pytest.raises(F.FemError) as e:
        F.fem_plan_create(ctx, F.form("helmholtz", 2, 3), args, None)
    assert e.value.status == F.FEM_E_ARG and "arity" in str(e.value)
    # reduced precision not provided -> FEM_E_UNSUPPORTED
    with pytest.raises(F.FemError) as e:
        F.fem_plan_create(ctx, F.form("helmholtz", 2, 2, prec=F.FEM_BF16), args, None)
    assert e.value.status == F.FEM_E_UNSUPPORTED
    # a Dat plan cannot assemble a Mat
    sp = F.fem_build_sparsity(ctx, cn, c.nnodes)
    vplan = F.fem_plan_create(ctx, frm, args, None)
    vals = torch.zeros(sp.col_idx.numel(), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FemError) as e:
        F.fem_par_loop_assemble_mat(ctx, vplan, frm, args, vals, sp)
    assert e.value.status == F.FEM_E_ARG
    # READ is not an output access
    mplan = F.fem_plan_create(ctx, frm, args, sp)
    with pytest.raises(F.FemError) as e:
        F.fem_par_loop_assemble_mat(ctx, mplan, frm, args, vals, sp, F.FEM_READ)
    assert e.value.status == F.FEM_E_ARG
    # missing kappa for a stiffness form
    with pytest.raises(F.FemError) as e:
        F.fem_par_loop_assemble_mat(ctx, mplan, frm, F.Args(cv, X, cn, c.nnodes, []), vals, sp)
    assert e.value.status == F.FEM_E_ARG
    # a plan built for other Maps is refused
    cn2 = cn.clone()
    with pytest.raises(F.FemError) as e:
        F.fem_par_loop_assemble_mat(ctx, mplan, frm, F.Args(cv, X, cn2, c.nnodes, [k]), vals, sp)
    assert e.value.status == F.FEM_E_ARG
    # a sparsity lacking the pattern is refused at plan creation
    sp2 = F.fem_build_sparsity(ctx, cn[:-1].contiguous(), c.nnodes)
    with pytest.raises(F.FemError):
        F.fem_plan_create(ctx, frm, args, sp2)
    F.fem_sync(ctx)
