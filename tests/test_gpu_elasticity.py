"""GPU parity of vector P2 linear elasticity (2 mu eps(u):eps(v) + lam div u div v)
on jittered Kuhn cubes with 1% of the cells flattened to aspect ratio ~1e3
(per-cell coordinates): the expanded sparsity bit-exact, FP64 values within
1e-12 of the term-level magnitude per entry, bitwise symmetry and
reproducibility, and the error of the FP32, BF16 and FP16 contractions against
the FP64 oracle, at a small size in full and at 48^3 x 6 on sampled rows."""
import numpy as np
import pytest

import fem_inputs as fi
import oracle

pytestmark = pytest.mark.gpu

# Stated bars for the reduced-precision contractions: relative Frobenius error
# of the assembled values, and (FP32) the row-relative max error, 1e-5 on rows
# whose cells are well shaped (cond(J) <= 100) and max(1e-5, eps32 cond(J)) on
# rows touching the flattened cells, whose inverse Jacobians amplify the
# rounding of the FP32 operands by cond(J).  Measured (small mesh / 48^3
# sampled rows): FP32 Frobenius ~1e-7, well-shaped rows 2.5e-7, flattened
# rows 0.08 eps32 cond(J); FP16 Frobenius 3.4e-4; BF16 3.2e-3 / 2.7e-3 (its blocks
# are stored in bfloat16 as well).
EPS32 = 2.0 ** -23
BARS = {"fp32": (1e-6, 1e-5), "fp16": (3e-3, None), "bf16": (2e-2, None)}


def _problem(n, seed, frac=0.01):
    st = fi.spawn_streams(seed)
    m = fi.jitter_interior(fi.unit_cube(n), 0.2, st["mesh"])
    xdg, chosen = fi.flatten_cells(fi.dg_coordinates(m), frac, st["flatten"])
    cn, N = fi.node_map(m, 2)
    mu = fi.field(st["mu"], m.nverts, 0.5, 2.0)
    lam = fi.field(st["lam"], m.nverts, 0.5, 2.0)
    return dict(cells=m.cells, xdg=xdg, chosen=chosen, cn=np.ascontiguousarray(cn, dtype=np.int32), N=N,
                mu=mu, lam=lam, nverts=m.nverts)


class ElRun:
    def __init__(self, p):
        import torch
        from paper_1501_01809_amd import fem as F
        self.F, self.torch, self.p = F, torch, p
        dev = "cuda"
        C = p["cells"].shape[0]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.cv, self.cn = t(p["cells"]), t(p["cn"])
        self.X = t(p["xdg"].reshape(-1, 3))
        self.cc = t(np.arange(4 * C, dtype=np.int32).reshape(C, 4))
        self.mu, self.lam = t(p["mu"]), t(p["lam"])
        self.ctx = F.Context(0)
        self.args = F.Args(self.cv, self.X, self.cn, p["N"], [self.mu, self.lam], cell_coord=self.cc)
        self.nsp = F.fem_build_sparsity(self.ctx, self.cn, p["N"])
        self.sp = F.fem_expand_sparsity(self.ctx, self.nsp, 3)
        self.plans = {}

    def assemble(self, prec="fp64", out=None, acc=None):
        F = self.F
        frm = F.form("elasticity", 3, 2, 3, F.PRECS[prec])
        if prec not in self.plans:
            self.plans[prec] = F.fem_plan_create(self.ctx, frm, self.args, self.sp)
        vals = out if out is not None else self.torch.empty(int(self.sp.col_idx.numel()),
                                                            dtype=self.torch.float64, device="cuda")
        F.fem_par_loop_assemble_mat(self.ctx, self.plans[prec], frm, self.args, vals, self.sp,
                                    F.FEM_WRITE if acc is None else acc)
        F.fem_sync(self.ctx)
        return vals


def _cond_rows(p, nrows):
    """Per vector row, the largest condition number of the Jacobian of a cell
    containing its node."""
    X = p["xdg"]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], 2)
    kc = np.linalg.cond(J)
    kn = np.zeros(p["N"])
    np.maximum.at(kn, p["cn"].ravel(), np.repeat(kc, p["cn"].shape[1]))
    return np.repeat(kn, 3)[:nrows]


EPS = 2.0 ** -52


def check_rows_fp64(got, ref, absref, ptr, kappa, what):
    """FP64 bar.
    Rows of well-shaped cells (cond(J) <= 100 over the row's cells), per
    entry: |gpu - oracle| <= 1e-12 S_rj + 64 eps max_j S_rj, S the oracle's
    term-level scale.  The second term is the floor of entries whose integrand
    vanishes identically (S_rj = 0 on axis-aligned boundary cells): there the
    oracle sums exact zeros while the contraction over 36 geometry terms, then
    over the cells, leaves rounding of the size of the row's terms (a sum of
    at most 64 such terms per cell group).
    Rows of flattened cells, per row: max |gpu - oracle| <= tol_r max_j S_rj
    with tol_r = max(1e-12, 100 eps cond(J)): an FP64 inverse of a Jacobian of
    condition cond(J) carries a relative error of order eps cond(J) in either
    implementation (measured up to ~32 eps cond(J)).
    Frobenius 1e-12 over the rows of well-shaped cells.  Returns the worst
    error as a fraction of its bar and the worst per-entry error / S_rj over
    the well-shaped entries with S_rj above the floor."""
    worst, worst_entry = 0.0, 0.0
    good = np.zeros(len(got), dtype=bool)
    for r in range(len(ptr) - 1):
        a, b = ptr[r], ptr[r + 1]
        if b == a:
            continue
        diff = np.abs(got[a:b] - ref[a:b])
        smax = np.max(absref[a:b])
        if kappa[r] <= 100:
            bar = 1e-12 * absref[a:b] + 64 * EPS * smax
            e = float(np.max(diff / bar))
            assert e <= 1.0, f"{what}: row {r} entry error {e:.3e} of its bar"
            big = absref[a:b] > 64 * EPS * smax * 1e12
            if big.any():
                worst_entry = max(worst_entry, float(np.max(diff[big] / absref[a:b][big])))
            good[a:b] = True
        else:
            tol = max(1e-12, 100 * EPS * kappa[r])
            e = float(np.max(diff)) / smax / tol
            assert e <= 1.0, f"{what}: row {r} error {e * tol:.3e} of the row scale, bar {tol:.3e}"
        worst = max(worst, e)
    assert np.linalg.norm(got[good] - ref[good]) <= 1e-12 * np.linalg.norm(ref[good]), f"{what}: Frobenius"
    print(f"{what}: worst error {worst:.3f} of its bar; worst per-entry error / S on well-shaped rows "
          f"{worst_entry:.2e}", flush=True)
    return worst


def _errors(got, ref, rows_ptr, kappa):
    """Relative Frobenius error; worst row-relative error (max |diff| over the
    row / max |ref| over the row) on rows whose cells all have cond(J) <= 100,
    and on the other rows the worst of that error divided by cond(J)."""
    frob = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    worst, worst_k = 0.0, 0.0
    for r, (a, b) in enumerate(zip(rows_ptr[:-1], rows_ptr[1:])):
        if b > a:
            e = np.max(np.abs(got[a:b] - ref[a:b])) / np.max(np.abs(ref[a:b]))
            if kappa[r] <= 100:
                worst = max(worst, e)
            else:
                worst_k = max(worst_k, e / kappa[r])
    return frob, worst, worst_k


def _assert_bars(res):
    for prec, (frob, worst, worst_k) in res.items():
        fb, rb = BARS[prec]
        assert frob <= fb, (prec, frob)
        if rb is not None:
            assert worst <= rb, (prec, worst)
            # rows of flattened cells: error <= max(1e-5, eps32 cond(J)), i.e.
            # error / cond(J) <= eps32 once cond(J) >= 1e-5 / eps32 ~ 84
            assert worst_k <= EPS32, (prec, worst_k)


def test_small_mesh_all_precisions():
    p = _problem(4, 2024, frac=0.05)
    assert p["chosen"].size > 0
    run = ElRun(p)
    vm = oracle.vector_map(p["cn"], 3)
    rp, ci = oracle.sparsity(vm, 3 * p["N"])
    assert np.array_equal(run.sp.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(run.sp.col_idx.cpu().numpy(), ci)
    ref, absv = oracle.elasticity_mat(3, 2, p["cells"], p["xdg"], p["cn"], p["mu"], p["lam"], rp, ci)
    v64 = run.assemble("fp64").cpu().numpy()
    R = 3 * p["N"]
    w = check_rows_fp64(v64, ref, absv, rp, _cond_rows(p, R), "elasticity fp64")
    print(f"fp64 small mesh: worst row error / bar {w:.3f}")
    A = np.zeros((R, R))
    for r in range(R):
        A[r, ci[rp[r]:rp[r + 1]]] = v64[rp[r]:rp[r + 1]]
    assert np.array_equal(A, A.T)
    assert np.array_equal(run.assemble("fp64").cpu().numpy().view(np.uint64), v64.view(np.uint64))
    # INC adds the same sums once more: exactly twice the WRITE result
    import torch
    twice = run.assemble("fp64", out=torch.from_numpy(v64.copy()).to("cuda"), acc=run.F.FEM_INC)
    assert np.array_equal(twice.cpu().numpy(), 2 * v64)
    kap = _cond_rows(p, R)
    print(f"cond(J): max {kap.max():.3e} over rows; rows above 100: {(kap > 100).sum()}")
    res = {}
    for prec in BARS:
        v = run.assemble(prec).cpu().numpy()
        assert np.array_equal(run.assemble(prec).cpu().numpy().view(np.uint64), v.view(np.uint64))
        res[prec] = _errors(v, ref, rp, kap)
        print(f"{prec} small mesh: relative Frobenius {res[prec][0]:.3e}, row-relative max {res[prec][1]:.3e} "
              f"(cond <= 100), max row error / cond(J) {res[prec][2]:.3e} (flattened rows)")
    _assert_bars(res)


def test_precision_workload_full_size():
    """48^3 x 6 cells, 6,636 flattened: sampled rows (including every row of
    some flattened cells) against the oracle."""
    p = _problem(48, 1501)
    assert p["cells"].shape[0] == 663552 and p["chosen"].size == 6636
    run = ElRun(p)
    rp = run.sp.row_ptr.cpu().numpy(); ci = run.sp.col_idx.cpu().numpy()
    rng = np.random.default_rng(3)
    flat_nodes = np.unique(p["cn"][p["chosen"][:4]].ravel())
    rows = np.unique(np.concatenate([3 * flat_nodes[:, None] + np.arange(3)]).ravel())
    rows = np.unique(np.concatenate([rows, rng.choice(3 * p["N"], 48, replace=False), [0, 3 * p["N"] - 1]]))
    ref = oracle.elasticity_rows(3, 2, p["cells"], p["xdg"], p["cn"], p["mu"], p["lam"], 3 * p["N"], rows)
    sel = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    for r, (cols, _, _) in zip(rows, ref):
        assert np.array_equal(cols, ci[rp[r]:rp[r + 1]])
    rv = np.concatenate([v for _, v, _ in ref]); ra = np.concatenate([a for _, _, a in ref])
    lens = np.array([len(c) for c, _, _ in ref]); ptr = np.concatenate([[0], np.cumsum(lens)])
    v64 = run.assemble("fp64").cpu().numpy()
    w = check_rows_fp64(v64[sel], rv, ra, ptr, _cond_rows(p, 3 * p["N"])[rows], "elasticity fp64 48^3")
    print(f"fp64 48^3 sampled rows: worst row error / bar {w:.3f}")
    kap = _cond_rows(p, 3 * p["N"])[rows]
    print(f"cond(J): max {kap.max():.3e} over sampled rows; rows above 100: {(kap > 100).sum()}")
    res = {}
    for prec in BARS:
        v = run.assemble(prec).cpu().numpy()[sel]
        res[prec] = _errors(v, rv, ptr, kap)
        print(f"{prec} 48^3 sampled rows: relative Frobenius {res[prec][0]:.3e}, row-relative max "
              f"{res[prec][1]:.3e} (cond <= 100), max row error / cond(J) {res[prec][2]:.3e} (flattened rows)")
    _assert_bars(res)


def test_rejections():
    import torch
    from paper_1501_01809_amd import fem as F
    p = _problem(2, 7, frac=0.0)
    run = ElRun(p)
    with pytest.raises(F.FemError) as e:                       # P1 vector elasticity is not provided
        F.fem_plan_create(run.ctx, F.form("elasticity", 3, 1, 3), run.args, run.sp)
    assert e.value.status == F.FEM_E_UNSUPPORTED
    with pytest.raises(F.FemError) as e:                       # the node CSR is not the vector CSR
        F.fem_plan_create(run.ctx, F.form("elasticity", 3, 2, 3), run.args, run.nsp)
    assert e.value.status == F.FEM_E_ARG
    R = 3 * p["N"]
    ci = run.sp.col_idx.clone()
    ci[1] = ci[0]                                              # right shape, not a 3x3-block expansion
    with pytest.raises(F.FemError) as e:
        F.fem_plan_create(run.ctx, F.form("elasticity", 3, 2, 3), run.args, F.Sparsity(run.sp.row_ptr, ci, R, R))
    assert e.value.status == F.FEM_E_ARG
    half = run.cn[: run.cn.shape[0] // 2].contiguous()          # a vector CSR of half the cells
    hsp = F.fem_expand_sparsity(run.ctx, F.fem_build_sparsity(run.ctx, half, p["N"]), 3)
    with pytest.raises(F.FemError) as e:                       # the sparsity lacks entries the Maps reach
        F.fem_plan_create(run.ctx, F.form("elasticity", 3, 2, 3), run.args, hsp)
    assert e.value.status == F.FEM_E_ARG
    no_cc = F.Args(run.cv, run.X, run.cn, p["N"], [run.mu, run.lam])
    with pytest.raises(F.FemError) as e:                       # coordinates need their own Map
        F.fem_plan_create(run.ctx, F.form("elasticity", 3, 2, 3), no_cc, run.sp)
    assert e.value.status == F.FEM_E_ARG
    plan = F.fem_plan_create(run.ctx, F.form("elasticity", 3, 2, 3, F.FEM_FP32), run.args, run.sp)
    vals = torch.zeros(int(run.sp.col_idx.numel()), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FemError) as e:                       # plan built for another precision
        F.fem_par_loop_assemble_mat(run.ctx, plan, F.form("elasticity", 3, 2, 3, F.FEM_BF16), run.args, vals,
                                    run.sp)
    assert e.value.status == F.FEM_E_ARG
    x = torch.zeros(3 * p["N"], dtype=torch.float64, device="cuda")
    with pytest.raises(F.FemError) as e:
        F.fem_apply_action(run.ctx, plan, F.form("elasticity", 3, 2, 3), run.args, x, x.clone())
    assert e.value.status == F.FEM_E_UNSUPPORTED
    with pytest.raises(F.FemError) as e:                       # the scalar kernels take no coordinate Map
        F.fem_plan_create(run.ctx, F.form("helmholtz", 3, 2), run.args.with_coeffs(run.mu), run.nsp)
    assert e.value.status == F.FEM_E_UNSUPPORTED
