"""The boundary's memory, versioning and quadrature contract, through the C
ABI: device memory from the caller's allocator (counted), caller-provided
sparsity scratch (query, then provide), Map versions that invalidate plans,
the quadrature degree, and the row-length limits of the sparsity build and
of the Mat and Dat plans as status codes."""
import numpy as np
import pytest

import oracle
from fem_case import GpuRun, check_close, make_case

pytestmark = pytest.mark.gpu


class Counting:
    """An allocator over torch's caching allocator that counts its calls."""

    def __init__(self, device, stream):
        from paper_1501_01809_amd import fem as F
        self.a, self.r = F.torch_allocator(device, stream)
        self.live = {}
        self.allocs = self.releases = 0

    def alloc(self, n):
        p = self.a(n)
        self.live[p] = n
        self.allocs += 1
        return p

    def release(self, p):
        assert p in self.live, "release of memory the allocator did not hand out"
        del self.live[p]
        self.releases += 1
        self.r(p)


def test_allocator_callbacks_carry_plan_and_setup_memory():
    import torch
    from paper_1501_01809_amd import fem as F
    c = make_case("cube", 4, 2, shuffle=True)
    ref = GpuRun(c)
    ref.ctx = F.Context(0, torch_memory=False)   # the HIP runtime's memory
    want_mat, want_vec = ref.mat(), ref.vec()

    g = GpuRun(c)
    cnt = Counting(0, g.ctx.stream)
    g.ctx.set_allocator(cnt.alloc, cnt.release)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    sp = g.sparsity()
    assert cnt.allocs > 0 and cnt.releases == cnt.allocs, "sparsity scratch is released before the call returns"
    n0 = cnt.allocs
    mplan, vplan = g.mat_plan(), g.vec_plan()
    held = sum(cnt.live.values())
    assert cnt.allocs > n0 and held >= mplan.info()["device_bytes"] + vplan.info()["device_bytes"]
    assert torch.cuda.memory_allocated() - before >= held   # visible to torch
    got_mat, got_vec = g.mat(), g.vec()
    assert np.array_equal(got_mat, want_mat) and np.array_equal(got_vec, want_vec)
    n1 = cnt.allocs
    g.mat(); g.vec(); g.action()
    assert cnt.allocs == n1, "assembly calls allocate nothing"
    g._mplan = g._vplan = None
    del mplan, vplan
    import gc
    gc.collect()
    assert cnt.releases == cnt.allocs and not cnt.live
    del sp


def test_sparsity_work_buffer_query_then_provide():
    import ctypes as C
    import torch
    from paper_1501_01809_amd import fem as F
    c = make_case("square", 12, 3, shuffle=True)
    g = GpuRun(c)
    rp, ci = oracle.sparsity(c.cell_node, c.nnodes)
    cnt = Counting(0, g.ctx.stream)
    g.ctx.set_allocator(cnt.alloc, cnt.release)
    sp = F.fem_build_sparsity(g.ctx, g.cn, c.nnodes, work="torch")
    assert cnt.allocs == 0, "with a work buffer the call allocates nothing"
    assert np.array_equal(sp.row_ptr.cpu().numpy(), rp) and np.array_equal(sp.col_idx.cpu().numpy(), ci)
    # too small, then misaligned: refused before anything is queued
    cells = F.fem_set(c.cell_node.shape[0]); rows = F.fem_set(c.nnodes)
    m = F.fem_map(C.pointer(cells), C.pointer(rows), c.cell_node.shape[1], F._ptr(g.cn), 0)
    row_ptr = torch.empty(c.nnodes + 1, dtype=torch.int64, device="cuda")
    s = F.fem_sparsity(0, 0, 0, F._ptr(row_ptr), None)
    need = C.c_size_t(0)
    g.ctx.check(F.lib().fem_build_sparsity(g.ctx.h, C.byref(m), C.byref(m), C.byref(s), None, C.byref(need)))
    assert need.value > 0
    buf = torch.empty(need.value + 512, dtype=torch.uint8, device="cuda")
    small = C.c_size_t(need.value - 256)
    assert F.lib().fem_build_sparsity(g.ctx.h, C.byref(m), C.byref(m), C.byref(s), F._ptr(buf),
                                      C.byref(small)) == F.FEM_E_ARG
    odd = C.c_size_t(need.value)
    assert F.lib().fem_build_sparsity(g.ctx.h, C.byref(m), C.byref(m), C.byref(s),
                                      C.c_void_p(buf.data_ptr() + 8), C.byref(odd)) == F.FEM_E_ARG
    F.fem_sync(g.ctx)


def test_map_version_invalidates_plans():
    from paper_1501_01809_amd import fem as F
    c = make_case("square", 8, 2, shuffle=True)
    g = GpuRun(c)
    want = g.mat()
    g.vec_plan()
    # the caller rewrites cell_node in place (here: the same contents) and says so
    g.args_k.set_versions(cell_node=1)
    with pytest.raises(F.FemError) as e:
        g.mat()
    assert e.value.status == F.FEM_E_ARG and "version" in str(e.value)
    with pytest.raises(F.FemError) as e:
        g.action()
    assert e.value.status == F.FEM_E_ARG
    g._mplan = g._vplan = None           # rebuilt at the new version
    assert np.array_equal(g.mat(), want)
    g.args_k.set_versions(cell_vertex=7)
    with pytest.raises(F.FemError):
        g.mat()


def test_quadrature_degree():
    from paper_1501_01809_amd import fem as F
    c = make_case("cube", 3, 2)
    g = GpuRun(c)
    want = g.mat()
    g.form = F.form("helmholtz", 3, 2, qdegree=6)   # above the integrand's degree 4: exact, the same values
    g._mplan = None
    assert np.array_equal(g.mat(), want)
    with pytest.raises(F.FemError) as e:
        F.fem_plan_create(g.ctx, F.form("helmholtz", 3, 2, qdegree=2), g.args_k, None)
    assert e.value.status == F.FEM_E_UNSUPPORTED


def test_long_rows_and_the_distinct_column_limit():
    """Fans of m triangles around one vertex: its row gathers 3m candidate
    columns (with repetition).  Up to 2048 candidates the row is formed in
    LDS; beyond, through the long-row hash set, up to 8192 distinct columns.
    Both match the oracle bit for bit (with ordinary rows around them, and
    several long rows in one 64-row group); a row of 8201 distinct columns
    makes the count pass report FEM_E_UNSUPPORTED instead of a wrong
    pattern."""
    import torch
    from paper_1501_01809_amd import fem as F
    ctx = F.Context(0)

    def fans(sizes):
        tris, off = [], 0
        for m in sizes:
            t = np.arange(m)
            tris.append(np.stack([np.full(m, off), off + 1 + t, off + 1 + (t + 1) % m], 1))
            off += m + 1
        return np.concatenate(tris).astype(np.int32), off

    for sizes in ([600], [700], [3000], [700, 3, 2100, 5, 8191], [40] * 10 + [683, 4000]):
        tri, nv = fans(sizes)
        sp = F.fem_build_sparsity(ctx, torch.from_numpy(tri).cuda(), nv)
        rp, ci = oracle.sparsity(tri, nv)
        assert np.array_equal(sp.row_ptr.cpu().numpy(), rp), sizes
        assert np.array_equal(sp.col_idx.cpu().numpy(), ci), sizes
    tri, nv = fans([8200])
    with pytest.raises(F.FemError) as e:
        F.fem_build_sparsity(ctx, torch.from_numpy(tri).cuda(), nv)
    assert e.value.status == F.FEM_E_UNSUPPORTED and "8192" in str(e.value)


def test_mat_row_longer_than_the_value_area():
    """A caller's CSR may hold more entries than the Maps reach.  A P2
    tetrahedron row whose CSR row is dense (9,261 columns, beyond the 6,392
    values a block's LDS holds) is cut into blocks of consecutive slices of
    its values, each gathering the row's cells; with row 0 dense, and with
    rows 0 and 7 dense around ordinary rows, the matrix matches the oracle,
    the entries the Maps do not reach assemble to zero, and INC adds to the
    values bit for bit as WRITE computes them."""
    import torch
    from paper_1501_01809_amd import fem as F
    c = make_case("cube", 10, 2)
    g = GpuRun(c)
    N = c.nnodes
    rp, ci = oracle.sparsity(c.cell_node, N)
    assert N > 6392

    def with_rows(dense):
        cols = [np.arange(N, dtype=np.int32) if r in dense else ci[rp[r]:rp[r + 1]] for r in range(N)]
        lens = np.array([len(x) for x in cols], dtype=np.int64)
        row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        col = np.concatenate(cols)
        return F.Sparsity(torch.from_numpy(row_ptr).cuda(), torch.from_numpy(col).cuda(), N, N), row_ptr, col

    for dense in ({0}, {0, 7}):
        sp, rp2, ci2 = with_rows(dense)
        plan = F.fem_plan_create(g.ctx, g.form, g.args_k, sp)
        vals = torch.zeros(ci2.size, dtype=torch.float64, device="cuda")
        F.fem_par_loop_assemble_mat(g.ctx, plan, g.form, g.args_k, vals, sp)
        F.fem_sync(g.ctx)
        got = vals.cpu().numpy()
        v, va = oracle.assemble_mat(c.dim, 2, c.cells, c.coords, c.cell_node, c.kappa, rp2, ci2)
        check_close(got, v, va, f"mat with dense rows {sorted(dense)}", row_ptr=rp2)
        for r in dense:
            mesh_cols = set(ci[rp[r]:rp[r + 1]].tolist())
            assert all(got[k] == 0.0 for k in range(rp2[r], rp2[r + 1]) if ci2[k] not in mesh_cols)
        base = torch.from_numpy(np.linspace(-1.0, 1.0, ci2.size)).cuda()
        acc = base.clone()
        F.fem_par_loop_assemble_mat(g.ctx, plan, g.form, g.args_k, acc, sp, F.FEM_INC)
        F.fem_sync(g.ctx)
        assert np.array_equal(acc.cpu().numpy(), (base + vals).cpu().numpy())


def test_dat_row_with_more_cells_than_a_block_holds_is_a_status():
    """A vertex with 4,000 triangles around it: its row's incident cells do
    not fit a Dat block's LDS (3,413 P1 triangles), so plan creation reports
    FEM_E_UNSUPPORTED; 3,000 triangles fit and the source vector matches the
    oracle."""
    import torch
    from paper_1501_01809_amd import fem as F
    ctx = F.Context(0)

    def fan(n):
        t = np.arange(n)
        tri = np.stack([np.zeros(n, dtype=np.int32), 1 + t, 1 + (t + 1) % n], 1).astype(np.int32)
        ang = 2 * np.pi * t / n
        X = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang)], 1)])
        f = np.linspace(-1.0, 1.0, n + 1)
        return tri, np.ascontiguousarray(X), f

    tri, X, f = fan(4000)
    dt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    args = F.Args(dt(tri), dt(X), dt(tri), tri.shape[0] + 1, [dt(f)])
    src = F.form("source", 2, 1)
    with pytest.raises(F.FemError) as e:
        F.fem_plan_create(ctx, src, args, None)
    assert e.value.status == F.FEM_E_UNSUPPORTED and "too long" in str(e.value)
    tri, X, f = fan(3000)
    args = F.Args(dt(tri), dt(X), dt(tri), tri.shape[0] + 1, [dt(f)])
    plan = F.fem_plan_create(ctx, src, args, None)
    b = torch.zeros(tri.shape[0] + 1, dtype=torch.float64, device="cuda")
    F.fem_par_loop_assemble_vec(ctx, plan, src, args, b)
    F.fem_sync(ctx)
    want, wabs = oracle.assemble_vec(2, 1, tri, X, tri, f, tri.shape[0] + 1)
    check_close(b.cpu().numpy(), want, wabs, "vec on a 3000-triangle fan")
