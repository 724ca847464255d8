"""Request server: resident models, admission by slots and HBM budget,
requests batched into shared persistent launches, overlapping batches; every
result bitwise the same alone, in a batch, and as the single-request entry
points compute it, and equal to the oracle on small meshes."""
import time

import numpy as np
import pytest

import fem_inputs as fi
import oracle
from fem_case import check_close

pytestmark = pytest.mark.gpu


def _model(kind, n, degree, seed):
    st = fi.spawn_streams(seed)
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    m = fi.jitter_interior(m, 0.2, st["mesh"])
    cn, N = fi.node_map(m, degree)
    kappa = fi.field(st["kappa"], m.nverts, 0.5, 1.5)
    f = fi.field(st["f"], m.nverts, 0.5, 1.5)
    x = fi.field(st["x"], N, 0.5, 1.5)
    return dict(dim=m.dim, degree=degree, cells=m.cells, coords=m.coords, cn=np.ascontiguousarray(cn, np.int32),
                N=N, kappa=kappa, f=f, x=x)


SPECS = [("square", 16, 1), ("square", 16, 2), ("square", 8, 3), ("cube", 3, 1), ("cube", 3, 2), ("cube", 2, 3)]


def _server(slots, budget, specs=SPECS):
    import torch
    from paper_1501_01809_amd import fem as F
    ctx = F.Context(0)
    srv = F.Server(ctx, slots, budget)
    models = []
    for i, (kind, n, k) in enumerate(specs):
        p = _model(kind, n, k, 900 + i)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
        p["g"] = dict(cv=t(p["cells"]), X=t(p["coords"]), cn=t(p["cn"]), kappa=t(p["kappa"]), f=t(p["f"]),
                      x=t(p["x"]))
        g = p["g"]
        args = F.Args(g["cv"], g["X"], g["cn"], p["N"], [g["kappa"], g["f"]])
        mid, res = srv.add_model(F.form("helmholtz", p["dim"], k), args)
        p["id"], p["resident"] = mid, res
        p["info"] = srv.model_info(mid)
        models.append(p)
    return F, ctx, srv, models


def _drain(srv, F, rids, models, ops, release=True):
    """Poll until every request is done; return its outputs as numpy arrays."""
    out = {}
    pending = set(rids)
    t0 = time.perf_counter()
    while pending:
        srv.poll(time.perf_counter() - t0)
        for r in list(pending):
            try:
                v, b, ta, td = srv.result(r)
            except F.FemError:
                continue
            m, op = models[r], ops[r]
            vec = F.device_copy(b, m["N"]).cpu().numpy()
            vals = F.device_copy(v, m["info"]["nnz"]).cpu().numpy() if op == F.FEM_REQ_ASSEMBLE else None
            out[r] = (vals, vec, ta, td)
            if release:
                srv.release(r)
            pending.discard(r)
        assert time.perf_counter() - t0 < 60, "requests did not complete"
    return out


def _workload(F, models, reps=3):
    seq = []
    for rep in range(reps):
        for p in models:
            seq.append((p, F.FEM_REQ_ASSEMBLE))
            seq.append((p, F.FEM_REQ_ACTION))
    return seq


def _direct(F, p):
    """The model's assembly and action through the single-request entry points."""
    import torch
    g = p["g"]
    ctx = F.Context(0)
    args = F.Args(g["cv"], g["X"], g["cn"], p["N"], [g["kappa"]])
    args_f = F.Args(g["cv"], g["X"], g["cn"], p["N"], [g["f"]])
    frm = F.form("helmholtz", p["dim"], p["degree"])
    sp = F.fem_build_sparsity(ctx, g["cn"], p["N"])
    mplan, vplan = F.fem_plan_create(ctx, frm, args, sp), F.fem_plan_create(ctx, frm, args, None)
    vals = torch.empty(max(sp.col_idx.numel(), 1), dtype=torch.float64, device="cuda")
    b = torch.empty(p["N"], dtype=torch.float64, device="cuda")
    y = torch.empty_like(b)
    F.fem_par_loop_assemble_mat(ctx, mplan, frm, args, vals, sp)
    F.fem_par_loop_assemble_vec(ctx, vplan, F.form("source", p["dim"], p["degree"]), args_f, b)
    F.fem_apply_action(ctx, vplan, frm, args, g["x"], y)
    F.fem_sync(ctx)
    return vals[:sp.col_idx.numel()].cpu().numpy(), b.cpu().numpy(), y.cpu().numpy()


def test_alone_equals_mix_and_oracle():
    F, ctx, srv1, models = _server(1, 8 << 30)
    srv1.set_batch(1)                                     # every request in launches of its own
    seq = _workload(F, models)
    alone = []
    for p, op in seq:                                     # one at a time, one slot
        rid = srv1.submit(p["id"], op, p["g"]["x"] if op == F.FEM_REQ_ACTION else None)
        res = _drain(srv1, F, [rid], {rid: p}, {rid: op})
        alone.append(res[rid])
    # the same requests, all submitted at once to a server with 8 slots and
    # batches of up to 8 requests: mixed meshes, degrees and operations share
    # launches, and batches overlap
    F2, ctx2, srv8, models8 = _server(8, 8 << 30)
    srv8.set_batch(8, 1e12)                               # no work bound: the whole mix in 8-request batches
    rids, mm, oo = [], {}, {}
    for p, op in seq:
        q = models8[p["id"]]
        r = srv8.submit(q["id"], op, q["g"]["x"] if op == F.FEM_REQ_ACTION else None)
        rids.append(r); mm[r] = q; oo[r] = op
    _, running, queued = srv8.poll(0.0)
    assert running == len(seq) and queued == 0, "one poll admits every request in batches"
    mix = _drain(srv8, F2, rids, mm, oo)
    for (p, op), a, r in zip(seq, alone, rids):
        b = mix[r]
        assert np.array_equal(a[1].view(np.uint64), b[1].view(np.uint64))
        if op == F.FEM_REQ_ASSEMBLE:
            assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64))
    # and as the single-request entry points compute them
    for k, p in enumerate(models):
        vals, b, y = _direct(F, p)
        i = 2 * k                                         # the first repetition: assembly, then action
        assert seq[i][0] is p and seq[i][1] == F.FEM_REQ_ASSEMBLE
        assert np.array_equal(alone[i][0].view(np.uint64), vals.view(np.uint64))
        assert np.array_equal(alone[i][1].view(np.uint64), b.view(np.uint64))
        assert np.array_equal(alone[i + 1][1].view(np.uint64), y.view(np.uint64))
    # every result against the oracle (first repetition)
    for (p, op), a in zip(seq[:2 * len(models)], alone):
        if op == F.FEM_REQ_ASSEMBLE:
            rp, ci = oracle.sparsity(p["cn"], p["N"])
            ref, absv = oracle.assemble_mat(p["dim"], p["degree"], p["cells"], p["coords"], p["cn"], p["kappa"], rp, ci)
            check_close(a[0], ref, absv, f"server mat {p['dim']}D P{p['degree']}", row_ptr=rp)
            b, ab = oracle.assemble_vec(p["dim"], p["degree"], p["cells"], p["coords"], p["cn"], p["f"], p["N"])
            check_close(a[1], b, ab, "server rhs")
        else:
            y, ay = oracle.apply_action(p["dim"], p["degree"], p["cells"], p["coords"], p["cn"], p["kappa"], p["x"],
                                        p["N"])
            check_close(a[1], y, ay, "server action")
    srv1.close(); srv8.close()


def test_admission_respects_the_budget_and_slots():
    F, ctx, srv, models = _server(4, 1 << 30, SPECS[:2])
    resident = sum(p["resident"] for p in models)
    big = models[1]
    req = 8 * (big["info"]["nnz"] + big["N"])
    srv.close()
    # a budget that holds the resident models and one assembly's outputs
    F, ctx, srv, models = _server(4, resident + req + req // 2, SPECS[:2])
    big = models[1]
    rids = [srv.submit(big["id"], F.FEM_REQ_ASSEMBLE) for _ in range(6)]
    t0 = time.perf_counter()
    seen_running = 0
    done = set()
    while len(done) < len(rids):
        _, running, queued = srv.poll(time.perf_counter() - t0)
        seen_running = max(seen_running, running)
        for r in rids:
            if r in done:
                continue
            try:
                srv.result(r)
            except F.FemError:
                continue
            srv.release(r)
            done.add(r)
        assert time.perf_counter() - t0 < 60
    assert seen_running == 1          # memory, not slots, limited admission
    srv.close()
    with pytest.raises(F.FemError) as e:              # resident models beyond the budget
        _server(2, resident // 2, SPECS[:2])
    assert e.value.status == F.FEM_E_NOMEM
    F, ctx, tiny, m2 = _server(2, resident + 64, SPECS[:2])
    with pytest.raises(F.FemError) as e:              # outputs that can never fit
        tiny.submit(m2[1]["id"], F.FEM_REQ_ASSEMBLE)
    assert e.value.status == F.FEM_E_NOMEM
    tiny.close()


def test_server_rejections():
    F, ctx, srv, models = _server(2, 4 << 30, SPECS[:1])
    p = models[0]
    for bad, work in ((0, 1e8), (65, 1e8), (4, 0.0)):
        with pytest.raises(F.FemError) as e:
            srv.set_batch(bad, work)
        assert e.value.status == F.FEM_E_ARG
    with pytest.raises(F.FemError) as e:
        srv.submit(5, F.FEM_REQ_ASSEMBLE)
    assert e.value.status == F.FEM_E_ARG
    with pytest.raises(F.FemError) as e:
        srv.submit(p["id"], F.FEM_REQ_ACTION, None)
    assert e.value.status == F.FEM_E_ARG
    rid = srv.submit(p["id"], F.FEM_REQ_ASSEMBLE)
    with pytest.raises(F.FemError) as e:              # not admitted yet: no poll has run
        srv.result(rid)
    assert e.value.status == F.FEM_E_ARG
    _drain(srv, F, [rid], {rid: p}, {rid: F.FEM_REQ_ASSEMBLE})
    with pytest.raises(F.FemError) as e:              # released already
        srv.release(rid)
    assert e.value.status == F.FEM_E_ARG
    srv.close()


def test_shortest_first_order():
    """FEM_SERVE_SHORTEST admits the smallest queued request first (unless the
    head has waited max_wait); results are bitwise those of FIFO admission."""
    F, ctx, srv, models = _server(1, 8 << 30)
    srv.set_batch(1)                       # admission order is visible one request at a time
    big, small = models[5], models[0]      # a P3 tetrahedron assembly, a P1 triangle action
    with pytest.raises(F.FemError):
        srv.set_order(7, 0.0)
    with pytest.raises(F.FemError):
        srv.set_order(F.FEM_SERVE_SHORTEST, -1.0)

    def run(order, max_wait):
        srv.set_order(order, max_wait)
        rb = srv.submit(big["id"], F.FEM_REQ_ASSEMBLE)
        rs = srv.submit(small["id"], F.FEM_REQ_ACTION, small["g"]["x"])
        res = _drain(srv, F, [rb, rs], {rb: big, rs: small}, {rb: F.FEM_REQ_ASSEMBLE, rs: F.FEM_REQ_ACTION})
        return res[rb], res[rs]

    fb, fs = run(F.FEM_SERVE_FIFO, 0.0)
    assert fb[2] < fs[2], "FIFO admits in arrival order"
    sb, ss = run(F.FEM_SERVE_SHORTEST, 1e9)
    assert ss[2] < sb[2], "the smaller request goes first"
    hb, hs = run(F.FEM_SERVE_SHORTEST, 0.0)
    assert hb[2] < hs[2], "a head that has waited max_wait goes first"
    for a, b in ((fb, sb), (fb, hb)):
        assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64))
        assert np.array_equal(a[1].view(np.uint64), b[1].view(np.uint64))
    for a, b in ((fs, ss), (fs, hs)):
        assert np.array_equal(a[1].view(np.uint64), b[1].view(np.uint64))
    srv.close()


def test_batch_work_bound():
    """A batch closes before a request that would take its estimated work
    past the bound; that request then runs in a batch of its own."""
    F, ctx, srv, models = _server(1, 8 << 30)
    small, big = models[0], models[5]          # a P1 triangle action, a P3 tetrahedron assembly
    # an action's estimated work: its Dat plan's cell visits times nloc^2 (the
    # server's plan is built the same way on the same device)
    g = small["g"]
    vplan = F.fem_plan_create(ctx, F.form("helmholtz", 2, 1), F.Args(g["cv"], g["X"], g["cn"], small["N"],
                                                                     [g["kappa"]]), None)
    w_small = vplan.info()["cell_visits"] * 9
    srv.set_batch(64, 2.5 * w_small)           # two small actions fit, a third or the large assembly not
    seq = [(small, F.FEM_REQ_ACTION), (small, F.FEM_REQ_ACTION), (big, F.FEM_REQ_ASSEMBLE),
           (small, F.FEM_REQ_ACTION)]
    rids = [srv.submit(p["id"], op, p["g"]["x"] if op == F.FEM_REQ_ACTION else None) for p, op in seq]
    _, running, queued = srv.poll(0.0)
    assert (running, queued) == (2, 2), "the batch closes before the large request"
    res = _drain(srv, F, rids, dict(zip(rids, [p for p, _ in seq])), dict(zip(rids, [op for _, op in seq])))
    assert res[rids[2]][2] > res[rids[0]][2], "the large request is admitted in a later batch"
    srv.close()
