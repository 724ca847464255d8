#!/usr/bin/env python3
"""Benchmark of the cell-loop assembler on one MI355X.

Workload (one "step" = one pass of the whole hot path over the mesh):
  P2 Lagrange Helmholtz form  kappa grad(u).grad(v) + u v  on the unit cube,
  64^3 cubes x 6 Kuhn tetrahedra = 1,572,864 cells, interior vertices jittered
  by U[-0.2h, 0.2h], kappa a P1 field U[0.5, 1.5], f a P1 field U[-1, 1],
  x U[-1, 1]; FP64.  Step = CSR matrix assembly (WRITE) + source vector
  assembly (WRITE) + matrix-free action y = A x (WRITE).
Inputs are seeded and synthetic: the lattice mesh is shuffled (seeded) to
emulate an unstructured numbering, then renumbered by the library's Hilbert
renumbering, as the paper renumbers its meshes for locality.  Setup (sparsity,
plans) is timed separately and is not part of a step.

Prints ONE JSON line (rank 0).  value = cells / step time.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "assembled cells/s + % HBM roofline vs plain FP64; p50/p99 batched latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_inputs(n: int, degree: int, seed: int, mesh: str = "cube"):
    import fem_inputs as fi
    st = fi.spawn_streams(seed)
    m = fi.jitter_interior(fi.unit_cube(n) if mesh == "cube" else fi.unit_square(n), 0.2, st["mesh"])
    cn, N = fi.node_map(m, degree)
    kappa = fi.field(st["kappa"], m.nverts, 0.5, 1.5)
    f = fi.field(st["f"], m.nverts, -1.0, 1.0)
    x = fi.field(st["x"], N, -1.0, 1.0)
    # seeded shuffle of cells, vertices and nodes (unstructured numbering)
    rng = np.random.default_rng(seed + 1)
    cp = rng.permutation(m.ncells)
    cells, cn = fi.permute_cells(cp, m.cells, cn)
    vp = rng.permutation(m.nverts)
    vinv = np.empty_like(vp); vinv[vp] = np.arange(vp.size)
    cells = vinv[cells].astype(np.int32)
    coords, kappa, f = m.coords[vp], kappa[vp], f[vp]
    npn = rng.permutation(N)
    ninv = np.empty_like(npn); ninv[npn] = np.arange(N)
    cn = ninv[cn].astype(np.int32)
    x = x[npn]
    return dict(cells=np.ascontiguousarray(cells), coords=np.ascontiguousarray(coords),
                cn=np.ascontiguousarray(cn), N=N, kappa=kappa, f=f, x=x)


def apply_perms(d, cp, vp, npn):
    vinv = np.empty_like(vp); vinv[vp] = np.arange(vp.size, dtype=vp.dtype)
    ninv = np.empty_like(npn); ninv[npn] = np.arange(npn.size, dtype=npn.dtype)
    return dict(cells=np.ascontiguousarray(vinv[d["cells"][cp]]).astype(np.int32),
                coords=np.ascontiguousarray(d["coords"][vp]),
                cn=np.ascontiguousarray(ninv[d["cn"][cp]]).astype(np.int32), N=d["N"],
                kappa=d["kappa"][vp].copy(), f=d["f"][vp].copy(), x=d["x"][npn].copy())


KERNEL_SOURCES = ["paper_1501_01809_amd/csrc/fem_assemble.hip", "paper_1501_01809_amd/csrc/fem_api.cpp",
                  "paper_1501_01809_amd/csrc/fem_internal.h", "paper_1501_01809_amd/csrc/gen_tables.py"]


def kernel_source_hash() -> str:
    """sha256 over the sources that decide what the Mat kernel reads and writes."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(args, name):
    """HBM bytes per launch of the dominant kernel, from the committed counter
    summary profiles/<name>_traffic.md (FETCH_SIZE and WRITE_SIZE, each scaled
    by the factor a plain copy of known size gives), or None when the summary
    is missing, was taken for another workload, or the kernel sources changed
    since (its recorded source hash differs)."""
    if args.n != 64 or args.degree != 2 or args.no_renumber or args.mesh != "cube":
        return None
    path = os.path.join(ROOT, "profiles", name + "_traffic.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                rec[k.strip()] = v.strip().strip("`")
    try:
        if rec.get("source_sha256") != kernel_source_hash():
            return None
        return int(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(d, degree, sample_cells, dim=3):
    """The oracle, as it stands, on the first `sample_cells` cells of the same
    (renumbered) mesh: sparsity + matrix + vector + action, one thread.  The
    paper's protocol: one dry run, then the minimum of three timed runs."""
    import oracle
    cells = d["cells"][:sample_cells]; cn = d["cn"][:sample_cells]
    oracle.lib()

    def once():
        t0 = time.perf_counter()
        rp, ci = oracle.sparsity(cn, d["N"])
        oracle.assemble_mat(dim, degree, cells, d["coords"], cn, d["kappa"], rp, ci)
        oracle.assemble_vec(dim, degree, cells, d["coords"], cn, d["f"], d["N"])
        oracle.apply_action(dim, degree, cells, d["coords"], cn, d["kappa"], d["x"], d["N"])
        return time.perf_counter() - t0

    once()
    runs = [once() for _ in range(3)]
    t = min(runs)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": sample_cells / t, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_cells} cells of the same renumbered mesh, full step "
                      f"(sparsity+mat+vec+action), one dry run then the minimum of 3 "
                      f"({', '.join(f'{r:.2f}' for r in runs)} s), single-threaded on {cpu}, "
                      f"{len(os.sched_getaffinity(0))} host cores visible"}


def bench_nl(ctx, steps: int, warmup: int, seed: int, n: int = 512):
    """The differentiation workload: the P1 residual
    F(u, kappa)_i = integral of kappa grad(u).grad(v_i) + u^3 v_i - f v_i and its
    vector-Jacobian products lambda^T dF/du, lambda^T dF/dkappa on the unit
    square, n x n x 2 triangles jittered by U[-0.2h, 0.2h], shuffled then
    Hilbert-renumbered; u U[-1,1], kappa U[0.5,1.5], f U[-1,1], lambda U[-1,1]
    on the nodes.  Timed per call with HIP events, FP64 and FP32 arithmetic."""
    import torch
    import fem_inputs as fi
    from paper_1501_01809_amd import fem as F
    dev = torch.device("cuda:0")
    st = fi.spawn_streams(seed)
    m = fi.jitter_interior(fi.unit_square(n), 0.2, st["mesh"])
    cn, N = fi.node_map(m, 1)
    rng = np.random.default_rng(seed + 1)
    cells, cn = fi.permute_cells(rng.permutation(m.ncells), m.cells, cn)
    vp = rng.permutation(m.nverts)
    vinv = np.empty_like(vp); vinv[vp] = np.arange(vp.size)
    cells = np.ascontiguousarray(vinv[cells].astype(np.int32))
    coords = np.ascontiguousarray(m.coords[vp])
    cn = np.ascontiguousarray(cn, dtype=np.int32)
    C, V = cells.shape[0], coords.shape[0]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g_cv, g_X, g_cn = t(cells), t(coords), t(cn)
    f64 = F.form("nl_residual", 2, 1)
    cp, vperm, nperm = F.fem_renumber(ctx, f64, F.Args(g_cv, g_X, g_cn, N))
    vi = np.empty_like(vperm); vi[vperm] = np.arange(vperm.size)
    ni = np.empty_like(nperm); ni[nperm] = np.arange(nperm.size)
    cells = np.ascontiguousarray(vi[cells[cp]].astype(np.int32))
    cn = np.ascontiguousarray(ni[cn[cp]].astype(np.int32))
    coords = np.ascontiguousarray(coords[vperm])
    g_cv, g_X, g_cn = t(cells), t(coords), t(cn)
    u, kap, f, lam = (t(fi.field(st[k], N, lo, hi)) for k, lo, hi in
                      (("u", -1.0, 1.0), ("kappa", 0.5, 1.5), ("f", -1.0, 1.0), ("lam_adj", -1.0, 1.0)))
    res = torch.empty(N, dtype=torch.float64, device=dev)
    gu, gk = torch.empty_like(res), torch.empty_like(res)
    a3 = F.Args(g_cv, g_X, g_cn, N, [u, kap, f], nodal=True)
    a2 = F.Args(g_cv, g_X, g_cn, N, [u, kap], nodal=True)
    stream = torch.cuda.current_stream(dev)
    per_launch = 4 * C * 3 + 8 * V * 2 + 8 * N * 3 + 8 * N   # the P1 Map, coords, 3 node fields, 1 output
    out = {"workload": f"P1 nonlinear residual and adjoint on the unit square, {n}x{n}x2 triangles "
                       f"({C} cells, {N} nodes), jitter 0.2h", "cells": C, "nodes": N}
    for name, prec in (("fp64", F.FEM_FP64), ("fp32", F.FEM_FP32)):
        frm = F.form("nl_residual", 2, 1, prec=prec)
        plan = F.fem_plan_create(ctx, frm, F.Args(g_cv, g_X, g_cn, N), None)
        calls = {"residual": (lambda: F.fem_par_loop_assemble_vec(ctx, plan, frm, a3, res), per_launch),
                 # both products from one launch: one gather, two outputs
                 "adjoint": (lambda: F.fem_par_loop_assemble_adjoint(ctx, plan, frm, a2, lam, gu, gk),
                             per_launch + 8 * N)}
        rec = {}
        for op, (fn, by) in calls.items():
            for _ in range(warmup):
                fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            torch.cuda.synchronize()
            ev[0].record(stream)
            for k in range(steps):
                fn()
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
            rec[op] = {"ms": float(ms.mean()), "ms_min": float(ms.min()), "cells_per_s": C / (ms.mean() * 1e-3),
                       "alg_bytes": by, "GBps": by / (ms.mean() * 1e-3) / 1e9,
                       "hbm_frac": by / (ms.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out[name] = rec
    return out


def bench_precision(ctx, steps: int, warmup: int, seed: int, n: int = 48):
    """The precision workload: vector P2 linear elasticity
    2 mu eps(u):eps(v) + lam div u div v on n^3 x 6 Kuhn tetrahedra jittered by
    U[-0.2h, 0.2h], per-cell coordinates with 1% of the cells flattened to
    aspect ratio ~1e3, mu and lam P1 U[0.5, 2]; CSR assembly (WRITE) with the
    element contraction in FP64, FP32, BF16 and FP16 (FP64 geometry and
    global sums).  Timed per call (element kernel + pull) with HIP events."""
    import torch
    import fem_inputs as fi
    from paper_1501_01809_amd import fem as F
    dev = torch.device("cuda:0")
    st = fi.spawn_streams(seed)
    m = fi.jitter_interior(fi.unit_cube(n), 0.2, st["mesh"])
    xdg, chosen = fi.flatten_cells(fi.dg_coordinates(m), 0.01, st["flatten"])
    cn, N = fi.node_map(m, 2)
    mu = fi.field(st["mu"], m.nverts, 0.5, 2.0)
    lam = fi.field(st["lam"], m.nverts, 0.5, 2.0)
    C = m.ncells
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    # Hilbert renumbering of cells, vertices and nodes (through the scalar P2
    # form on the continuous mesh), as for the other workloads
    t0 = time.perf_counter()
    cells = m.cells.astype(np.int32); cn = cn.astype(np.int32)
    cp, vp, npn = F.fem_renumber(ctx, F.form("helmholtz", 3, 2),
                                 F.Args(t(cells), t(m.coords), t(cn), N, [t(mu)]))
    vinv = np.empty_like(vp); vinv[vp] = np.arange(vp.size, dtype=vp.dtype)
    ninv = np.empty_like(npn); ninv[npn] = np.arange(npn.size, dtype=npn.dtype)
    cells = vinv[cells[cp]].astype(np.int32); cn = ninv[cn[cp]].astype(np.int32)
    xdg = xdg[cp]; mu = mu[vp]; lam = lam[vp]
    renumber_ms = (time.perf_counter() - t0) * 1e3
    g_cv, g_cn, g_X = t(cells), t(cn), t(xdg.reshape(-1, 3))
    g_cc = t(np.arange(4 * C, dtype=np.int32).reshape(C, 4))
    args = F.Args(g_cv, g_X, g_cn, N, [t(mu), t(lam)], cell_coord=g_cc)
    t0 = time.perf_counter()
    sp = F.fem_expand_sparsity(ctx, F.fem_build_sparsity(ctx, g_cn, N), 3)
    torch.cuda.synchronize()
    setup = {"renumber_ms": renumber_ms, "sparsity_ms": (time.perf_counter() - t0) * 1e3}
    nnz = int(sp.col_idx.numel())
    vals = torch.empty(nnz, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    V = m.nverts
    alg = C * (4 * 10 + 4 * 4 + 4 * 4) + C * 4 * 3 * 8 + V * 16 + (3 * N + 1) * 8 + 4 * nnz + 8 * nnz
    out = {"workload": f"vector P2 elasticity on the unit cube, {n}^3x6 Kuhn tets ({C} cells, {3 * N} DOFs, "
                       f"nnz {nnz}), jitter 0.2h, {chosen.size} cells flattened to aspect ~1e3, mu, lam P1 "
                       f"U[0.5,2], Hilbert-renumbered", "cells": C, "dofs": 3 * N, "nnz": nnz, "alg_bytes": alg,
           "flop_per_cell": 2 * 55 * 9 * 36}
    for name in ("fp64", "fp32", "bf16", "fp16"):
        frm = F.form("elasticity", 3, 2, 3, F.PRECS[name])
        t0 = time.perf_counter()
        plan = F.fem_plan_create(ctx, frm, args, sp)
        setup[f"plan_{name}_ms"] = (time.perf_counter() - t0) * 1e3
        for _ in range(warmup):
            F.fem_par_loop_assemble_mat(ctx, plan, frm, args, vals, sp)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            F.fem_par_loop_assemble_mat(ctx, plan, frm, args, vals, sp)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        out[name] = {"ms": float(ms.mean()), "ms_min": float(ms.min()), "cells_per_s": C / (ms.mean() * 1e-3),
                     "GBps": alg / (ms.mean() * 1e-3) / 1e9,
                     "hbm_frac": alg / (ms.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del plan
    for name in ("fp32", "bf16", "fp16"):
        out[name]["speedup_vs_fp64"] = out["fp64"]["ms"] / out[name]["ms"]
    out["setup_ms"] = setup
    return out


def bench_serving(ctx, seed: int, nreq: int = 4096, loads=(0.5, 0.8, 1.2), slots: int = 4,
                  max_wait_ms: float = 100.0, max_batch: int = 64):
    """The serving workload: a stream of `nreq` requests with Poisson arrivals
    at rate load / s, s the mean isolated service time of the mix, for each
    load in `loads`.  Each request is an assembly (CSR matrix + right-hand
    side) or a matrix-free action, drawn uniformly, on a resident model drawn
    uniformly by mesh kind (unit-square triangles, n in 16..512; Kuhn cubes,
    n in 8..64), size and Lagrange degree 1..3; jittered meshes, fields
    U[0.5, 1.5].  The same request sequence (arrival times scaled by the
    load) is served by each policy: `slots` slots with batches of up to
    `max_batch` requests in shared persistent launches, in arrival order
    ("batched") or smallest first with a queue head that has waited
    max_wait_ms going first ("batched_shortest"); and one slot with one
    request per launch ("one_slot", requests served one at a time).  Latency =
    completion seen by the poll loop minus arrival; cells/s = cells of the
    requests / makespan."""
    import torch
    import fem_inputs as fi
    from paper_1501_01809_amd import fem as F
    dev = torch.device("cuda:0")
    kinds = {"square": [16, 32, 64, 128, 256, 512], "cube": [8, 16, 32, 64]}
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rng = np.random.default_rng(seed + 5)
    specs = []
    t0 = time.perf_counter()
    for kind, sizes in kinds.items():
        for n in sizes:
            st = fi.spawn_streams(seed + n)
            m = fi.jitter_interior(fi.unit_square(n) if kind == "square" else fi.unit_cube(n), 0.2, st["mesh"])
            for k in (1, 2, 3):
                cn, N = fi.node_map(m, k)
                g = dict(cv=t(m.cells), X=t(m.coords), cn=t(cn.astype(np.int32)),
                         kappa=t(fi.field(st["kappa"], m.nverts, 0.5, 1.5)),
                         f=t(fi.field(st["f"], m.nverts, 0.5, 1.5)), x=t(fi.field(st["x"], N, 0.5, 1.5)))
                specs.append(dict(kind=kind, n=n, degree=k, dim=m.dim, cells=m.ncells, N=N, g=g))
    build_ms = (time.perf_counter() - t0) * 1e3

    def make_server(ns):
        srv = F.Server(ctx, ns, 96 << 30)
        for sp_ in specs:
            g = sp_["g"]
            mid, res = srv.add_model(F.form("helmholtz", sp_["dim"], sp_["degree"]),
                                     F.Args(g["cv"], g["X"], g["cn"], sp_["N"], [g["kappa"], g["f"]]))
            sp_["id"], sp_["resident"] = mid, res
        return srv

    log(f"serving: inputs of {len(specs)} models built ({build_ms / 1e3:.1f} s)")
    t0 = time.perf_counter()
    srv = make_server(slots)
    setup_ms = (time.perf_counter() - t0) * 1e3
    resident = sum(sp_["resident"] for sp_ in specs)

    def serve_one(srv_, sp_, op):
        rid = srv_.submit(sp_["id"], op, sp_["g"]["x"] if op == F.FEM_REQ_ACTION else None, 0.0)
        c0 = time.perf_counter()
        while True:
            c, _, _ = srv_.poll(time.perf_counter() - c0)
            if c and rid in srv_.take_completed():
                break
        _, _, _, td = srv_.result(rid)
        srv_.release(rid)
        return td

    srv.configure(1, False)
    srv.set_batch(1)
    # service time of every (model, op) alone with warm caches (best of two
    # after a warm-up), for reference
    iso = {}
    for sp_ in specs:
        for op in (F.FEM_REQ_ASSEMBLE, F.FEM_REQ_ACTION):
            serve_one(srv, sp_, op)
            iso[(sp_["id"], op)] = min(serve_one(srv, sp_, op), serve_one(srv, sp_, op))
    # the request mix: kind uniform, then size, degree and op uniform
    by_kind = {kd: [sp_ for sp_ in specs if sp_["kind"] == kd] for kd in kinds}

    def draw():
        kd = list(kinds)[rng.integers(2)]
        return by_kind[kd][rng.integers(len(by_kind[kd]))], int(rng.integers(2))

    # mean isolated service time s of the mix: a sample of 512 requests, each
    # served alone (submitted after the previous one completed), in mix order,
    # so that caches hold what a stream of mixed requests leaves in them
    sample = [draw() for _ in range(512)]
    sbar = float(np.mean([serve_one(srv, sp_, op) for sp_, op in sample]))
    gaps = rng.exponential(1.0, nreq)          # unit-rate gaps, scaled per load
    mix = [draw() for _ in range(nreq)]

    def run(srv_, arrivals):
        lat = np.zeros(nreq); svc = np.zeros(nreq); cells = 0
        ids = {}
        nxt = 0; done = 0
        c0 = time.perf_counter()
        while done < nreq:
            now = time.perf_counter() - c0
            while nxt < nreq and arrivals[nxt] <= now:
                sp_, op = mix[nxt]
                rid = srv_.submit(sp_["id"], op, sp_["g"]["x"] if op == F.FEM_REQ_ACTION else None,
                                  float(arrivals[nxt]))
                ids[rid] = nxt
                nxt += 1
            c, _, _ = srv_.poll(now)
            if c:
                for rid in srv_.take_completed():
                    _, _, ta, td = srv_.result(rid)
                    i = ids.pop(rid)
                    lat[i] = td - arrivals[i]
                    svc[i] = td - ta
                    cells += mix[i][0]["cells"]
                    srv_.release(rid)
                    done += 1
        span = time.perf_counter() - c0
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "makespan_s": span, "arrival_span_s": float(arrivals[-1]),
                "cells_per_s": cells / span, "admit_to_done_mean_ms": float(svc.mean() * 1e3)}

    out = {"workload": f"{nreq} requests, Poisson arrivals at load x (1 / mean isolated service time) for load in "
                       f"{list(loads)}; assembly (CSR + RHS) or action, unit-square triangle meshes n=16..512 and "
                       f"Kuhn cubes n=8..64, P1-P3, fields U[0.5,1.5]; {len(specs)} resident models",
           "models": len(specs), "resident_bytes": resident, "inputs_ms": build_ms, "setup_ms": setup_ms,
           "mean_isolated_service_ms": sbar * 1e3, "slots": slots, "max_batch": max_batch,
           "shortest_max_wait_ms": max_wait_ms,
           "isolated_ms": {f"{sp_['kind']}{sp_['n']}p{sp_['degree']}": [round(iso[(sp_['id'], 0)] * 1e3, 3),
                                                                       round(iso[(sp_['id'], 1)] * 1e3, 3)]
                           for sp_ in specs}, "loads": {}}
    log(f"serving: {len(specs)} models resident ({resident / 1e9:.1f} GB), setup {setup_ms / 1e3:.1f} s, "
        f"mean isolated service {sbar * 1e3:.3f} ms; {slots} slots, batches of up to {max_batch}")
    # (name, slots, requests per batch, order, Mat launches on half the CUs
    # while others run); one slot has nothing to share the GPU with
    policies = (("batched", slots, max_batch, F.FEM_SERVE_FIFO, True),
                ("batched_shortest", slots, max_batch, F.FEM_SERVE_SHORTEST, True),
                ("batched_full_grid", slots, max_batch, F.FEM_SERVE_FIFO, False),
                ("one_slot", 1, 1, F.FEM_SERVE_FIFO, False))
    for load in loads:
        arrivals = np.cumsum(gaps) * sbar / load
        rec = {"arrival_rate_per_s": load / sbar}
        for name, ns, nb, order, share in policies:
            srv.configure(ns, share)
            srv.set_batch(nb)
            srv.set_order(order, max_wait_ms * 1e-3)
            rec[name] = run(srv, arrivals)
            log(f"serving: load {load} {name}: p50 {rec[name]['p50_ms']:.2f} ms p99 {rec[name]['p99_ms']:.2f} ms "
                f"{rec[name]['cells_per_s']:.3g} cells/s")
        out["loads"][str(load)] = rec
    srv.close()
    return out


def bench_extras(ctx, d, g, sp, mplan, vplan, dim, degree, steps, warmup):
    """The paper-adjacent steps on the main workload's mesh, each timed per
    call with HIP events: the Global SUM of the cell energies x^T A x, the
    Dirichlet rows and columns of the assembled system (boundary nodes of the
    cube, lifted boundary values), the exterior facet integral of g v, and a
    two-field mixed system by blocks (four Mats)."""
    import torch
    import fem_inputs as fi
    from paper_1501_01809_amd import fem as F
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def timeit(fn):
        for _ in range(warmup):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        return float(ms.mean()), float(ms.min())

    C = d["cells"].shape[0]; N = d["N"]; V = d["coords"].shape[0]; nl = d["cn"].shape[1]
    nnz = int(sp.col_idx.numel())
    form = F.form("helmholtz", dim, degree)
    args_k = F.Args(g["cv"], g["X"], g["cn"], N, [g["kappa"]])
    out = {}
    gl = torch.zeros(1, dtype=torch.float64, device=dev)
    ms, mn = timeit(lambda: F.fem_par_loop_reduce(ctx, vplan, form, args_k, g["x"], gl, F.FEM_SUM))
    by = 4 * C * (nl + dim + 1) + 8 * V * (dim + 1) + 8 * N
    out["global_energy_sum"] = {"ms": ms, "ms_min": mn, "cells_per_s": C / (ms * 1e-3), "alg_bytes": by,
                                "GBps": by / (ms * 1e-3) / 1e9}
    mesh = fi.Mesh(dim, d["coords"], d["cells"])
    mask = fi.boundary_nodes(mesh, d["cn"], degree)
    vals = torch.empty(nnz, dtype=torch.float64, device=dev)
    F.fem_par_loop_assemble_mat(ctx, mplan, form, args_k, vals, sp)
    b = torch.zeros(N, dtype=torch.float64, device=dev)
    gv = t(np.where(mask == 1, 1.0, 0.0))
    gm = t(mask)
    ms, mn = timeit(lambda: F.fem_apply_dirichlet(ctx, sp, vals, gm, 1.0, b, gv))
    by = 8 * (N + 1) + 4 * nnz + 16 * nnz + N + 24 * N
    out["dirichlet"] = {"ms": ms, "ms_min": mn, "boundary_dofs": int(mask.sum()), "alg_bytes": by,
                        "GBps": by / (ms * 1e-3) / 1e9}
    fv, fn = fi.exterior_facets(mesh, d["cn"], degree)
    fa = F.Facets(t(fv), t(fn), g["X"], g["f"], N)
    src = F.form("source", dim, degree)
    fplan = F.fem_facet_plan_create(ctx, src, fa)
    bf = torch.empty(N, dtype=torch.float64, device=dev)
    ms, mn = timeit(lambda: F.fem_par_loop_assemble_facets(ctx, fplan, src, fa, bf))
    out["exterior_facets"] = {"ms": ms, "ms_min": mn, "facets": int(fv.shape[0]),
                              "facets_per_s": fv.shape[0] / (ms * 1e-3)}
    blocks = [[("mass", 1.0, None), ("laplace", 0.25, g["kappa"])],
              [("laplace", -0.01, g["kappa"]), ("mass", 1.0, None)]]
    bvals = [[torch.empty(nnz, dtype=torch.float64, device=dev) for _ in range(2)] for _ in range(2)]
    ms, mn = timeit(lambda: F.fem_par_loop_assemble_mixed(ctx, mplan, form, args_k, blocks, bvals, sp))
    out["mixed_2x2_blocks"] = {"ms": ms, "ms_min": mn, "cells_per_s": C / (ms * 1e-3)}
    del bvals, vals
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="cubes (or squares) per side")
    ap.add_argument("--mesh", choices=("cube", "square"), default="cube",
                    help="n^3 x 6 Kuhn tetrahedra (default) or n x n x 2 triangles")
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1501)
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-renumber", action="store_true")
    ap.add_argument("--no-nl", action="store_true",
                    help="skip the differentiation workload (residual and adjoint, 512x512x2 triangles)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the precision workload (vector P2 elasticity, 48^3x6, four precisions)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving workload (4096 requests on 30 resident models)")
    ap.add_argument("--serving-requests", type=int, default=4096)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the paper-adjacent steps (Global energy, Dirichlet rows, facets, mixed blocks)")
    ap.add_argument("--ops", default="mat,vec,action",
                    help="operations run in a step (a subset is for profiling the kernels one by one; "
                         "the reported metric needs all three)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (3 launches) to calibrate the "
                         "HBM byte counters of a profiler, then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py runs on exactly one GPU: the library has no multi-GPU path "
                 "(one GPU's share of the mesh is the measured unit).")

    import torch
    from paper_1501_01809_amd import fem as F
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": 8 * n, "calibrate_copy_bytes_written": 8 * n}))
        return
    t0 = time.perf_counter()
    d = build_inputs(args.n, args.degree, args.seed, args.mesh)
    dim = 3 if args.mesh == "cube" else 2
    log(f"inputs: {d['cells'].shape[0]} cells, {d['N']} nodes ({time.perf_counter() - t0:.1f} s)")
    ctx = F.Context(0)
    C = d["cells"].shape[0]

    def upload(dd):
        return dict(cv=torch.from_numpy(dd["cells"]).to(dev), X=torch.from_numpy(dd["coords"]).to(dev),
                    cn=torch.from_numpy(dd["cn"]).to(dev), kappa=torch.from_numpy(dd["kappa"]).to(dev),
                    f=torch.from_numpy(dd["f"]).to(dev), x=torch.from_numpy(dd["x"]).to(dev))

    form = F.form("helmholtz", dim, args.degree)
    src = F.form("source", dim, args.degree)
    setup = {}
    g = upload(d)
    if not args.no_renumber:
        t = time.perf_counter()
        a0 = F.Args(g["cv"], g["X"], g["cn"], d["N"], [g["kappa"]])
        cp, vp, npn = F.fem_renumber(ctx, form, a0)
        setup["renumber_ms"] = (time.perf_counter() - t) * 1e3
        d = apply_perms(d, cp, vp, npn)
        g = upload(d)
    args_k = F.Args(g["cv"], g["X"], g["cn"], d["N"], [g["kappa"]])
    args_f = F.Args(g["cv"], g["X"], g["cn"], d["N"], [g["f"]])
    torch.cuda.synchronize()
    t = time.perf_counter()
    sp = F.fem_build_sparsity(ctx, g["cn"], d["N"])
    torch.cuda.synchronize()
    setup["sparsity_ms"] = (time.perf_counter() - t) * 1e3
    t = time.perf_counter()
    mplan = F.fem_plan_create(ctx, form, args_k, sp)
    setup["mat_plan_ms"] = (time.perf_counter() - t) * 1e3
    t = time.perf_counter()
    vplan = F.fem_plan_create(ctx, form, args_k, None)
    setup["vec_plan_ms"] = (time.perf_counter() - t) * 1e3
    nnz = int(sp.col_idx.numel()); N = d["N"]
    log(f"setup: nnz={nnz} {setup} mat plan {mplan.info()} vec plan {vplan.info()}")

    vals = torch.empty(nnz, dtype=torch.float64, device=dev)
    b = torch.empty(N, dtype=torch.float64, device=dev)
    y = torch.empty(N, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    ops_on = set(args.ops.split(","))

    def step(ev=None):
        if ev: ev[0].record(stream)
        if "mat" in ops_on:
            F.fem_par_loop_assemble_mat(ctx, mplan, form, args_k, vals, sp, F.FEM_WRITE)
        if ev: ev[1].record(stream)
        if "vec" in ops_on:
            F.fem_par_loop_assemble_vec(ctx, vplan, src, args_f, b, F.FEM_WRITE)
        if ev: ev[2].record(stream)
        if "action" in ops_on:
            F.fem_apply_action(ctx, vplan, form, args_k, g["x"], y, F.FEM_WRITE)
        if ev: ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    per = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                     e[0].elapsed_time(e[3])] for e in evs])   # ms
    ms_step = wall * 1e3 / args.steps
    mat_ms, vec_ms, act_ms = (float(np.mean(per[:, i])) for i in range(3))

    # algorithmic bytes per launch (one read of inputs and structure, one write of outputs)
    V = d["coords"].shape[0]; nl = d["cn"].shape[1]
    # the cell-to-node Map, plus the cell-to-vertex Map when it is a different
    # Map (degree > 1; at P1 the nodes are the vertices and one Map serves both)
    maps = 4 * C * nl + (4 * C * (dim + 1) if args.degree > 1 else 0)
    vdata = 8 * V * dim + 8 * V
    mat_bytes = maps + vdata + 8 * (N + 1) + 4 * nnz + 8 * nnz
    vec_bytes = maps + vdata + 8 * N
    act_bytes = maps + vdata + 8 * N + 8 * N
    gbs = lambda by, ms: by / (ms * 1e-3) / 1e9
    ops = {
        "mat": {"ms": mat_ms, "ms_min": float(per[:, 0].min()), "cells_per_s": C / (mat_ms * 1e-3),
                "alg_bytes": mat_bytes, "GBps": gbs(mat_bytes, mat_ms),
                "hbm_frac": gbs(mat_bytes, mat_ms) / HBM_PEAK_GBS,
                "plan": mplan.info()},
        "vec": {"ms": vec_ms, "cells_per_s": C / (vec_ms * 1e-3), "alg_bytes": vec_bytes,
                "GBps": gbs(vec_bytes, vec_ms), "hbm_frac": gbs(vec_bytes, vec_ms) / HBM_PEAK_GBS},
        "action": {"ms": act_ms, "cells_per_s": C / (act_ms * 1e-3), "alg_bytes": act_bytes,
                   "GBps": gbs(act_bytes, act_ms), "hbm_frac": gbs(act_bytes, act_ms) / HBM_PEAK_GBS,
                   "plan": vplan.info()},
    }
    out = {
        "metric": METRIC,
        "value": C / (ms_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"P{args.degree} Lagrange Helmholtz on the unit "
                               + (f"cube, {args.n}^3x6 Kuhn tets" if dim == 3 else
                                  f"square, {args.n}x{args.n}x2 triangles")
                               + f" ({C} cells, {N} DOFs, nnz {nnz}), jitter 0.2h, kappa P1 "
                               f"U[0.5,1.5], f P1 U[-1,1]; step = CSR matrix + source vector + "
                               f"matrix-free action, FP64",
                   "cells": C, "dofs": N, "nnz": nnz, "renumbered": not args.no_renumber},
        "roofline": {"bound": "hbm", "achieved": gbs(mat_bytes, mat_ms), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs(mat_bytes, mat_ms) / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args, "k_assemble_mat_p2tet64"),
                     "kernel": f"k_assemble_mat<{dim},{args.degree}>", "alg_bytes_per_launch": mat_bytes},
        "ops": ops,
        "step_ms_p50": float(np.percentile(per[:, 3], 50)),
        "step_ms_p99": float(np.percentile(per[:, 3], 99)),
        "setup_ms": setup,
        "host": platform.node(),
    }
    if not args.no_extras:
        out["paper_adjacent"] = bench_extras(ctx, d, g, sp, mplan, vplan, dim, args.degree, args.steps, args.warmup)
    if not args.no_nl:
        out["differentiation"] = bench_nl(ctx, args.steps, args.warmup, args.seed)
    if not args.no_precision:
        out["precision"] = bench_precision(ctx, args.steps, args.warmup, args.seed)
    if not args.no_serving:
        out["serving"] = bench_serving(ctx, args.seed, args.serving_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, args.degree, min(args.cpu_sample, C), dim)
        out["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
