#!/usr/bin/env python3
"""Generate ``fem_tables.h``: exact reference integrals of the Lagrange P1-P3
bases on triangles and tetrahedra, emitted as straight-line FP64 device code.

The element tensors of the local kernels are written in "metric" form
(the reference-tensor idea the paper cites for FFC: a per-cell geometry
tensor contracted with a cell-independent reference tensor):

  A_ij = sum_k sum_{m<=n} P[k][mn] W[k][mn][i][j]  +  madet * Mref_ij
  P[k][mn] = cstiff * kappa_k * |det J| grad(l_m).grad(l_n)
  W[k][mn][i][j] = int_ref l_k (d_m phi_i d_n phi_j + [m!=n] d_n phi_i d_m phi_j)
  Mref_ij = int_ref phi_i phi_j,   madet = cmass * |det J|
  b_i = |det J| sum_k f_k int_ref l_k phi_i

with l_0..l_d the barycentric coordinates and d_m the derivative with respect
to l_m (chain rule: grad phi = sum_m d_m phi grad l_m).  All integrals are
exact rationals (int_ref l^a = a!/(|a|+d)!), rounded once to double and
printed as hexadecimal literals; zero terms are dropped at generation time.

Each element tensor is emitted twice: from P (mat_group*, act) and from
kc[k] = cstiff kappa_k and the metric G[mn] = |det J| grad l_m . grad l_n
with the terms of an entry grouped by metric pair (mat_group_t*, act_t),
A_ij = sum_mn G[mn] (sum_k W[k][mn][i][j] kc[k]) + madet Mref_ij, which keeps
d+1 + NM values live instead of (d+1) x NM.

Local node order: vertices; edges (a<b lexicographic), the two P3 edge nodes
ordered from a; P3 tetrahedron faces (a<b<c lexicographic) or the P3
triangle's interior node.
"""
from __future__ import annotations

import itertools
import os
import sys
from fractions import Fraction
from math import factorial


def poly_mul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            e = tuple(x + y for x, y in zip(a, b))
            out[e] = out.get(e, 0) + ca * cb
    return {k: v for k, v in out.items() if v != 0}


def poly_add(*ps):
    out = {}
    for p in ps:
        for a, c in p.items():
            out[a] = out.get(a, 0) + c
    return {k: v for k, v in out.items() if v != 0}


def poly_scale(p, s):
    return {a: c * s for a, c in p.items()}


def poly_d(p, m):
    out = {}
    for a, c in p.items():
        if a[m]:
            e = list(a); e[m] -= 1
            out[tuple(e)] = out.get(tuple(e), 0) + c * a[m]
    return out


def integrate(p, d):
    s = Fraction(0)
    for a, c in p.items():
        num = 1
        for x in a:
            num *= factorial(x)
        s += c * Fraction(num, factorial(sum(a) + d))
    return s


def lam(nv, m):
    e = [0] * nv; e[m] = 1
    return {tuple(e): Fraction(1)}


def const(nv, c):
    return {tuple([0] * nv): Fraction(c)}


def basis(d, k):
    """Lagrange basis as polynomials in the barycentrics l_0..l_d."""
    nv = d + 1
    L = [lam(nv, m) for m in range(nv)]
    B = []
    for i in range(nv):
        if k == 1:
            B.append(L[i])
        elif k == 2:   # l (2l - 1)
            B.append(poly_mul(L[i], poly_add(poly_scale(L[i], 2), const(nv, -1))))
        else:          # l (3l - 1)(3l - 2) / 2
            B.append(poly_scale(poly_mul(L[i], poly_mul(poly_add(poly_scale(L[i], 3), const(nv, -1)),
                                                         poly_add(poly_scale(L[i], 3), const(nv, -2)))),
                                Fraction(1, 2)))
    for a, b in itertools.combinations(range(nv), 2):
        if k == 2:
            B.append(poly_scale(poly_mul(L[a], L[b]), 4))
        elif k == 3:
            ab = poly_mul(L[a], L[b])
            B.append(poly_scale(poly_mul(ab, poly_add(poly_scale(L[a], 3), const(nv, -1))), Fraction(9, 2)))
            B.append(poly_scale(poly_mul(ab, poly_add(poly_scale(L[b], 3), const(nv, -1))), Fraction(9, 2)))
    if k == 3:
        for f in itertools.combinations(range(nv), 3):
            p = const(nv, 27)
            for a in f:
                p = poly_mul(p, L[a])
            B.append(p)
    return B


def hexlit(x: Fraction) -> str:
    v = float(x)
    if v == 0.0:
        return "0.0"
    return v.hex()


def metric_pairs(nv):
    return [(m, n) for m in range(nv) for n in range(m, nv)]


def tables(d, k):
    nv = d + 1
    B = basis(d, k)
    n = len(B)
    dB = [[poly_d(B[i], m) for m in range(nv)] for i in range(n)]
    pairs = metric_pairs(nv)
    # stiffness terms for each upper entry (i<=j): list of (k, mn, coef)
    stiff = {}
    for i in range(n):
        for j in range(i, n):
            terms = []
            for kk in range(nv):
                for t, (m, q) in enumerate(pairs):
                    w = integrate(poly_mul(lam(nv, kk), poly_mul(dB[i][m], dB[j][q])), d)
                    if m != q:
                        w += integrate(poly_mul(lam(nv, kk), poly_mul(dB[i][q], dB[j][m])), d)
                    if w != 0:
                        terms.append((kk, t, w))
            stiff[(i, j)] = terms
    mass = {(i, j): integrate(poly_mul(B[i], B[j]), d) for i in range(n) for j in range(i, n)}
    src = [[integrate(poly_mul(lam(nv, kk), B[i]), d) for kk in range(nv)] for i in range(n)]
    return n, pairs, stiff, mass, src


def entry_expr(i, j, NM, stiff, mass):
    lines = []
    first = True
    for (kk, t, w) in stiff[(i, j)]:
        idx = kk * NM + t
        if first:
            lines.append(f"double e = {hexlit(w)} * P[{idx}];")
            first = False
        else:
            lines.append(f"e = __builtin_fma({hexlit(w)}, P[{idx}], e);")
    mw = mass[(i, j)]
    if mw != 0:
        if first:
            lines.append(f"double e = {hexlit(mw)} * madet;")
            first = False
        else:
            lines.append(f"e = __builtin_fma({hexlit(mw)}, madet, e);")
    if first:
        lines.append("double e = 0.0;")
    return lines


def upper_index(i, j, n):
    """Position of (i, j), i <= j, in the row-major packed upper triangle."""
    return i * (2 * n - i + 1) // 2 + (j - i)


def split_groups(entries, cost, G):
    """Greedy longest-processing-time partition of entries into G groups."""
    groups = [[] for _ in range(G)]
    load = [0] * G
    for e in sorted(entries, key=lambda e: -cost[e]):
        g = min(range(G), key=lambda g: load[g])
        groups[g].append(e); load[g] += cost[e]
    return [sorted(g) for g in groups], load


def emit_act_t(d, n, NM, stiff, mass):
    """y += A x with the stiffness terms grouped by metric pair.

    A_ij = sum_mn G[mn] s_ij,mn + madet Mref_ij with s_ij,mn = sum_k kc[k]
    W[k][mn][i][j], kc[k] = cstiff kappa_k and G[mn] = |det J| grad l_m .
    grad l_n: only the d+1 values kc and the metric are live instead of the
    (d+1) x NM products P.  Where at most d+1 distinct coefficient vectors
    W[.][mn][i][j] occur (P1: one, the mean of kappa) their dot products
    with kc are formed once per cell.
    """
    nv = d + 1
    groups = {}
    for e, terms in stiff.items():
        byt = {}
        for (kk, t, w) in terms:
            byt.setdefault(t, {})[kk] = w
        groups[e] = [(t, tuple(byt[t].get(kk, Fraction(0)) for kk in range(nv))) for t in sorted(byt)]
    vecs = sorted({v for g in groups.values() for (_, v) in g})
    shared = len(vecs) <= nv

    def dot(v):
        expr = None
        for kk, w in enumerate(v):
            if w == 0:
                continue
            expr = f"{hexlit(w)} * kc[{kk}]" if expr is None else f"__builtin_fma({hexlit(w)}, kc[{kk}], {expr})"
        return expr

    out = ["  // y += A x for one cell, stiffness terms grouped by metric pair (kc = cstiff kappa, G = metric)",
           "  __device__ __forceinline__ static void act_t(const double* __restrict__ kc, const double* __restrict__ G, double madet, const double* __restrict__ x, double* __restrict__ y) {"]
    if shared:
        for q, v in enumerate(vecs):
            out.append(f"    const double q{q} = {dot(v)};")
    for i in range(n):
        for j in range(i, n):
            expr = None
            mw = mass[(i, j)]
            if mw != 0:
                expr = f"{hexlit(mw)} * madet"
            for (t, v) in groups[(i, j)]:
                s = f"q{vecs.index(v)}" if shared else f"({dot(v)})"
                expr = f"G[{t}] * {s}" if expr is None else f"__builtin_fma(G[{t}], {s}, {expr})"
            out.append("    {")
            out.append(f"      const double e = {expr if expr else '0.0'};")
            out.append(f"      y[{i}] = __builtin_fma(e, x[{j}], y[{i}]);" + (f" y[{j}] = __builtin_fma(e, x[{i}], y[{j}]);" if i != j else ""))
            out.append("    }")
    out.append("  }")
    return out


# Degree-3 rules on the reference simplex, as (weight, barycentric point)
# with the weights summing to 1 (the integral over the reference simplex is
# the weighted sum divided by d!): the tetrahedron's five-point rule (centroid
# weight -4/5, four points (1/2, 1/6, 1/6, 1/6) of weight 9/20) and the
# triangle's four-point rule (centroid -9/16, three points (3/5, 1/5, 1/5) of
# weight 25/48).  Both are checked below to integrate every monomial of
# degree <= 3 exactly.
def _perms(pt):
    return sorted(set(itertools.permutations(pt)))


QRULES = {
    3: [(Fraction(-4, 5), (Fraction(1, 4),) * 4)] +
       [(Fraction(9, 20), p) for p in _perms((Fraction(1, 2), Fraction(1, 6), Fraction(1, 6), Fraction(1, 6)))],
    2: [(Fraction(-9, 16), (Fraction(1, 3),) * 3)] +
       [(Fraction(25, 48), p) for p in _perms((Fraction(3, 5), Fraction(1, 5), Fraction(1, 5)))],
}


def gm_rule(d, s):
    """Grundmann-Moeller rule of degree 2s+1 on the d-simplex (rational
    points and weights, some negative): level i = 0..s contributes the
    points with barycentric coordinates (2 beta_j + 1) / (2s+1 + d - 2i),
    |beta| = s - i, with weight proportional to
    (-1)^i (2s+1 + d - 2i)^(2s+1) / (i! (2s+1 + d - i)!); the weights are
    normalised to sum to 1."""
    deg = 2 * s + 1
    rule = []
    for i in range(s + 1):
        w = Fraction((-1) ** i * (deg + d - 2 * i) ** deg, 2 ** (2 * s) * factorial(i) * factorial(deg + d - i))
        for beta in itertools.product(range(s - i + 1), repeat=d + 1):
            if sum(beta) == s - i:
                rule.append((w, tuple(Fraction(2 * b + 1, deg + d - 2 * i) for b in beta)))
    tot = sum(w for w, _ in rule)
    return [(w / tot, pt) for w, pt in rule]


def check_rule(d, rule, degree=3):
    nv = d + 1
    for tot in range(degree + 1):
        for a in itertools.product(range(tot + 1), repeat=nv):
            if sum(a) != tot:
                continue
            q = sum(w * poly_eval({a: Fraction(1)}, pt) for w, pt in rule)
            assert q == factorial(d) * integrate({a: Fraction(1)}, d), f"rule not exact for {a}"


def poly_eval(p, pt):
    s = Fraction(0)
    for a, c in p.items():
        t = c
        for x, e in zip(pt, a):
            t *= x ** e
        s += t
    return s


def emit_act_q(d, k):
    """y += A x for one cell with the stiffness part evaluated at the points
    of a rule exact for its integrand (P1 kappa times two gradients of
    degree k-1: degree 2k-1; the rules above for P2, the degree-5
    Grundmann-Moeller rule for P3), and the mass part from the exact
    reference mass matrix:

      y_i += sum_q (w_q / d!) kappa(q) sum_m d_m phi_i(q) sum_n G[mn] a_n(q)
             + madet sum_j Mref_ij x_j,   a_n(q) = sum_j d_n phi_j(q) x_j

    with kappa(q) = sum_k kc[k] l_k(q).  About 380 FMAs per P2 tetrahedron
    against 835 for act_t; the result equals the exact integral up to
    rounding."""
    assert k in (2, 3)
    nv = d + 1
    rule = QRULES[d] if k == 2 else gm_rule(d, 2)
    check_rule(d, rule, 2 * k - 1)
    B = basis(d, k)
    n = len(B)
    dB = [[poly_d(B[i], m) for m in range(nv)] for i in range(n)]
    pairs = metric_pairs(nv)
    gidx = {}
    for t, (m, q) in enumerate(pairs):
        gidx[(m, q)] = gidx[(q, m)] = t
    mass = {(i, j): integrate(poly_mul(B[i], B[j]), d) for i in range(n) for j in range(n)}
    out = [f"  // y += A x for one cell: stiffness at the points of an exact degree-{2 * k - 1} rule,",
           "  // mass from the exact reference mass matrix (kc = cstiff kappa, G = metric)",
           "  __device__ __forceinline__ static void act_q(const double* __restrict__ kc, const double* __restrict__ G, double madet, const double* __restrict__ x, double* __restrict__ y) {"]
    for i in range(n):
        expr = None
        for j in range(n):
            w = mass[(i, j)]
            if w == 0:
                continue
            expr = f"{hexlit(w)} * x[{j}]" if expr is None else f"__builtin_fma({hexlit(w)}, x[{j}], {expr})"
        out.append(f"    y[{i}] = __builtin_fma(madet, {expr}, y[{i}]);")
    for qi, (w, pt) in enumerate(rule):
        sc = w / factorial(d)
        out.append("    {")
        kexpr = None
        for kk in range(nv):
            cf = sc * pt[kk]
            kexpr = f"{hexlit(cf)} * kc[{kk}]" if kexpr is None else f"__builtin_fma({hexlit(cf)}, kc[{kk}], {kexpr})"
        out.append(f"      const double kq = {kexpr};")
        for m in range(nv):
            expr = None
            for j in range(n):
                cf = poly_eval(dB[j][m], pt)
                if cf == 0:
                    continue
                expr = f"{hexlit(cf)} * x[{j}]" if expr is None else f"__builtin_fma({hexlit(cf)}, x[{j}], {expr})"
            out.append(f"      const double a{m} = {expr if expr else '0.0'};")
        for m in range(nv):
            expr = None
            for q in range(nv):
                g = f"G[{gidx[(m, q)]}]"
                expr = f"{g} * a{q}" if expr is None else f"__builtin_fma({g}, a{q}, {expr})"
            out.append(f"      const double c{m} = kq * ({expr});")
        for i in range(n):
            expr = f"y[{i}]"
            for m in range(nv):
                cf = poly_eval(dB[i][m], pt)
                if cf == 0:
                    continue
                expr = f"__builtin_fma({hexlit(cf)}, c{m}, {expr})"
            if expr != f"y[{i}]":
                out.append(f"      y[{i}] = {expr};")
        out.append("    }")
    out.append("  }")
    return out


def emit(d, k, G):
    n, pairs, stiff, mass, src = tables(d, k)
    nv = d + 1
    NM = len(pairs)
    NE = n * (n + 1) // 2
    name = f"Tab{d}{k}"
    out = []
    out.append(f"struct {name} {{")
    out.append(f"  static constexpr int DIM = {d}, DEG = {k}, NLOC = {n}, NV = {nv}, NM = {NM}, NE = {NE}, NG = {G};")
    nterms = sum(len(v) for v in stiff.values()) + sum(1 for v in mass.values() if v != 0)
    out.append(f"  static constexpr int TERMS = {nterms};")
    entries = sorted(stiff)
    cost = {e: len(stiff[e]) + (1 if mass[e] != 0 else 0) for e in entries}
    groups, load = split_groups(entries, cost, G)
    out.append(f"  // entry-group loads (terms): {load}")
    for g, grp in enumerate(groups):
        out.append(f"  // entries of group {g}, written to the packed upper triangle E[NE]")
        out.append(f"  __device__ __forceinline__ static void mat_group{g}(const double* __restrict__ P, double madet, double* __restrict__ E) {{")
        for (i, j) in grp:
            out.append("    {")
            for l in entry_expr(i, j, NM, stiff, mass):
                out.append("      " + l)
            out.append(f"      E[{upper_index(i, j, n)}] = e;")
            out.append("    }")
        out.append("  }")
    # the same entry groups from kc[k] = cstiff kappa_k and the metric G[mn]
    # (terms grouped by metric pair: d+1 + NM values live instead of P)
    nv_ = d + 1
    for g, grp in enumerate(groups):
        out.append(f"  // entries of group {g} from kc and the metric, written to E[NE]")
        out.append(f"  __device__ __forceinline__ static void mat_group_t{g}(const double* __restrict__ kc, const double* __restrict__ G, double madet, double* __restrict__ E) {{")
        for (i, j) in grp:
            byt = {}
            for (kk, t, w) in stiff[(i, j)]:
                byt.setdefault(t, {})[kk] = w
            expr = None
            mw = mass[(i, j)]
            if mw != 0:
                expr = f"{hexlit(mw)} * madet"
            for t in sorted(byt):
                dot = None
                for kk in range(nv_):
                    w = byt[t].get(kk, Fraction(0))
                    if w == 0:
                        continue
                    dot = f"{hexlit(w)} * kc[{kk}]" if dot is None else f"__builtin_fma({hexlit(w)}, kc[{kk}], {dot})"
                expr = f"G[{t}] * ({dot})" if expr is None else f"__builtin_fma(G[{t}], ({dot}), {expr})"
            out.append(f"    E[{upper_index(i, j, n)}] = {expr if expr else '0.0'};")
        out.append("  }")
    # entry group g by number (a switch: uniform when g is the same on a wave)
    out.append("  __device__ __forceinline__ static void mat_group_n(int g, const double* __restrict__ P, double madet, double* __restrict__ E) {")
    out.append("    switch (g) {")
    for g in range(G):
        out.append(f"    {'default' if g == G - 1 else f'case {g}'}: mat_group{g}(P, madet, E); break;")
    out.append("    }")
    out.append("  }")
    out.append("  __device__ __forceinline__ static void mat_group_tn(int g, const double* __restrict__ kc, const double* __restrict__ G, double madet, double* __restrict__ E) {")
    out.append("    switch (g) {")
    for g in range(G):
        out.append(f"    {'default' if g == G - 1 else f'case {g}'}: mat_group_t{g}(kc, G, madet, E); break;")
    out.append("    }")
    out.append("  }")
    out.append("  // upper triangle, row-major (i<=j), Eu[NE]")
    out.append("  __device__ __forceinline__ static void mat_upper(const double* __restrict__ P, double madet, double* __restrict__ Eu) {")
    u = 0
    for i in range(n):
        for j in range(i, n):
            out.append("    {")
            for l in entry_expr(i, j, NM, stiff, mass):
                out.append("      " + l)
            out.append(f"      Eu[{u}] = e;")
            out.append("    }")
            u += 1
    out.append("  }")
    out.append("  // y += A x for one cell, entries consumed as soon as they are formed")
    out.append("  __device__ __forceinline__ static void act(const double* __restrict__ P, double madet, const double* __restrict__ x, double* __restrict__ y) {")
    for i in range(n):
        for j in range(i, n):
            out.append("    {")
            for l in entry_expr(i, j, NM, stiff, mass):
                out.append("      " + l)
            out.append(f"      y[{i}] = __builtin_fma(e, x[{j}], y[{i}]);" + (f" y[{j}] = __builtin_fma(e, x[{i}], y[{j}]);" if i != j else ""))
            out.append("    }")
    out.append("  }")
    out.extend(emit_act_t(d, n, NM, stiff, mass))
    if k >= 2:
        out.extend(emit_act_q(d, k))
    out.append("  // b_i = adet * sum_k f_k int l_k phi_i")
    out.append("  __device__ __forceinline__ static void vec(const double* __restrict__ f, double adet, double* __restrict__ b) {")
    for i in range(n):
        terms = [(kk, src[i][kk]) for kk in range(nv) if src[i][kk] != 0]
        expr = None
        for kk, w in terms:
            expr = f"{hexlit(w)} * f[{kk}]" if expr is None else f"__builtin_fma({hexlit(w)}, f[{kk}], {expr})"
        out.append(f"    b[{i}] = adet * ({expr if expr else '0.0'});")
    out.append("  }")
    out.append("};")
    return "\n".join(out), nterms


# Entry groups per element tensor (one lane of a cell evaluates NG/LPC of
# them).  P1 tensors are one group; P3 tetrahedra are split into 8 so that
# eight lanes share a cell's 210 entries.
GROUPS = {(2, 1): 1, (3, 1): 1, (3, 3): 8}


def main(path):
    parts = ["// Generated by gen_tables.py -- exact reference integrals of Lagrange P1-P3",
             "// bases (see the generator's docstring for the formulas).  Do not edit.",
             "#pragma once", "namespace femtab {"]
    summary = []
    for d in (2, 3):
        for k in (1, 2, 3):
            G = GROUPS.get((d, k), 4)
            code, nt = emit(d, k, G)
            parts.append(code)
            summary.append((d, k, nt))
    parts.append("}  // namespace femtab")
    txt = "\n".join(parts) + "\n"
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(txt)
    os.replace(tmp, path)
    return summary


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "fem_tables.h")
    for d, k, nt in main(out):
        print(f"dim {d} degree {k}: {nt} terms")
