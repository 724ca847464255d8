"""CPU oracle for the cell-loop assembler -- TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded FP64 C implementation (``oracle.c``) of what
the parallel loop computes: the global assembly sums of the Helmholtz-type
bilinear form, the source linear form and the matrix-free action, with its own
sparsity; and the nonlinear residual kappa grad(u).grad(v) + u^3 v - f v with
its vector-Jacobian products (the adjoint assembly); and vector Lagrange
linear elasticity 2 mu eps(u):eps(v) + lam div(u) div(v) on per-cell
coordinates (the precision benchmark); and per-cell contributions to Global
reductions (cell energies x_K^T A_K x_K, integrals of f); the monolithic
matrix of a form on a mixed space; exterior facet integrals of g v.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product library never does.

Every function here follows the paper's definition of a parallel loop over
cells with data gathered through Maps and INC contributions summed
(PyOP2 section: "Parloops and kernels", "Access descriptors",
"Matrix arguments").

Parity unpinned: none of the functions below lacks a pin; the pins live in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-std=c99", "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p; I = C.c_int; L64 = C.c_int64; D = C.c_double
        L.oracle_gauss_jacobi.argtypes = [I, I, P, P]; L.oracle_gauss_jacobi.restype = I
        L.oracle_simplex_rule.argtypes = [I, I, P, P]; L.oracle_simplex_rule.restype = I
        L.oracle_nloc.argtypes = [I, I]; L.oracle_nloc.restype = I
        L.oracle_basis.argtypes = [I, I, P, P, P]; L.oracle_basis.restype = None
        L.oracle_element_matrix.argtypes = [I, I, P, P, D, D, P, P]; L.oracle_element_matrix.restype = I
        L.oracle_element_vector.argtypes = [I, I, P, P, P, P]; L.oracle_element_vector.restype = I
        L.oracle_sparsity.argtypes = [L64, I, P, I, P, L64, L64, P, P]; L.oracle_sparsity.restype = L64
        L.oracle_assemble_mat.argtypes = [I, I, L64, P, P, P, P, D, D, P, P, L64, P, P, P]
        L.oracle_assemble_mat.restype = I
        L.oracle_assemble_vec.argtypes = [I, I, L64, P, P, P, P, L64, P, P]
        L.oracle_assemble_vec.restype = I
        L.oracle_apply_action.argtypes = [I, I, L64, P, P, P, P, D, D, P, L64, P, P]
        L.oracle_apply_action.restype = I
        L.oracle_mat_rows.argtypes = [I, I, L64, P, P, P, P, D, D, L64, L64, P, L64, P, P, P, P, P]
        L.oracle_mat_rows.restype = L64
        L.oracle_vec_rows.argtypes = [I, I, I, L64, P, P, P, P, D, D, P, L64, L64, P, P, P]
        L.oracle_vec_rows.restype = I
        L.oracle_nl_element.argtypes = [I, P, P, P, P, P, P, P, P, P, P, P]
        L.oracle_nl_element.restype = I
        L.oracle_nl_residual.argtypes = [I, L64, P, P, P, L64, P, P, P, P, P]
        L.oracle_nl_residual.restype = I
        L.oracle_nl_adjoint.argtypes = [I, L64, P, P, P, L64, P, P, P, P, P, P, P]
        L.oracle_nl_adjoint.restype = I
        L.oracle_facet_vec.argtypes = [I, I, L64, P, P, P, P, L64, P, P]
        L.oracle_facet_vec.restype = I
        L.oracle_mixed_mat.argtypes = [I, I, I, L64, P, P, P, L64, P, P, P, P, P, P, P]
        L.oracle_mixed_mat.restype = I
        L.oracle_cell_values.argtypes = [I, I, I, L64, P, P, P, P, D, D, P, P, P, P, P]
        L.oracle_cell_values.restype = I
        L.oracle_elasticity_element.argtypes = [I, I, P, P, P, P, P]
        L.oracle_elasticity_element.restype = I
        L.oracle_elasticity_mat.argtypes = [I, I, L64, P, P, P, P, P, P, P, L64, P, P]
        L.oracle_elasticity_mat.restype = I
        L.oracle_elasticity_rows.argtypes = [I, I, L64, P, P, P, P, P, L64, L64, P, L64, P, P, P, P]
        L.oracle_elasticity_rows.restype = L64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# Form coefficients: (cstiff, cmass) of  cstiff*kappa grad u.grad v + cmass*u v
FORMS = {"helmholtz": (1.0, 1.0), "laplace": (1.0, 0.0), "mass": (0.0, 1.0)}


def gauss_jacobi(n: int, alpha: int):
    t = np.zeros(n); w = np.zeros(n)
    rc = lib().oracle_gauss_jacobi(n, alpha, _p(t), _p(w))
    if rc:
        raise RuntimeError(f"gauss_jacobi failed ({rc})")
    return t, w


def simplex_rule(dim: int, q: int):
    pts = np.zeros((q ** dim, dim)); wts = np.zeros(q ** dim)
    n = lib().oracle_simplex_rule(dim, q, _p(pts), _p(wts))
    if n <= 0:
        raise RuntimeError("simplex_rule failed")
    return pts[:n], wts[:n]


def nloc(dim: int, degree: int) -> int:
    return lib().oracle_nloc(dim, degree)


def basis(dim: int, degree: int, lam):
    lam = _c(lam, np.float64)
    n = nloc(dim, degree)
    phi = np.zeros(n); dphi = np.zeros((n, dim + 1))
    lib().oracle_basis(dim, degree, _p(lam), _p(phi), _p(dphi))
    return phi, dphi


def element_matrix(dim, degree, xv, kv, form="helmholtz"):
    cs, cm = FORMS[form]
    xv = _c(xv, np.float64); kv = _c(kv, np.float64)
    n = nloc(dim, degree); A = np.zeros((n, n))
    if lib().oracle_element_matrix(dim, degree, _p(xv), _p(kv), cs, cm, _p(A), None):
        raise RuntimeError("element_matrix failed")
    return A


def element_vector(dim, degree, xv, fv):
    xv = _c(xv, np.float64); fv = _c(fv, np.float64)
    n = nloc(dim, degree); b = np.zeros(n)
    if lib().oracle_element_vector(dim, degree, _p(xv), _p(fv), _p(b), None):
        raise RuntimeError("element_vector failed")
    return b


def sparsity(rmap, nrows, cmap=None, ncols=None):
    """Oracle CSR pattern (row_ptr int64, col_idx int32)."""
    rmap = _c(rmap, np.int32)
    cmap = rmap if cmap is None else _c(cmap, np.int32)
    ncols = nrows if ncols is None else ncols
    ncells = rmap.shape[0]
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    L = lib()
    nnz = L.oracle_sparsity(ncells, rmap.shape[1], _p(rmap), cmap.shape[1], _p(cmap),
                            nrows, ncols, _p(row_ptr), None)
    if nnz < 0:
        raise ValueError(f"oracle sparsity failed ({nnz})")
    col_idx = np.zeros(max(nnz, 1), dtype=np.int32)
    nnz2 = L.oracle_sparsity(ncells, rmap.shape[1], _p(rmap), cmap.shape[1], _p(cmap),
                             nrows, ncols, _p(row_ptr), _p(col_idx))
    assert nnz2 == nnz
    return row_ptr, col_idx[:nnz]


def assemble_mat(dim, degree, cell_vertex, coords, cell_node, kappa, row_ptr, col_idx,
                 form="helmholtz", contrib_scale=False):
    """Assembled CSR values and the term-level rounding scale of each entry
    (sum over cells and quadrature points of |weight * integrand term|); with
    contrib_scale also the contribution-level scale (sum over cells of
    |element entry|), which is never larger."""
    cs, cm = FORMS[form]
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    k = _c(kappa, np.float64); rp = _c(row_ptr, np.int64); ci = _c(col_idx, np.int32)
    nrows = rp.size - 1
    vals = np.zeros(max(int(rp[-1]), 1)); absv = np.zeros_like(vals)
    cabs = np.zeros_like(vals) if contrib_scale else None
    rc = lib().oracle_assemble_mat(dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(k),
                                   cs, cm, _p(rp), _p(ci), nrows, _p(vals), _p(absv),
                                   _p(cabs) if contrib_scale else None)
    if rc:
        raise RuntimeError(f"oracle assemble_mat failed ({rc})")
    nnz = int(rp[-1])
    if contrib_scale:
        return vals[:nnz], absv[:nnz], cabs[:nnz]
    return vals[:nnz], absv[:nnz]


def assemble_vec(dim, degree, cell_vertex, coords, cell_node, f, nrows):
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    fv = _c(f, np.float64)
    b = np.zeros(nrows); ab = np.zeros(nrows)
    rc = lib().oracle_assemble_vec(dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(fv),
                                   nrows, _p(b), _p(ab))
    if rc:
        raise RuntimeError(f"oracle assemble_vec failed ({rc})")
    return b, ab


def apply_action(dim, degree, cell_vertex, coords, cell_node, kappa, x, nrows,
                 form="helmholtz"):
    cs, cm = FORMS[form]
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    k = _c(kappa, np.float64); xx = _c(x, np.float64)
    y = np.zeros(nrows); ay = np.zeros(nrows)
    rc = lib().oracle_apply_action(dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(k),
                                   cs, cm, _p(xx), nrows, _p(y), _p(ay))
    if rc:
        raise RuntimeError(f"oracle apply_action failed ({rc})")
    return y, ay


def mat_rows(dim, degree, cell_vertex, coords, cell_node, kappa, nrows, rows,
             form="helmholtz", contrib_scale=False):
    """Assembled rows ``rows`` (distinct): list of (cols, vals, abs) per row,
    abs the term-level scale; with contrib_scale (cols, vals, abs, cabs), cabs
    the contribution-level scale (sum over cells of |element entry|)."""
    cs, cm = FORMS[form]
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    k = _c(kappa, np.float64); rows = _c(rows, np.int64)
    cap = rows.size * 1024
    ptr = np.zeros(rows.size + 1, dtype=np.int64)
    cols = np.zeros(cap, dtype=np.int32); vals = np.zeros(cap); absv = np.zeros(cap)
    cabs = np.zeros(cap)
    tot = lib().oracle_mat_rows(dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(k), cs, cm,
                                nrows, rows.size, _p(rows), cap, _p(ptr), _p(cols), _p(vals),
                                _p(absv), _p(cabs))
    if tot < 0:
        raise RuntimeError(f"oracle mat_rows failed ({tot})")
    out = []
    for s in range(rows.size):
        sl = slice(ptr[s], ptr[s + 1])
        t = (cols[sl].copy(), vals[sl].copy(), absv[sl].copy())
        out.append(t + (cabs[sl].copy(),) if contrib_scale else t)
    return out


def vec_rows(dim, degree, cell_vertex, coords, cell_node, f, nrows, rows):
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    fv = _c(f, np.float64); rows = _c(rows, np.int64)
    out = np.zeros(rows.size); absv = np.zeros(rows.size)
    rc = lib().oracle_vec_rows(0, dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(fv),
                               0.0, 0.0, None, nrows, rows.size, _p(rows), _p(out), _p(absv))
    if rc:
        raise RuntimeError("oracle vec_rows failed")
    return out, absv


def action_rows(dim, degree, cell_vertex, coords, cell_node, kappa, x, nrows, rows,
                form="helmholtz"):
    cs, cm = FORMS[form]
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    k = _c(kappa, np.float64); xx = _c(x, np.float64); rows = _c(rows, np.int64)
    out = np.zeros(rows.size); absv = np.zeros(rows.size)
    rc = lib().oracle_vec_rows(1, dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(k),
                               cs, cm, _p(xx), nrows, rows.size, _p(rows), _p(out), _p(absv))
    if rc:
        raise RuntimeError("oracle action_rows failed")
    return out, absv


def nl_element(dim, xv, uv, kv, fv=None, lv=None):
    """Element residual F, adjoint products gu, gk (P1) and their magnitude scales."""
    n = dim + 1
    xv = _c(xv, np.float64); uv = _c(uv, np.float64); kv = _c(kv, np.float64)
    fv = None if fv is None else _c(fv, np.float64); lv = None if lv is None else _c(lv, np.float64)
    out = [np.zeros(n) for _ in range(6)]
    rc = lib().oracle_nl_element(dim, _p(xv), _p(uv), _p(kv), None if fv is None else _p(fv),
                                 None if lv is None else _p(lv), *[_p(o) for o in out])
    if rc:
        raise RuntimeError(f"oracle nl_element failed ({rc})")
    return out


def nl_residual(dim, cell_vertex, coords, cell_node, u, kappa, f, nnodes):
    """F_i = integral of kappa grad(u).grad(phi_i) + u^3 phi_i - f phi_i (P1 fields on the nodes)."""
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    u = _c(u, np.float64); k = _c(kappa, np.float64); f = _c(f, np.float64)
    F = np.zeros(nnodes); Fa = np.zeros(nnodes)
    rc = lib().oracle_nl_residual(dim, cv.shape[0], _p(cv), _p(X), _p(cn), nnodes, _p(u), _p(k), _p(f),
                                  _p(F), _p(Fa))
    if rc:
        raise RuntimeError(f"oracle nl_residual failed ({rc})")
    return F, Fa


def nl_adjoint(dim, cell_vertex, coords, cell_node, u, kappa, lam, nnodes):
    """lambda^T dF/du and lambda^T dF/dkappa with their magnitude scales."""
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    u = _c(u, np.float64); k = _c(kappa, np.float64); lam = _c(lam, np.float64)
    gu = np.zeros(nnodes); gua = np.zeros(nnodes); gk = np.zeros(nnodes); gka = np.zeros(nnodes)
    rc = lib().oracle_nl_adjoint(dim, cv.shape[0], _p(cv), _p(X), _p(cn), nnodes, _p(u), _p(k), _p(lam),
                                 _p(gu), _p(gua), _p(gk), _p(gka))
    if rc:
        raise RuntimeError(f"oracle nl_adjoint failed ({rc})")
    return gu, gua, gk, gka


def vector_map(cell_node, dim):
    """Cell-to-DOF Map of the vector space: DOF dim*node + a, local (i, a) at i*dim + a."""
    cn = np.asarray(cell_node, dtype=np.int64)
    return np.ascontiguousarray((dim * cn[:, :, None] + np.arange(dim)).reshape(cn.shape[0], -1)
                                .astype(np.int32))


def elasticity_element(dim, degree, xv, muv, lav):
    """Element matrix [dim*n][dim*n] (row (i, a) = i*dim + a) and its magnitude scale."""
    xv = _c(xv, np.float64); muv = _c(muv, np.float64); lav = _c(lav, np.float64)
    N = dim * nloc(dim, degree)
    A = np.zeros((N, N)); Aa = np.zeros((N, N))
    if lib().oracle_elasticity_element(dim, degree, _p(xv), _p(muv), _p(lav), _p(A), _p(Aa)):
        raise RuntimeError("oracle elasticity_element failed")
    return A, Aa


def elasticity_mat(dim, degree, cell_vertex, xdg, cell_node, mu, lam, row_ptr, col_idx):
    """Global elasticity matrix on the vector CSR (row_ptr, col_idx); xdg [C][dim+1][dim]."""
    cv = _c(cell_vertex, np.int32); X = _c(xdg, np.float64); cn = _c(cell_node, np.int32)
    m = _c(mu, np.float64); la = _c(lam, np.float64); rp = _c(row_ptr, np.int64); ci = _c(col_idx, np.int32)
    nrows = rp.size - 1
    vals = np.zeros(max(int(rp[-1]), 1)); absv = np.zeros_like(vals)
    rc = lib().oracle_elasticity_mat(dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(m), _p(la),
                                     _p(rp), _p(ci), nrows, _p(vals), _p(absv))
    if rc:
        raise RuntimeError(f"oracle elasticity_mat failed ({rc})")
    nnz = int(rp[-1])
    return vals[:nnz], absv[:nnz]


def elasticity_rows(dim, degree, cell_vertex, xdg, cell_node, mu, lam, nrows, rows):
    """Assembled vector rows ``rows`` (distinct): list of (cols, vals, abs) per row."""
    cv = _c(cell_vertex, np.int32); X = _c(xdg, np.float64); cn = _c(cell_node, np.int32)
    m = _c(mu, np.float64); la = _c(lam, np.float64); rows = _c(rows, np.int64)
    cap = rows.size * 1024
    ptr = np.zeros(rows.size + 1, dtype=np.int64)
    cols = np.zeros(cap, dtype=np.int32); vals = np.zeros(cap); absv = np.zeros(cap)
    tot = lib().oracle_elasticity_rows(dim, degree, cv.shape[0], _p(cv), _p(X), _p(cn), _p(m), _p(la),
                                       nrows, rows.size, _p(rows), cap, _p(ptr), _p(cols), _p(vals),
                                       _p(absv))
    if tot < 0:
        raise RuntimeError(f"oracle elasticity_rows failed ({tot})")
    return [(cols[ptr[s]:ptr[s + 1]].copy(), vals[ptr[s]:ptr[s + 1]].copy(),
             absv[ptr[s]:ptr[s + 1]].copy()) for s in range(rows.size)]


def cell_values(kind, dim, degree, cell_vertex, coords, cell_node, field, x=None, form="helmholtz"):
    """Per-cell Global contributions: kind "energy" (x_K^T A_K x_K, field =
    kappa) or "integral" (integral of f over K, field = f).  Returns (q, q_abs,
    sum in cell order, sum of magnitudes)."""
    cs, cm = FORMS[form]
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    fld = _c(field, np.float64)
    xx = _c(x, np.float64) if x is not None else None
    C_ = cv.shape[0]
    q = np.zeros(C_); qa = np.zeros(C_); s_ = np.zeros(1); sa = np.zeros(1)
    rc = lib().oracle_cell_values(0 if kind == "energy" else 1, dim, degree, C_, _p(cv), _p(X), _p(cn), _p(fld),
                                  cs, cm, None if xx is None else _p(xx), _p(q), _p(qa), _p(s_), _p(sa))
    if rc:
        raise RuntimeError(f"oracle cell_values failed ({rc})")
    return q, qa, float(s_[0]), float(sa[0])


def apply_dirichlet(row_ptr, col_idx, values, b, mask, g=None, diag=1.0):
    """Symmetric Dirichlet rows and columns of an assembled system (the
    boundary condition applied at assembly in the paper's Firedrake example):
    for every DOF r with mask[r], b[i] -= A[i][r] g[r] on the free rows i
    (lifting), then row r and column r become zero except A[r][r] = diag, and
    b[r] = diag g[r].  Plain loops over the CSR, rows in order; returns new
    arrays (values, b) and the magnitude scale of each b entry."""
    vals = np.array(values, dtype=np.float64, copy=True)
    bb = np.array(b, dtype=np.float64, copy=True)
    babs = np.abs(bb)
    gg = np.zeros(len(bb)) if g is None else np.asarray(g, dtype=np.float64)
    for r in range(len(row_ptr) - 1):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            c = col_idx[k]
            if mask[r]:
                continue
            if mask[c]:
                bb[r] -= vals[k] * gg[c]
                babs[r] += abs(vals[k] * gg[c])
                vals[k] = 0.0
        if mask[r]:
            for k in range(row_ptr[r], row_ptr[r + 1]):
                vals[k] = diag if col_idx[k] == r else 0.0
            bb[r] = diag * gg[r]
            babs[r] = abs(bb[r])
    return vals, bb, babs


def mixed_mat(dim, degree, cell_vertex, coords, cell_node, nnodes, blocks):
    """Monolithic matrix of a form on V^nf: blocks[a][b] = (cstiff, cmass, kappa or None)
    for test field a and trial field b.  Returns (row_ptr, col_idx, values, abs)
    over the DOFs f*nnodes + node, with the oracle's own sparsity."""
    nf = len(blocks)
    cv = _c(cell_vertex, np.int32); X = _c(coords, np.float64); cn = _c(cell_node, np.int32)
    n = cn.shape[1]
    mixed_map = np.concatenate([cn + f * nnodes for f in range(nf)], axis=1).astype(np.int32)
    rp, ci = sparsity(mixed_map, nf * nnodes)
    cs = np.array([blocks[a][b][0] for a in range(nf) for b in range(nf)], dtype=np.float64)
    cm = np.array([blocks[a][b][1] for a in range(nf) for b in range(nf)], dtype=np.float64)
    kaps = [None if blocks[a][b][2] is None else _c(blocks[a][b][2], np.float64)
            for a in range(nf) for b in range(nf)]
    kp = (C.c_void_p * (nf * nf))(*[None if k is None else k.ctypes.data for k in kaps])
    vals = np.zeros(max(int(rp[-1]), 1)); absv = np.zeros_like(vals)
    rc = lib().oracle_mixed_mat(dim, degree, nf, cv.shape[0], _p(cv), _p(X), _p(cn), nnodes,
                                C.cast(kp, C.c_void_p), _p(cs), _p(cm), _p(rp), _p(ci), _p(vals), _p(absv))
    if rc:
        raise RuntimeError(f"oracle mixed_mat failed ({rc})")
    nnz = int(rp[-1])
    return rp, ci, vals[:nnz], absv[:nnz]


def facet_vec(dim, degree, facet_vertex, coords, facet_node, g, nrows):
    """b_i = sum over the given facets of the integral of g v_i ds (P1 g)."""
    fv = _c(facet_vertex, np.int32); X = _c(coords, np.float64); fn = _c(facet_node, np.int32)
    gg = _c(g, np.float64)
    b = np.zeros(nrows); ab = np.zeros(nrows)
    rc = lib().oracle_facet_vec(dim, degree, fv.shape[0], _p(fv), _p(X), _p(fn), _p(gg), nrows, _p(b), _p(ab))
    if rc:
        raise RuntimeError(f"oracle facet_vec failed ({rc})")
    return b, ab
