"""Exact (rational) element tensors for pinning the oracle.

Independent of the oracle's construction: the nodal Lagrange basis is obtained
by inverting, in exact rational arithmetic, the Vandermonde matrix of the
monomials x^a (|a| <= k, reference coordinates) at the local node positions
given by ``fem_inputs.local_node_barycentrics``; integrals over the reference
simplex use the Dirichlet formula  int x^a dx = a! / (|a| + d)!  ; the physical
tensors follow from the affine map exactly (Fractions).  No quadrature and no
closed-form basis expressions are involved.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np

from fem_inputs import local_node_barycentrics


def _monomials(dim, k):
    return [a for a in itertools.product(range(k + 1), repeat=dim) if sum(a) <= k]


def _solve_exact(A, B):
    """Solve A X = B over Fractions by Gauss-Jordan elimination."""
    n = len(A)
    M = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


def poly_mul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            e = tuple(x + y for x, y in zip(a, b))
            out[e] = out.get(e, 0) + ca * cb
    return out


def poly_diff(p, var):
    out = {}
    for a, c in p.items():
        if a[var]:
            e = list(a); e[var] -= 1
            out[tuple(e)] = out.get(tuple(e), 0) + c * a[var]
    return out


def poly_int_ref(p, dim):
    """Exact integral over the reference simplex {x >= 0, sum x <= 1}."""
    s = Fraction(0)
    for a, c in p.items():
        num = 1
        for x in a:
            num *= factorial(x)
        s += c * Fraction(num, factorial(sum(a) + dim))
    return s


@lru_cache(maxsize=None)
def nodal_basis(dim, k):
    """Basis polynomials (dict exponent->Fraction) in reference coordinates."""
    W = local_node_barycentrics(dim, k)            # [nloc][dim+1], sums to k
    mons = _monomials(dim, k)
    nloc = W.shape[0]
    assert len(mons) == nloc
    pts = [[Fraction(int(W[i, m + 1]), k) for m in range(dim)] for i in range(nloc)]
    V = []
    for x in pts:
        row = []
        for a in mons:
            v = Fraction(1)
            for xi, ai in zip(x, a):
                v *= xi ** ai
            row.append(v)
        V.append(row)
    # phi_i(x) = sum_a C[a][i] x^a with V C = I
    I = [[Fraction(int(i == j)) for j in range(nloc)] for i in range(nloc)]
    Cm = _solve_exact(V, I)
    return tuple({a: Cm[r][i] for r, a in enumerate(mons) if Cm[r][i] != 0} for i in range(nloc))


def _lam_poly(dim, m):
    if m == 0:
        p = {tuple([0] * dim): Fraction(1)}
        for a in range(dim):
            e = [0] * dim; e[a] = 1
            p[tuple(e)] = Fraction(-1)
        return p
    e = [0] * dim; e[m - 1] = 1
    return {tuple(e): Fraction(1)}


@lru_cache(maxsize=None)
def reference_tensors(dim, k):
    """M[i][j] = int phi_i phi_j,  S[m][a][b][i][j] = int lam_m d_a phi_i d_b phi_j."""
    B = nodal_basis(dim, k)
    n = len(B)
    M = [[poly_int_ref(poly_mul(B[i], B[j]), dim) for j in range(n)] for i in range(n)]
    dB = [[poly_diff(B[i], a) for a in range(dim)] for i in range(n)]
    S = [[[[[poly_int_ref(poly_mul(_lam_poly(dim, m), poly_mul(dB[i][a], dB[j][b])), dim)
             for j in range(n)] for i in range(n)] for b in range(dim)] for a in range(dim)]
         for m in range(dim + 1)]
    F = [[poly_int_ref(poly_mul(_lam_poly(dim, m), B[i]), dim) for m in range(dim + 1)]
         for i in range(n)]
    return M, S, F


def _inv_exact(J):
    d = len(J)
    I = [[Fraction(int(i == j)) for j in range(d)] for i in range(d)]
    return _solve_exact(J, I)


def _det_exact(J):
    if len(J) == 2:
        return J[0][0] * J[1][1] - J[0][1] * J[1][0]
    a, b, c = J[0]; d, e, f = J[1]; g, h, i = J[2]
    return a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g)


def element_matrix_exact(dim, k, xv, kv, cstiff=1, cmass=1):
    """Exact A[i][j] for rational vertex coordinates xv [dim+1][dim] and P1 kappa."""
    xv = [[Fraction(v) for v in row] for row in xv]
    kv = [Fraction(v) for v in kv]
    J = [[xv[c + 1][r] - xv[0][r] for c in range(dim)] for r in range(dim)]
    det = _det_exact(J)
    Ji = _inv_exact(J)
    adet = abs(det)
    # K_ab = |det| (J^-1 J^-T)_ab
    K = [[adet * sum(Ji[a][r] * Ji[b][r] for r in range(dim)) for b in range(dim)]
         for a in range(dim)]
    M, S, _ = reference_tensors(dim, k)
    n = len(M)
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            s = Fraction(0)
            if cstiff:
                for m in range(dim + 1):
                    for a in range(dim):
                        for b in range(dim):
                            s += kv[m] * K[a][b] * S[m][a][b][i][j]
            A[i][j] = cstiff * s + cmass * adet * M[i][j]
    return A


def element_vector_exact(dim, k, xv, fv):
    xv = [[Fraction(v) for v in row] for row in xv]
    fv = [Fraction(v) for v in fv]
    J = [[xv[c + 1][r] - xv[0][r] for c in range(dim)] for r in range(dim)]
    adet = abs(_det_exact(J))
    _, _, F = reference_tensors(dim, k)
    return [adet * sum(fv[m] * F[i][m] for m in range(dim + 1)) for i in range(len(F))]


def to_float(A):
    return np.array([[float(v) for v in row] for row in A]) if isinstance(A[0], list) \
        else np.array([float(v) for v in A])
