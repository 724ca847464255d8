"""Pins of the oracle's nonlinear residual and its vector-Jacobian products.

F_i(u, kappa) = integral of kappa grad(u).grad(phi_i) + u^3 phi_i - f phi_i
(P1 fields u, kappa, f on the nodes), and for a P1 field lambda
  gu_j = integral of kappa grad(phi_j).grad(lambda) + 3 u^2 phi_j lambda,
  gk_k = integral of phi_k grad(u).grad(lambda).
The pins do not use the oracle's quadrature: exact rational integrals of
barycentric monomials, central finite differences of the residual itself, and
textbook integrals of polynomials over the unit square.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import fem_inputs as fi
import oracle


def _bary_integral(a, vol, d):
    """Exact integral over a simplex of volume vol of prod lambda_m^a_m."""
    num = 1
    for x in a:
        num *= factorial(x)
    return vol * Fraction(factorial(d) * num, factorial(sum(a) + d))


def _exact_element(xv, uv, kv, fv, lv):
    d = len(xv) - 1
    X = [[Fraction(c) for c in p] for p in xv]
    J = [[X[c + 1][r] - X[0][r] for c in range(d)] for r in range(d)]
    if d == 2:
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0]
        Jinv = [[J[1][1] / det, -J[0][1] / det], [-J[1][0] / det, J[0][0] / det]]
    else:
        (a, b, c), (e, f, g), (h, i, k) = J
        det = a * (f * k - g * i) - b * (e * k - g * h) + c * (e * i - f * h)
        Jinv = [[(f * k - g * i) / det, (c * i - b * k) / det, (b * g - c * f) / det],
                [(g * h - e * k) / det, (a * k - c * h) / det, (c * e - a * g) / det],
                [(e * i - f * h) / det, (b * h - a * i) / det, (a * f - b * e) / det]]
    vol = abs(det) / factorial(d)
    grad = [[-sum(Jinv[m][r] for m in range(d)) for r in range(d)]] + [Jinv[m] for m in range(d)]
    n = d + 1
    u = [Fraction(x) for x in uv]; kap = [Fraction(x) for x in kv]
    f = [Fraction(x) for x in fv]; lam = [Fraction(x) for x in lv]
    dot = lambda p, q: sum(p[r] * q[r] for r in range(d))
    gu_ = [sum(u[m] * grad[m][r] for m in range(n)) for r in range(d)]
    gl_ = [sum(lam[m] * grad[m][r] for m in range(n)) for r in range(d)]
    kint = sum(kap) * vol / n                      # integral of kappa
    unit = lambda *idx: tuple(sum(1 for t in idx if t == m) for m in range(n))
    F, GU, GK = [], [], []
    for i in range(n):
        cub = sum(u[m] * u[p] * u[q] * _bary_integral(unit(m, p, q, i), vol, d)
                  for m in range(n) for p in range(n) for q in range(n))
        src = sum(f[m] * _bary_integral(unit(m, i), vol, d) for m in range(n))
        F.append(kint * dot(gu_, grad[i]) + cub - src)
        sq = sum(u[m] * u[p] * lam[q] * _bary_integral(unit(m, p, q, i), vol, d)
                 for m in range(n) for p in range(n) for q in range(n))
        GU.append(kint * dot(grad[i], gl_) + 3 * sq)
        GK.append(vol / n * dot(gu_, gl_))
    return [np.array([float(x) for x in v]) for v in (F, GU, GK)]


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matches_exact_rationals(dim):
    rng = np.random.default_rng(7 + dim)
    for _ in range(4):
        xv = np.zeros((dim + 1, dim))
        for m in range(1, dim + 1):
            xv[m, m - 1] = 1.0
        xv = xv + rng.integers(-2, 3, size=xv.shape) / 8.0    # dyadic: exact in both
        uv = rng.integers(-8, 9, dim + 1) / 4.0
        kv = rng.integers(2, 7, dim + 1) / 4.0
        fv = rng.integers(-8, 9, dim + 1) / 4.0
        lv = rng.integers(-8, 9, dim + 1) / 4.0
        F, Fa, gu, gua, gk, gka = oracle.nl_element(dim, xv, uv, kv, fv, lv)
        eF, egu, egk = _exact_element(xv.tolist(), uv, kv, fv, lv)
        assert np.all(np.abs(F - eF) <= 1e-14 * (1 + Fa))
        assert np.all(np.abs(gu - egu) <= 1e-14 * (1 + gua))
        assert np.all(np.abs(gk - egk) <= 1e-14 * (1 + gka))


def _mesh(n, jitter, seed):
    st = fi.spawn_streams(seed)
    m = fi.unit_square(n)
    if jitter:
        m = fi.jitter_interior(m, jitter, st["mesh"])
    cn, N = fi.node_map(m, 1)
    return m, cn, N, st


def test_vjp_matches_central_differences():
    m, cn, N, st = _mesh(6, 0.2, 11)
    u = fi.field(st["u"], N, -1, 1); k = fi.field(st["kappa"], N, 0.5, 1.5)
    f = fi.field(st["f"], N, -1, 1); lam = fi.field(st["lam_adj"], N, -1, 1)
    rng = np.random.default_rng(3)
    du = rng.uniform(-1, 1, N); dk = rng.uniform(-1, 1, N)
    gu, _, gk, _ = oracle.nl_adjoint(2, m.cells, m.coords, cn, u, k, lam, N)
    h = 1e-6
    R = lambda uu, kk: lam @ oracle.nl_residual(2, m.cells, m.coords, cn, uu, kk, f, N)[0]
    fd_u = (R(u + h * du, k) - R(u - h * du, k)) / (2 * h)
    fd_k = (R(u, k + h * dk) - R(u, k - h * dk)) / (2 * h)
    assert abs(fd_u - gu @ du) <= 1e-7 * max(1.0, abs(fd_u))
    assert abs(fd_k - gk @ dk) <= 1e-7 * max(1.0, abs(fd_k))


def _square_integral(coef, power):
    """Exact integral over [0,1]^2 of (a x + b y + c)^power."""
    a, b, c = (Fraction(x) for x in coef)
    tot = Fraction(0)
    for i in range(power + 1):
        for j in range(power + 1 - i):
            kk = power - i - j
            mult = Fraction(factorial(power), factorial(i) * factorial(j) * factorial(kk))
            tot += mult * a ** i * b ** j * c ** kk * Fraction(1, (i + 1) * (j + 1))
    return tot


def test_global_closed_forms():
    n = 8
    m, cn, N, st = _mesh(n, 0.0, 5)
    xy = np.zeros((N, 2))
    xy[cn.ravel()] = m.coords[m.cells.ravel()]            # P1 nodes are the vertices
    ucoef = (0.75, -0.5, 0.25); fcoef = (0.5, 0.25, -0.125)
    u = ucoef[0] * xy[:, 0] + ucoef[1] * xy[:, 1] + ucoef[2]
    f = fcoef[0] * xy[:, 0] + fcoef[1] * xy[:, 1] + fcoef[2]
    k = fi.field(st["kappa"], N, 0.5, 1.5)
    F, Fa = oracle.nl_residual(2, m.cells, m.coords, cn, u, k, f, N)
    # stiffness rows sum to zero (sum of the basis is 1), so sum F = int u^3 - int f
    exact = float(_square_integral(ucoef, 3) - _square_integral(fcoef, 1))
    assert abs(F.sum() - exact) <= 1e-12 * Fa.sum()
    gu, gua, gk, gka = oracle.nl_adjoint(2, m.cells, m.coords, cn, u, k, np.ones(N), N)
    assert np.all(np.abs(gk) <= 1e-13 * (1 + gka))         # grad(lambda) = 0
    assert abs(gu.sum() - 3 * float(_square_integral(ucoef, 2))) <= 1e-12 * gua.sum()
