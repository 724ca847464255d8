"""Pins of the oracle's vector Lagrange linear elasticity,
a(u, v) = integral of 2 mu eps(u):eps(v) + lam div(u) div(v), with per-cell
coordinates (some cells flattened to aspect ratio ~1e3).

The pins do not use the oracle's quadrature or basis: exact rational element
matrices built from a Vandermonde nodal basis, the rigid motions that every
elasticity operator annihilates, energies of linear displacement fields
against sums over cells of |K| times mean coefficients, bitwise symmetry and
positive semi-definiteness.
"""
from fractions import Fraction

import numpy as np
import pytest

import fem_inputs as fi
import oracle
from exact_fem import _det_exact, _inv_exact, reference_tensors


def _exact_elasticity(dim, k, xv, muv, lav):
    """A[(i,a),(j,b)] = sum_m mu_m (delta_ab sum_p P_m[p][p] + P_m[b][a]) + lam_m P_m[a][b],
    P_m[p][q][i][j] = integral over K of lambda_m d_p phi_i d_q phi_j, exactly."""
    X = [[Fraction(v) for v in row] for row in xv]
    mu = [Fraction(v) for v in muv]; la = [Fraction(v) for v in lav]
    J = [[X[c + 1][r] - X[0][r] for c in range(dim)] for r in range(dim)]
    adet = abs(_det_exact(J))
    Ji = _inv_exact(J)                      # Ji[r][p] = d xi_r / d x_p
    _, S, _ = reference_tensors(dim, k)     # S[m][r][s][i][j] on the reference cell
    n = len(S[0][0][0])
    N = dim * n
    A = [[Fraction(0)] * N for _ in range(N)]
    for m in range(dim + 1):
        P = [[[[adet * sum(Ji[r][p] * Ji[s][q] * S[m][r][s][i][j] for r in range(dim) for s in range(dim))
                for j in range(n)] for i in range(n)] for q in range(dim)] for p in range(dim)]
        for i in range(n):
            for j in range(n):
                tr = sum(P[p][p][i][j] for p in range(dim))
                for a in range(dim):
                    for b in range(dim):
                        A[i * dim + a][j * dim + b] += (mu[m] * ((tr if a == b else 0) + P[b][a][i][j])
                                                        + la[m] * P[a][b][i][j])
    return np.array([[float(v) for v in row] for row in A])


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_element_matches_exact_rationals(dim, k):
    rng = np.random.default_rng(31 + 10 * dim + k)
    for _ in range(2):
        xv = np.zeros((dim + 1, dim))
        for m in range(1, dim + 1):
            xv[m, m - 1] = 1.0
        xv = xv + rng.integers(-2, 3, size=xv.shape) / 8.0
        muv = rng.integers(2, 9, dim + 1) / 4.0
        lav = rng.integers(2, 9, dim + 1) / 4.0
        A, Aa = oracle.elasticity_element(dim, k, xv, muv, lav)
        E = _exact_elasticity(dim, k, xv.tolist(), muv, lav)
        assert np.all(np.abs(A - E) <= 1e-13 * (1 + Aa))


def _flattened_cube(n, seed, frac=0.01):
    st = fi.spawn_streams(seed)
    m = fi.jitter_interior(fi.unit_cube(n), 0.2, st["mesh"])
    xdg, chosen = fi.flatten_cells(fi.dg_coordinates(m), frac, st["flatten"])
    cn, N = fi.node_map(m, 2)
    mu = fi.field(st["mu"], m.nverts, 0.5, 2.0)
    lam = fi.field(st["lam"], m.nverts, 0.5, 2.0)
    return m, xdg, chosen, cn, N, mu, lam


def _node_positions(xv, dim, k):
    W = fi.local_node_barycentrics(dim, k) / k
    return W @ xv


def _rigid_modes(P):
    """Translations and infinitesimal rotations sampled at points P [n][3]: [6][3n]."""
    modes = []
    for a in range(3):
        t = np.zeros_like(P); t[:, a] = 1.0
        modes.append(t.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w, P).ravel())
    return modes


def test_rigid_motions_in_the_kernel_of_every_element():
    m, xdg, chosen, cn, N, mu, lam = _flattened_cube(4, 77, frac=0.05)
    assert chosen.size > 0
    for c in list(chosen[:6]) + [0, 17, 101]:
        A, Aa = oracle.elasticity_element(3, 2, xdg[c], mu[m.cells[c]], lam[m.cells[c]])
        P = _node_positions(xdg[c], 3, 2)
        for r in _rigid_modes(P):
            assert np.all(np.abs(A @ r) <= 1e-12 * (Aa @ np.abs(r)) + 1e-300)


def _global(n, seed, frac):
    m, xdg, chosen, cn, N, mu, lam = _flattened_cube(n, seed, frac)
    vm = oracle.vector_map(cn, 3)
    rp, ci = oracle.sparsity(vm, 3 * N)
    vals, absv = oracle.elasticity_mat(3, 2, m.cells, xdg, cn, mu, lam, rp, ci)
    return m, xdg, chosen, cn, N, mu, lam, rp, ci, vals, absv


def _dense(rp, ci, vals, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, ci[rp[r]:rp[r + 1]]] = vals[rp[r]:rp[r + 1]]
    return A


def test_global_translations_symmetry_and_semidefiniteness():
    m, xdg, chosen, cn, N, mu, lam, rp, ci, vals, absv = _global(3, 5, 0.05)
    assert chosen.size > 0
    A = _dense(rp, ci, vals, 3 * N)
    Aa = _dense(rp, ci, absv, 3 * N)
    assert np.array_equal(A, A.T)                         # bitwise symmetric
    for a in range(3):
        t = np.zeros(3 * N); t[a::3] = 1.0
        assert np.all(np.abs(A @ t) <= 1e-12 * (Aa @ t) + 1e-300)
    rng = np.random.default_rng(2)
    w = np.linalg.eigvalsh(A)
    assert w.min() >= -1e-12 * w.max()
    assert np.sum(w < 1e-10 * w.max()) >= 3               # at least the translations
    for _ in range(3):
        x = rng.uniform(-1, 1, 3 * N)
        assert x @ A @ x > 0


def test_energy_of_linear_displacements():
    """Unflattened (conforming) mesh: u = (x,0,0) has energy sum_K |K| (2 mu_K + lam_K),
    u = (y,0,0) has sum_K |K| mu_K (mean of the P1 coefficient over K)."""
    m, xdg, chosen, cn, N, mu, lam, rp, ci, vals, absv = _global(3, 9, 0.0)
    assert chosen.size == 0
    A = _dense(rp, ci, vals, 3 * N)
    pos = np.zeros((N, 3))
    for c in range(m.ncells):
        pos[cn[c]] = _node_positions(xdg[c], 3, 2)
    X = xdg
    vol = np.abs(np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], 2))) / 6
    mbar = mu[m.cells].mean(1); lbar = lam[m.cells].mean(1)
    u = np.zeros(3 * N); u[0::3] = pos[:, 0]
    assert abs(u @ A @ u - np.sum(vol * (2 * mbar + lbar))) <= 1e-12 * np.sum(vol * (2 * mbar + lbar))
    u = np.zeros(3 * N); u[0::3] = pos[:, 1]
    assert abs(u @ A @ u - np.sum(vol * mbar)) <= 1e-12 * np.sum(vol * mbar)


def test_rows_equal_full_assembly():
    m, xdg, chosen, cn, N, mu, lam, rp, ci, vals, absv = _global(3, 12, 0.05)
    rows = np.array([0, 1, 5, 3 * N // 2, 3 * N - 1])
    out = oracle.elasticity_rows(3, 2, m.cells, xdg, cn, mu, lam, 3 * N, rows)
    for r, (cols, v, a) in zip(rows, out):
        assert np.array_equal(cols, ci[rp[r]:rp[r + 1]])
        assert np.array_equal(v, vals[rp[r]:rp[r + 1]])
        assert np.array_equal(a, absv[rp[r]:rp[r + 1]])


def test_flattened_cells_generator():
    """round(1%) of the cells, chosen by the seeded permutation, keep their
    orientation; det J scales by (new height) / (old height) exactly as the
    construction says, and the aspect ratio reaches ~1e3."""
    st = fi.spawn_streams(1501)
    m = fi.jitter_interior(fi.unit_cube(8), 0.2, st["mesh"])
    x0 = fi.dg_coordinates(m)
    x1, chosen = fi.flatten_cells(x0, 0.01, st["flatten"])
    assert chosen.size == round(0.01 * m.ncells)
    same = np.setdiff1d(np.arange(m.ncells), chosen)
    assert np.array_equal(x0[same], x1[same])
    J = lambda X: np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], 2)
    d0 = np.linalg.det(J(x0[chosen])); d1 = np.linalg.det(J(x1[chosen]))
    assert np.all(d0 > 0) and np.all(d1 > 0)
    v0, v1, v2 = x0[chosen, 0], x0[chosen, 1], x0[chosen, 2]
    area2 = np.linalg.norm(np.cross(v1 - v0, v2 - v0), axis=1)
    L = np.max(np.stack([np.linalg.norm(v1 - v0, axis=1), np.linalg.norm(v2 - v0, axis=1),
                         np.linalg.norm(v2 - v1, axis=1)]), axis=0)
    assert np.allclose(d1, area2 * L / 1e3, rtol=1e-12)   # det = 2 * area * height
    edges = np.stack([np.linalg.norm(x1[chosen, a] - x1[chosen, b], axis=1)
                      for a in range(4) for b in range(a + 1, 4)], 1)
    alt = d1 / np.max(np.stack([np.linalg.norm(np.cross(x1[chosen, b] - x1[chosen, a],
                                                        x1[chosen, c] - x1[chosen, a]), axis=1)
                                for a, b, c in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))]), axis=0)
    assert np.all(edges.max(1) / alt > 500)
