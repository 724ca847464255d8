"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test targets a plausible mistake: a wrong quadrature node/weight, a basis
function in the wrong local slot or with a wrong constant, a transposed
Jacobian, a missing |det J|, a dropped mass or stiffness term, a wrong sign.
"""
import itertools
from fractions import Fraction
from math import factorial

import os

import numpy as np
import pytest

import fem_inputs as fi
import oracle
import exact_fem as ef


# --------------------------------------------------------------- quadrature

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_simplex_rule_exact_on_monomials(dim, q):
    """int over the reference simplex of x^a = a!/(|a|+d)!  for |a| <= 2q-1."""
    pts, w = oracle.simplex_rule(dim, q)
    for a in itertools.product(range(2 * q), repeat=dim):
        if sum(a) > 2 * q - 1:
            continue
        exact = np.prod([factorial(x) for x in a]) / factorial(sum(a) + dim)
        got = np.sum(w * np.prod(pts ** np.array(a), axis=1))
        assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-16, (a, got, exact)


def test_simplex_rule_not_exact_beyond_order():
    """A rule that is secretly of higher order would hide a wrong point count."""
    pts, w = oracle.simplex_rule(2, 2)
    a = (4, 0)
    exact = factorial(4) / factorial(6)
    assert abs(np.sum(w * pts[:, 0] ** 4) - exact) > 1e-6


@pytest.mark.parametrize("alpha", [0, 1, 2])
def test_gauss_jacobi_matches_legendre_table(alpha):
    """alpha=0 must reduce to the textbook 2-point Gauss-Legendre rule."""
    t, w = oracle.gauss_jacobi(2, alpha)
    if alpha == 0:
        np.testing.assert_allclose(np.sort(t), [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)],
                                   rtol=0, atol=1e-15)
        np.testing.assert_allclose(w, [0.5, 0.5], atol=1e-15)
    # total mass of the weight (1-t)^alpha on [0,1]
    assert abs(w.sum() - 1.0 / (alpha + 1)) < 1e-15


# --------------------------------------------------------------- basis

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("deg", [1, 2, 3])
def test_basis_lagrange_property(dim, deg):
    """phi_i(node_j) = delta_ij at the node positions of the local ordering."""
    W = fi.local_node_barycentrics(dim, deg) / deg
    for j, lam in enumerate(W):
        phi, _ = oracle.basis(dim, deg, lam)
        e = np.zeros(len(W)); e[j] = 1
        np.testing.assert_allclose(phi, e, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("deg", [1, 2, 3])
def test_basis_partition_of_unity_and_derivatives(dim, deg):
    rng = np.random.default_rng(7)
    for _ in range(5):
        lam = rng.dirichlet(np.ones(dim + 1))
        phi, dphi = oracle.basis(dim, deg, lam)
        assert abs(phi.sum() - 1) < 1e-13
        h = 1e-6
        for m in range(dim + 1):
            lp = lam.copy(); lp[m] += h
            lm = lam.copy(); lm[m] -= h
            fd = (oracle.basis(dim, deg, lp)[0] - oracle.basis(dim, deg, lm)[0]) / (2 * h)
            np.testing.assert_allclose(dphi[:, m], fd, atol=1e-7)


# --------------------------------------------------------------- element tensors

def _random_rational_cell(rng, dim):
    while True:
        xv = rng.integers(-8, 9, size=(dim + 1, dim)) / 8.0
        J = (xv[1:] - xv[0]).T
        if abs(np.linalg.det(J)) > 0.05:
            return xv


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("deg", [1, 2, 3])
def test_element_matrix_matches_exact(dim, deg):
    """Oracle element matrix vs exact rational integration (independent path)."""
    rng = np.random.default_rng(100 + 10 * dim + deg)
    for trial in range(2):
        xv = _random_rational_cell(rng, dim)
        if trial == 1:
            xv = xv[[0, 2, 1] + list(range(3, dim + 1))]   # negative orientation
        kv = rng.integers(1, 9, size=dim + 1) / 4.0
        for form, (cs, cm) in oracle.FORMS.items():
            A = oracle.element_matrix(dim, deg, xv, kv, form)
            E = ef.to_float(ef.element_matrix_exact(dim, deg, xv, kv, cs, cm))
            scale = np.abs(E).max()
            np.testing.assert_allclose(A, E, rtol=0, atol=1e-13 * scale, err_msg=form)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("deg", [1, 2, 3])
def test_element_vector_matches_exact(dim, deg):
    rng = np.random.default_rng(200 + 10 * dim + deg)
    xv = _random_rational_cell(rng, dim)
    fv = rng.integers(-8, 9, size=dim + 1) / 4.0
    b = oracle.element_vector(dim, deg, xv, fv)
    e = ef.to_float(ef.element_vector_exact(dim, deg, xv, fv))
    np.testing.assert_allclose(b, e, rtol=0, atol=1e-14 * np.abs(e).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_closed_forms(dim):
    """P1 mass = |K|(1+delta_ij)/((d+1)(d+2)); P1 stiffness = kbar |K| grad l_i . grad l_j."""
    rng = np.random.default_rng(3)
    xv = rng.normal(size=(dim + 1, dim))
    kv = rng.uniform(0.5, 1.5, size=dim + 1)
    J = (xv[1:] - xv[0]).T
    vol = abs(np.linalg.det(J)) / factorial(dim)
    Mex = vol * (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / ((dim + 1) * (dim + 2))
    G = np.linalg.inv(J)                               # rows: grad lambda_1..d
    glam = np.vstack([-G.sum(0), G])
    Kex = kv.mean() * vol * glam @ glam.T
    np.testing.assert_allclose(oracle.element_matrix(dim, 1, xv, kv, "mass"), Mex,
                               rtol=0, atol=1e-14 * np.abs(Mex).max())
    np.testing.assert_allclose(oracle.element_matrix(dim, 1, xv, kv, "laplace"), Kex,
                               rtol=0, atol=1e-13 * np.abs(Kex).max())


# Integer reference matrices of the P2 spaces (derived by exact integration of
# the Lagrange basis; local order vertices then edges (0,1),(0,2),...).
P2_TET_MASS_420 = np.array([
    [6, 1, 1, 1, -4, -4, -4, -6, -6, -6], [1, 6, 1, 1, -4, -6, -6, -4, -4, -6],
    [1, 1, 6, 1, -6, -4, -6, -4, -6, -4], [1, 1, 1, 6, -6, -6, -4, -6, -4, -4],
    [-4, -4, -6, -6, 32, 16, 16, 16, 16, 8], [-4, -6, -4, -6, 16, 32, 16, 16, 8, 16],
    [-4, -6, -6, -4, 16, 16, 32, 8, 16, 16], [-6, -4, -4, -6, 16, 16, 8, 32, 16, 16],
    [-6, -4, -6, -4, 16, 8, 16, 16, 32, 16], [-6, -6, -4, -4, 8, 16, 16, 16, 16, 32]])
P2_REFTET_STIFF_30 = np.array([
    [9, 1, 1, 1, -6, -6, -6, 2, 2, 2], [1, 3, 0, 0, -4, 1, 1, -1, -1, 0],
    [1, 0, 3, 0, 1, -4, 1, -1, 0, -1], [1, 0, 0, 3, 1, 1, -4, 0, -1, -1],
    [-6, -4, 1, 1, 24, 4, 4, -8, -8, -8], [-6, 1, -4, 1, 4, 24, 4, -8, -8, -8],
    [-6, 1, 1, -4, 4, 4, 24, -8, -8, -8], [2, -1, -1, 0, -8, -8, -8, 16, 4, 4],
    [2, -1, 0, -1, -8, -8, -8, 4, 16, 4], [2, 0, -1, -1, -8, -8, -8, 4, 4, 16]])
P2_TRI_MASS_180 = np.array([
    [6, -1, -1, 0, 0, -4], [-1, 6, -1, 0, -4, 0], [-1, -1, 6, -4, 0, 0],
    [0, 0, -4, 32, 16, 16], [0, -4, 0, 16, 32, 16], [-4, 0, 0, 16, 16, 32]])


def test_p2_integer_reference_matrices():
    ref_tet = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    ref_tri = np.array([[0, 0], [1, 0], [0, 1]], float)
    M = oracle.element_matrix(3, 2, ref_tet, np.ones(4), "mass")
    np.testing.assert_allclose(M * 420 * 6, P2_TET_MASS_420, atol=1e-11)
    K = oracle.element_matrix(3, 2, ref_tet, np.ones(4), "laplace")
    np.testing.assert_allclose(K * 30, P2_REFTET_STIFF_30, atol=1e-11)
    M = oracle.element_matrix(2, 2, ref_tri, np.ones(3), "mass")
    np.testing.assert_allclose(M * 180 * 2, P2_TRI_MASS_180, atol=1e-11)
    # and the exact path agrees with the integers too (pins the pin)
    Mx = ef.to_float(ef.element_matrix_exact(3, 2, ref_tet, np.ones(4), 0, 1))
    np.testing.assert_allclose(Mx * 420 * 6, P2_TET_MASS_420, atol=1e-11)


# --------------------------------------------------------------- two-cell meshes

def _assemble_dense(mesh, deg, kappa, form):
    cn, N = fi.node_map(mesh, deg)
    rp, ci = oracle.sparsity(cn, N)
    v, _ = oracle.assemble_mat(mesh.dim, deg, mesh.cells, mesh.coords, cn, kappa, rp, ci, form)
    A = np.full((N, N), np.nan)
    for r in range(N):
        for k in range(rp[r], rp[r + 1]):
            A[r, ci[k]] = v[k]
    return A


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    """Hand-derived scaled matrices of a fixture file: {form: (scale, matrix)},
    NaN where the fixture marks a pair absent from the sparsity."""
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("scale"):
                _, sc, form = line.split()
                cur = (form, float(sc), [])
                out[form] = cur
                continue
            cur[2].append([np.nan if t == "x" else float(t) for t in line.split()])
    return {f: (sc, np.array(rows)) for f, (_, sc, rows) in out.items()}


def test_two_triangles_hand_values():
    m = fi.two_triangles()
    g = _golden("two_triangles_p1.txt")
    K = _assemble_dense(m, 1, np.ones(4), "laplace")
    M = _assemble_dense(m, 1, np.ones(4), "mass")
    np.testing.assert_allclose(g["laplace"][0] * K, g["laplace"][1], atol=1e-14)   # nan positions must match
    np.testing.assert_allclose(g["mass"][0] * M, g["mass"][1], atol=1e-14)
    assert K[0, 2] == 0.0                                # structurally present, value 0


def test_two_tets_hand_values():
    m = fi.two_tets()
    g = _golden("two_tets_p1.txt")
    K = _assemble_dense(m, 1, np.ones(5), "laplace")
    M = _assemble_dense(m, 1, np.ones(5), "mass")
    np.testing.assert_allclose(g["laplace"][0] * K, g["laplace"][1], atol=1e-13)
    np.testing.assert_allclose(g["mass"][0] * M, g["mass"][1], atol=1e-13)
    assert abs(np.nansum(M) - 0.5) < 1e-15


# --------------------------------------------------------------- sparsity

def _brute_pattern(cn, N):
    P = np.zeros((N, N), bool)
    for c in cn:
        P[np.ix_(c, c)] = True
    return P


@pytest.mark.parametrize("kind,n", [("square", 1), ("square", 3), ("cube", 1), ("cube", 2)])
@pytest.mark.parametrize("deg", [1, 2, 3])
def test_sparsity_brute_force(kind, n, deg):
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    cn, N = fi.node_map(m, deg)
    rp, ci = oracle.sparsity(cn, N)
    P = _brute_pattern(cn, N)
    for r in range(N):
        np.testing.assert_array_equal(ci[rp[r]:rp[r + 1]], np.nonzero(P[r])[0])


NNZ_FORMULAS = {
    ("square", 1): lambda n: 7 * n * n + 6 * n + 1,
    ("square", 2): lambda n: 46 * n * n + 16 * n + 1,
    ("square", 3): lambda n: 153 * n * n + 30 * n + 1,
    ("cube", 1): lambda n: 15 * n ** 3 + 21 * n * n + 9 * n + 1,
    ("cube", 2): lambda n: 230 * n ** 3 + 138 * n * n + 24 * n + 1,
    ("cube", 3): lambda n: 1311 * n ** 3 + 459 * n * n + 45 * n + 1,
}


@pytest.mark.parametrize("key", list(NNZ_FORMULAS))
def test_sparsity_nnz_closed_forms(key):
    kind, deg = key
    for n in ([1, 2, 5, 9] if kind == "square" else [1, 2, 4]):
        m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
        cn, N = fi.node_map(m, deg)
        rp, ci = oracle.sparsity(cn, N)
        assert rp[-1] == NNZ_FORMULAS[key](n), (key, n)


def test_sparsity_p1_tri_nnz_from_edges():
    """P1 nnz = V + 2E (each edge couples two vertices both ways)."""
    m = fi.unit_square(6)
    edges = set()
    for c in m.cells:
        for a, b in itertools.combinations(sorted(c), 2):
            edges.add((a, b))
    rp, _ = oracle.sparsity(m.cells, m.nverts)
    assert rp[-1] == m.nverts + 2 * len(edges)


def test_sparsity_invariant_under_cell_permutation_and_local_order():
    m = fi.unit_cube(2)
    cn, N = fi.node_map(m, 2)
    rp, ci = oracle.sparsity(cn, N)
    rng = np.random.default_rng(5)
    cn2 = cn[rng.permutation(len(cn))]
    cn2 = np.take_along_axis(cn2, np.argsort(rng.random(cn2.shape), 1), 1)
    rp2, ci2 = oracle.sparsity(cn2, N)
    np.testing.assert_array_equal(rp, rp2)
    np.testing.assert_array_equal(ci, ci2)


def test_sparsity_rejects_out_of_range():
    cn = np.array([[0, 1, 5]], np.int32)
    with pytest.raises(ValueError):
        oracle.sparsity(cn, 3)
