"""Global-assembly invariants of the oracle (no GPU).

What the method fixes for the assembled Helmholtz/Laplace/mass operators:
the mass matrix sums to the domain measure; Laplace rows sum to zero; A is
symmetric; linear (and, at P2/P3, quadratic) functions pass the patch test;
the assembled action equals the CSR matrix times x; A 1 = M 1 (the lumped
mass of the wave benchmark); the source vector sums to the integral of f.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import fem_inputs as fi
import oracle


def _mesh(kind, n, seed=11, amp=0.2):
    m = fi.unit_square(n) if kind == "square" else fi.unit_cube(n)
    return fi.jitter_interior(m, amp, np.random.default_rng(seed)) if amp else m


def _node_coords(m, cn, N, deg):
    W = fi.local_node_barycentrics(m.dim, deg) / deg
    X = np.zeros((N, m.dim))
    pos = np.einsum("lv,cvd->cld", W, m.coords[m.cells])
    X[cn.ravel()] = pos.reshape(-1, m.dim)
    return X


def _csr(vals, rp, ci, N):
    return sp.csr_matrix((vals, ci, rp), shape=(N, N))


CASES = [("square", 6, 1), ("square", 5, 2), ("square", 4, 3),
         ("cube", 3, 1), ("cube", 2, 2), ("cube", 2, 3)]


@pytest.mark.parametrize("kind,n,deg", CASES)
def test_global_invariants(kind, n, deg):
    m = _mesh(kind, n)
    cn, N = fi.node_map(m, deg)
    rng = np.random.default_rng(1)
    kappa = rng.uniform(0.5, 1.5, m.nverts)
    rp, ci = oracle.sparsity(cn, N)
    M, Ma = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kappa, rp, ci, "mass")
    K, Ka = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kappa, rp, ci, "laplace")
    H, Ha = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kappa, rp, ci, "helmholtz")
    # domain measure
    assert abs(M.sum() - 1.0) < 1e-13
    # Laplace rows sum to zero (relative to the abs-sum of contributions)
    Kc = _csr(K, rp, ci, N); Kac = _csr(Ka, rp, ci, N)
    assert np.all(np.abs(Kc @ np.ones(N)) <= 1e-13 * (Kac @ np.ones(N)))
    # bitwise symmetry (same cell order for (i,j) and (j,i))
    Hc = _csr(H, rp, ci, N)
    assert (Hc != Hc.T).nnz == 0
    # A 1 = M 1
    Mc = _csr(M, rp, ci, N)
    np.testing.assert_allclose(Hc @ np.ones(N), Mc @ np.ones(N), rtol=0,
                               atol=1e-13 * (_csr(Ha, rp, ci, N) @ np.ones(N)).max())
    # stiffness is the Helmholtz form minus the mass form
    np.testing.assert_allclose(H, K + M, rtol=0, atol=1e-14 * Ha.max())


@pytest.mark.parametrize("kind,n,deg", CASES)
def test_patch_tests(kind, n, deg):
    m = _mesh(kind, n, seed=4)
    cn, N = fi.node_map(m, deg)
    X = _node_coords(m, cn, N, deg)
    rp, ci = oracle.sparsity(cn, N)
    one = np.ones(m.nverts)
    K, Ka = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, one, rp, ci, "laplace")
    M, _ = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, one, rp, ci, "mass")
    Kc = _csr(K, rp, ci, N); S = _csr(Ka, rp, ci, N) @ np.ones(N)
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    # linear: K u = 0 in interior rows
    u = 0.3 + X @ np.linspace(1.0, 2.0, m.dim)
    r = Kc @ u
    assert np.all(np.abs(r[interior]) <= 1e-12 * S[interior] * np.abs(u).max())
    # boundary rows are not zero (the test would pass vacuously otherwise)
    assert np.abs(r[~interior]).max() > 1e-6
    if deg >= 2:
        # quadratic u = x0^2: Laplacian 2, so (K u)_i = -2 (M 1)_i in interior rows
        u2 = X[:, 0] ** 2
        lhs = (Kc @ u2)[interior]
        rhs = -2.0 * (_csr(M, rp, ci, N) @ np.ones(N))[interior]
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12 * S[interior].max())


@pytest.mark.parametrize("kind,n,deg", CASES)
def test_vector_and_action(kind, n, deg):
    m = _mesh(kind, n, seed=9)
    cn, N = fi.node_map(m, deg)
    rng = np.random.default_rng(2)
    kappa = rng.uniform(0.5, 1.5, m.nverts)
    f = rng.uniform(-1, 1, m.nverts)
    x = rng.uniform(-1, 1, N)
    rp, ci = oracle.sparsity(cn, N)
    H, Ha = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kappa, rp, ci)
    y, ya = oracle.apply_action(m.dim, deg, m.cells, m.coords, cn, kappa, x, N)
    np.testing.assert_allclose(y, _csr(H, rp, ci, N) @ x, rtol=0, atol=1e-13 * ya.max())
    y1, _ = oracle.apply_action(m.dim, deg, m.cells, m.coords, cn, kappa, np.ones(N), N)
    M, _ = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kappa, rp, ci, "mass")
    np.testing.assert_allclose(y1, _csr(M, rp, ci, N) @ np.ones(N), rtol=0, atol=1e-13)
    # sum of b = integral of f = 1^T M_P1 f
    b, _ = oracle.assemble_vec(m.dim, deg, m.cells, m.coords, cn, f, N)
    rp1, ci1 = oracle.sparsity(m.cells, m.nverts)
    M1, _ = oracle.assemble_mat(m.dim, 1, m.cells, m.coords, m.cells, kappa, rp1, ci1, "mass")
    assert abs(b.sum() - np.ones(m.nverts) @ (_csr(M1, rp1, ci1, m.nverts) @ f)) < 1e-13
    # f = 1 reproduces the lumped mass
    b1, _ = oracle.assemble_vec(m.dim, deg, m.cells, m.coords, cn, np.ones(m.nverts), N)
    np.testing.assert_allclose(b1, _csr(M, rp, ci, N) @ np.ones(N), rtol=0, atol=1e-14)


def test_unjittered_square_stencil():
    """64x64 unit square, P1, kappa=1: 5-point Laplacian (diagonal neighbours
    structurally present with value 0); mass h^2/2 and h^2/12."""
    n = 64; h = 1.0 / n
    m = fi.unit_square(n)
    rp, ci = oracle.sparsity(m.cells, m.nverts)
    one = np.ones(m.nverts)
    K, _ = oracle.assemble_mat(2, 1, m.cells, m.coords, m.cells, one, rp, ci, "laplace")
    M, _ = oracle.assemble_mat(2, 1, m.cells, m.coords, m.cells, one, rp, ci, "mass")
    i, j = 20, 33
    r = j * (n + 1) + i
    cols = ci[rp[r]:rp[r + 1]]
    kr = dict(zip(cols, K[rp[r]:rp[r + 1]])); mr = dict(zip(cols, M[rp[r]:rp[r + 1]]))
    assert len(cols) == 7
    vid = lambda a, b: b * (n + 1) + a
    assert abs(kr[r] - 4) < 1e-13
    for nb in (vid(i + 1, j), vid(i - 1, j), vid(i, j + 1), vid(i, j - 1)):
        assert abs(kr[nb] + 1) < 1e-13
    for nb in (vid(i + 1, j + 1), vid(i - 1, j - 1)):
        assert nb in kr and abs(kr[nb]) < 1e-13
    assert abs(mr[r] - h * h / 2) < 1e-17
    for c in cols:
        if c != r:
            assert abs(mr[c] - h * h / 12) < 1e-17


@pytest.mark.parametrize("kind,n,deg", [("square", 4, 2), ("cube", 2, 3)])
def test_sampled_rows_match_full_assembly(kind, n, deg):
    m = _mesh(kind, n, seed=21)
    cn, N = fi.node_map(m, deg)
    rng = np.random.default_rng(8)
    kappa = rng.uniform(0.5, 1.5, m.nverts); f = rng.uniform(-1, 1, m.nverts)
    x = rng.uniform(-1, 1, N)
    rp, ci = oracle.sparsity(cn, N)
    H, Ha = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kappa, rp, ci)
    rows = rng.choice(N, 7, replace=False)
    got = oracle.mat_rows(m.dim, deg, m.cells, m.coords, cn, kappa, N, rows)
    for r, (c, v, a) in zip(rows, got):
        np.testing.assert_array_equal(c, ci[rp[r]:rp[r + 1]])
        np.testing.assert_array_equal(v, H[rp[r]:rp[r + 1]])     # same cell order
        np.testing.assert_array_equal(a, Ha[rp[r]:rp[r + 1]])
    b, _ = oracle.assemble_vec(m.dim, deg, m.cells, m.coords, cn, f, N)
    bs, _ = oracle.vec_rows(m.dim, deg, m.cells, m.coords, cn, f, N, rows)
    np.testing.assert_array_equal(bs, b[rows])
    y, _ = oracle.apply_action(m.dim, deg, m.cells, m.coords, cn, kappa, x, N)
    ys, _ = oracle.action_rows(m.dim, deg, m.cells, m.coords, cn, kappa, x, N, rows)
    np.testing.assert_array_equal(ys, y[rows])


@pytest.mark.parametrize("kind,n,deg", CASES)
def test_scales_bracket_the_values(kind, n, deg):
    """The two rounding scales the oracle returns bracket each entry:
    |a_ij| <= sum over cells of |element entry| <= sum over cells and points
    of |term| (triangle inequality, twice).  The P1 mass matrix has only
    positive element entries (|K|(1 + delta_ij)/((d+1)(d+2))), so there the
    contribution-level scale is the value itself, bit for bit; mat_rows
    returns the same scales as the full assembly."""
    m = _mesh(kind, n)
    cn, N = fi.node_map(m, deg)
    kap = np.random.default_rng(3).uniform(0.5, 1.5, m.nverts)
    rp, ci = oracle.sparsity(cn, N)
    v, a, ca = oracle.assemble_mat(m.dim, deg, m.cells, m.coords, cn, kap, rp, ci, contrib_scale=True)
    assert np.all(np.abs(v) <= ca * (1 + 1e-14)) and np.all(ca <= a * (1 + 1e-14))
    rows = np.array([0, N // 2, N - 1])
    for r, (cols, vr, ar, car) in zip(rows, oracle.mat_rows(m.dim, deg, m.cells, m.coords, cn, kap, N, rows,
                                                          contrib_scale=True)):
        np.testing.assert_array_equal(cols, ci[rp[r]:rp[r + 1]])
        np.testing.assert_allclose(car, ca[rp[r]:rp[r + 1]], rtol=1e-13)
    if deg == 1:
        vm, am, cm = oracle.assemble_mat(m.dim, 1, m.cells, m.coords, cn, kap, rp, ci, "mass", contrib_scale=True)
        assert np.all(vm > 0) and np.array_equal(vm, cm)
