"""Checks of the seeded input generators (no GPU)."""
import numpy as np
import pytest

import fem_inputs as fi


def _dets(m):
    X = m.coords[m.cells]
    return np.linalg.det(np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1)))


@pytest.mark.parametrize("n", [1, 3, 8])
def test_generated_meshes_positive_and_conforming(n):
    for m in (fi.unit_square(n), fi.unit_cube(n)):
        d = _dets(m)
        assert d.min() > 0
        # total measure 1
        from math import factorial
        assert abs(d.sum() / factorial(m.dim) - 1.0) < 1e-12
        # conforming: every facet is shared by at most two cells
        facets = {}
        for c in m.cells:
            for skip in range(m.dim + 1):
                f = tuple(sorted(np.delete(c, skip)))
                facets[f] = facets.get(f, 0) + 1
        assert max(facets.values()) <= 2


def test_jitter_keeps_boundary_and_orientation_at_config_sizes():
    """The jittered 64^3 Kuhn cube (seed stream 'mesh' of 1501) stays valid."""
    rng = fi.spawn_streams(1501)["mesh"]
    m = fi.jitter_interior(fi.unit_cube(64), 0.2, rng)
    d = _dets(m)
    assert d.min() > 0
    assert abs(d.sum() / 6 - 1.0) < 1e-12
    b = np.any((m.vlat == 0) | (m.vlat == 64), axis=1)
    np.testing.assert_array_equal(m.coords[b], m.vlat[b] / 64.0)


def test_node_map_counts_and_sharing():
    m = fi.unit_cube(3)
    for k, N in ((1, 4 ** 3), (2, 7 ** 3), (3, 10 ** 3)):
        cn, NN = fi.node_map(m, k)
        assert NN == N and len(np.unique(cn)) == N
        ft, NF = fi.node_map(m, k, "first_touch")
        assert NF == N
        # both numberings describe the same node sets per cell up to relabelling
        lab = {}
        for a, b in zip(cn.ravel(), ft.ravel()):
            assert lab.setdefault(a, b) == b


def test_seed_streams_are_independent():
    a = fi.spawn_streams(1501); b = fi.spawn_streams(1501)
    x1 = fi.field(a["kappa"], 5, 0.5, 1.5)
    _ = fi.field(b["f"], 100, -1, 1)                 # drawing another stream first
    x2 = fi.field(b["kappa"], 5, 0.5, 1.5)
    np.testing.assert_array_equal(x1, x2)
    assert x1.min() >= 0.5 and x1.max() < 1.5
