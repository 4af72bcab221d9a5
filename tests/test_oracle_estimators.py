"""Pins of the edge-intersection and distance estimators of the solid
fraction (the alternatives Sec. 2.3.2 names) against closed forms."""
import math

import numpy as np
import pytest

from oracle import geometry as geo


def test_edge_estimate_closed_forms():
    assert geo.eps_edge(np.zeros(3), 5.0) == 1.0  # cell deep inside
    assert geo.eps_edge(np.array([9.0, 0.0, 0.0]), 5.0) == 0.0  # far outside
    # sphere of radius 1/2 centred on a cell corner: the three edges from that
    # corner are covered over half their length
    assert geo.eps_edge(np.array([0.5, 0.5, 0.5]), 0.5) == pytest.approx(1.5 / 12.0, abs=1e-15)
    # radius 1 on a corner: those three edges fully, nothing else (the next
    # corners are at distance 1, exactly on the surface)
    assert geo.eps_edge(np.array([0.5, 0.5, 0.5]), 1.0) == pytest.approx(3.0 / 12.0, abs=1e-15)
    # a very large sphere whose surface passes through the cell centre: a plane
    # -> half the edge length
    R = 1e6
    assert geo.eps_edge(np.array([R, 0.0, 0.0]), R) == pytest.approx(0.5, abs=1e-6)
    # plane through the cell at x = +0.25 (inside on -x): x-edges 3/4, faces
    # at x = -1/2 fully, at x = +1/2 not
    assert geo.eps_edge(np.array([R - 0.25, 0.0, 0.0]), R) == pytest.approx((4 * 0.75 + 4) / 12.0, abs=1e-6)


def test_edge_estimate_symmetry():
    rng = np.random.default_rng(3)
    for _ in range(200):
        R = rng.uniform(2, 9)
        d = rng.standard_normal(3)
        d *= (R + rng.uniform(-0.9, 0.9)) / np.linalg.norm(d)
        e = geo.eps_edge(d, R)
        assert 0.0 <= e <= 1.0
        for perm in ([1, 2, 0], [2, 0, 1]):
            assert geo.eps_edge(d[perm], R) == pytest.approx(e, abs=1e-14)
        assert geo.eps_edge(-d, R) == pytest.approx(e, abs=1e-14)


def test_distance_estimate():
    R = 6.0
    assert geo.eps_distance(np.array([R, 0.0, 0.0]), R) == 0.5
    assert geo.eps_distance(np.array([R - 0.5, 0.0, 0.0]), R) == 1.0
    assert geo.eps_distance(np.array([R + 0.5, 0.0, 0.0]), R) == 0.0
    assert geo.eps_distance(np.array([0.0, R + 0.25, 0.0]), R) == 0.25
    r = np.linspace(R - 1, R + 1, 41)
    v = [geo.eps_distance(np.array([0.0, 0.0, x]), R) for x in r]
    assert all(a >= b for a, b in zip(v, v[1:]))


@pytest.mark.parametrize("est,tol", [(geo.eps_edge, 0.01), (geo.eps_distance, 0.01)])
def test_total_is_sphere_volume(est, tol):
    # summed over all cells both estimators approach the sphere volume
    R = 7.3
    X = np.array([0.31, -0.17, 0.42])
    r = np.arange(-10, 10)
    tot = 0.0
    for i in r:
        for j in r:
            for k in r:
                d = np.array([i + 0.5, j + 0.5, k + 0.5]) - X
                tot += est(d, R)
    V = 4.0 / 3.0 * math.pi * R ** 3
    assert abs(tot - V) / V < tol


def test_count_rounding():
    assert geo.eps_count(0.5, 16) == 2048
    assert geo.eps_count(1.0 / 8192.0, 16) == 0  # a tie: to even
    assert geo.eps_count(3.0 / 8192.0, 16) == 2
