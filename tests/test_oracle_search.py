"""Pins of the oracle's NEAREST, random stream and informed sampling."""
import math

import numpy as np
import pytest


def test_splitmix64_published_outputs(oracle_lib):
    # SplitMix64 seeded with 0: the first three outputs of the reference
    # generator (Steele, Lea and Flood 2014; Vigna's splitmix64.c).
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    gamma = 0x9E3779B97F4A7C15
    got = [oracle_lib.mix64((gamma * (i + 1)) & 0xFFFFFFFFFFFFFFFF) for i in range(3)]
    assert got == want


def test_u01_range_and_uniformity(oracle_lib):
    u = oracle_lib.u01(oracle_lib.key(123, 1, 2, 3), 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))  # exactly 24-bit
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    chi2 = ((hist - 4000.0) ** 2 / 4000.0).sum()
    assert chi2 < 100  # 49 dof; p ~ 1e-5 threshold
    assert oracle_lib.key(1, 2, 3, 4) != oracle_lib.key(1, 2, 3, 5)


def _brute_nearest(V, g, q, c):
    d = np.sqrt(((q[None].astype(np.float64) - V.astype(np.float64)) ** 2).sum(1))
    ok = np.nonzero(g.astype(np.float64) + d < c)[0]
    if ok.size == 0:
        return -1
    order = np.lexsort((ok, g[ok].astype(np.float64), d[ok]))
    return int(ok[order[0]])


def test_nearest_brute_force(oracle_lib):
    rng = np.random.default_rng(0)
    for _ in range(20):
        N, D = int(rng.integers(1, 60)), int(rng.integers(1, 10))
        V = rng.normal(size=(N, D)).astype(np.float32)
        g = rng.uniform(0, 3, N).astype(np.float32)
        q = rng.normal(size=D).astype(np.float32)
        for c in (np.inf, 2.0, 4.0, 0.1):
            assert oracle_lib.nearest(V, g, q, c) == _brute_nearest(V, g, q, c)


def test_nearest_ties_and_budget(oracle_lib):
    V = np.array([[1, 0], [1, 0], [0, 1], [5, 5]], np.float32)
    g = np.array([2.0, 1.0, 1.0, 0.0], np.float32)
    q = np.array([0, 0], np.float32)
    # vertices 0 and 1 share a configuration: the lower cost wins; vertex 2 is
    # at the same distance with the same cost and a higher index
    assert oracle_lib.nearest(V, g, q, np.inf) == 1
    # strict budget: g + d < c, so c = 2.0 excludes vertices 1 and 2 (1 + 1)
    assert oracle_lib.nearest(V, g, q, 2.0) == -1
    assert oracle_lib.nearest(V, g, q, 2.0000001) == 1
    # only the far vertex with zero cost fits a budget of 7.1 > 5*sqrt(2)
    assert oracle_lib.nearest(V[3:], g[3:], q, 7.1) == 0
    assert oracle_lib.nearest(V[3:], g[3:], q, 7.0) == -1


def test_unit_ball_radial_law(oracle_lib):
    D = 6
    r = np.array([np.linalg.norm(oracle_lib.unit_ball(oracle_lib.key(5, 0, i, 0), D)) for i in range(4000)])
    assert r.max() <= 1.0 + 1e-12
    # radius of a uniform point in the D-ball has CDF r^D: r^D is U(0,1)
    from scipy import stats
    assert stats.kstest(r ** D, "uniform").pvalue > 1e-3


def test_unit_ball_direction_isotropic(oracle_lib):
    D = 4
    x = np.array([oracle_lib.unit_ball(oracle_lib.key(6, 0, i, 0), D) for i in range(4000)])
    u = x / np.linalg.norm(x, axis=1, keepdims=True)
    np.testing.assert_allclose(u.mean(0), 0.0, atol=0.05)
    np.testing.assert_allclose(u.T @ u / len(u), np.eye(D) / D, atol=0.03)


def test_ellipsoid_map_focal_property(oracle_lib):
    rng = np.random.default_rng(1)
    for D in (2, 7, 28):
        qs = rng.uniform(-1, 1, D).astype(np.float32)
        qg = rng.uniform(-1, 1, D).astype(np.float32)
        cmin = np.linalg.norm(qg.astype(np.float64) - qs)
        cb = 1.3 * cmin
        for i in range(200):
            x = oracle_lib.unit_ball(oracle_lib.key(7, D, i, 0), D)
            q = oracle_lib.ellipsoid_map(qs, qg, cb, x)
            assert np.linalg.norm(q - qs) + np.linalg.norm(q - qg) <= cb * (1 + 1e-9)


def test_ellipsoid_map_axes_closed_form(oracle_lib):
    qs = np.array([0.0, 0.0], np.float32)
    qg = np.array([3.0, 4.0], np.float32)  # c_min = 5, axis (0.6, 0.8)
    cb = 13.0                               # semi-axes 6.5 and 6
    a1 = np.array([0.6, 0.8])
    ctr = np.array([1.5, 2.0])
    np.testing.assert_allclose(oracle_lib.ellipsoid_map(qs, qg, cb, [1.0, 0.0]), ctr + 6.5 * a1, atol=1e-12)
    q = oracle_lib.ellipsoid_map(qs, qg, cb, [0.0, 1.0])
    assert abs(np.dot(q - ctr, a1)) < 1e-12 and np.linalg.norm(q - ctr) == pytest.approx(6.0, abs=1e-12)
    # c_best = c_min collapses onto the segment between the foci
    q = oracle_lib.ellipsoid_map(qs, qg, 5.0, [0.3, 0.9])
    np.testing.assert_allclose(q, ctr + 0.3 * 2.5 * a1, atol=1e-12)
