"""Pins of the oracle's collision margins, edge discretisation and
coarse-to-fine checker: textbook cases, analytic sweeps, brute force on tiny
scenes and invariants."""
import math

import numpy as np
import pytest

import workloads as W

Z4 = np.zeros((0, 4), np.float32)
Z6 = np.zeros((0, 6), np.float32)


def _point_robot(radius=0.05):
    """One sphere on link 1 of a 1-joint chain at the base origin: a point
    robot whose world centre is the base translation."""
    m = W.RobotModel("point", np.zeros((1, 4), np.float32), np.array([-1], np.float32),
                     np.array([1], np.float32), np.array([1], np.int32),
                     np.array([[0, 0, 0, radius]], np.float32))
    return m


def _scene_point(x, y, z, radius=0.05, spheres=Z4, boxes=Z6):
    return W.Scene([_point_robot(radius)], W.base_transform(x, y, 0.0, z)[None],
                   np.asarray(spheres, np.float32).reshape(-1, 4),
                   np.asarray(boxes, np.float32).reshape(-1, 6))


def test_sphere_sphere_margin(oracle_lib):
    sc = _scene_point(0.3, 0.4, 0.0, 0.05, spheres=[[0, 0, 0, 0.2]])
    m = oracle_lib.state_margins(sc, np.zeros((1, 1), np.float32))[0]
    assert m == pytest.approx(0.5 - 0.25, abs=1e-7)


@pytest.mark.parametrize("pt,want", [
    ((0.5, 0.5, 0.5), -0.05),                       # centre inside the box
    ((1.25, 0.5, 0.5), 0.25 - 0.05),                # offset along x only
    ((0.5, -0.5, 0.5), 0.5 - 0.05),                 # offset along y only
    ((1.3, 1.4, 0.5), math.hypot(0.3, 0.4) - 0.05),  # edge region
    ((2.0, 3.0, 3.0), math.sqrt(1 + 4 + 4) - 0.05),  # corner region
])
def test_sphere_box_margin_arvo_cases(oracle_lib, pt, want):
    sc = _scene_point(*pt, 0.05, boxes=[[0, 0, 0, 1, 1, 1]])
    m = oracle_lib.state_margins(sc, np.zeros((1, 1), np.float32))[0]
    assert m == pytest.approx(want, abs=1e-6)


def test_robot_robot_margin(oracle_lib):
    p = _point_robot(0.1)
    q = _point_robot(0.15)
    sc = W.Scene([p, q], np.stack([W.base_transform(0, 0, 0), W.base_transform(0.2, 0, 0)]), Z4, Z6)
    m = oracle_lib.state_margins(sc, np.zeros((1, 2), np.float32))[0]
    assert m == pytest.approx(0.2 - 0.25, abs=1e-7)


def test_nstates_closed_form(oracle_lib):
    qa = np.zeros((5, 3), np.float32)
    qb = np.array([[0, 0, 0], [0.05, 0, 0], [0, -0.5, 0.1], [0.0, 0.0, 0.051], [1.0, 0.0, 0.0]], np.float32)
    n = oracle_lib.edge_nstates(qa, qb, 0.05)
    # n = 1 + ceil(Linf / res) in single precision, n = 1 for a null edge
    want = [1, 1 + math.ceil(np.float32(0.05) / np.float32(0.05)), 1 + 10, 1 + 2, 1 + 20]
    assert list(n) == want


def test_planar_sweep_against_analytic_distance(oracle_lib):
    """A planar 2R arm sweeps joint 1 with joint 2 fixed; its tool sphere moves
    on a circle.  The edge margin must be the minimum, over the discretised
    states, of the closed-form tool-obstacle clearance (the link-1 sphere is
    kept far from the obstacle)."""
    l1, l2, r = 0.6, 0.4, 0.05
    ob = np.array([[0.2, 0.95, 0.0, 0.1]], np.float32)
    sc = W.Scene([W.planar_two_link(l1, l2, r)], W.base_transform(0, 0, 0)[None], ob, Z6)
    qa = np.array([[-0.3, 0.5]], np.float32)
    qb = np.array([[2.2, 0.5]], np.float32)
    res = 0.05
    n, m = oracle_lib.classify_edges(sc, qa, qb, res)
    assert n[0] == 1 + math.ceil(np.float32(2.5) / np.float32(res))
    t = np.arange(n[0]) / (n[0] - 1)
    q1 = qa[0, 0].astype(np.float64) + t * (np.float64(qb[0, 0]) - np.float64(qa[0, 0]))
    q2 = np.float64(qa[0, 1])
    # the model and the obstacle are stored in single precision
    f = lambda v: float(np.float32(v))
    L1, L2, R, ox, oy, orad = f(l1), f(l2), f(r), f(0.2), f(0.95), f(0.1)
    tx = L1 * np.cos(q1) + L2 * np.cos(q1 + q2)
    ty = L1 * np.sin(q1) + L2 * np.sin(q1 + q2)
    mx = f(0.5 * l1) * np.cos(q1)
    my = f(0.5 * l1) * np.sin(q1)
    d_tool = np.hypot(tx - ox, ty - oy) - (R + orad)
    d_mid = np.hypot(mx - ox, my - oy) - (R + orad)
    assert m[0] == pytest.approx(min(d_tool.min(), d_mid.min()), abs=1e-9)


def _tiny_scene(rng, n_rob=2, n_obs=3):
    m = W.panda_like(20)
    b = np.stack([W.base_transform(-0.45 + 0.9 * i, 0, math.pi * i) for i in range(n_rob)])
    sph = np.concatenate([rng.uniform([-0.6, -0.6, 0.1], [0.6, 0.6, 1.0], (n_obs, 3)),
                          rng.uniform(0.05, 0.15, (n_obs, 1))], 1).astype(np.float32)
    c = rng.uniform([-0.6, -0.6, 0.1], [0.6, 0.6, 1.0], (n_obs, 3))
    h = rng.uniform(0.025, 0.15, (n_obs, 3))
    box = np.concatenate([c - h, c + h], 1).astype(np.float32)
    return W.Scene([m] * n_rob, b, sph, box)


def _brute_margin(scene, q):
    """Independent numpy brute force over every pair, given world spheres."""
    import oracle
    w = oracle.fk_spheres(scene, q)[0]
    m = np.inf
    if scene.env_spheres.shape[0]:
        o = scene.env_spheres.astype(np.float64)
        d = np.linalg.norm(w[:, None, :3] - o[None, :, :3], axis=-1) - (w[:, None, 3] + o[None, :, 3])
        m = min(m, d.min())
    if scene.env_boxes.shape[0]:
        b = scene.env_boxes.astype(np.float64)
        lo, hi = b[None, :, :3], b[None, :, 3:]
        c = w[:, None, :3]
        e = np.maximum(np.maximum(lo - c, c - hi), 0.0)
        m = min(m, (np.linalg.norm(e, axis=-1) - w[:, None, 3]).min())
    off = np.cumsum([0] + [mm.n_spheres for mm in scene.models])
    for i in range(scene.n_robots):
        for j in range(i + 1, scene.n_robots):
            a, bb = w[off[i]:off[i + 1]], w[off[j]:off[j + 1]]
            d = np.linalg.norm(a[:, None, :3] - bb[None, :, :3], axis=-1) - (a[:, None, 3] + bb[None, :, 3])
            m = min(m, d.min())
    return m


def test_state_margin_brute_force_tiny(oracle_lib):
    rng = np.random.default_rng(4)
    for _ in range(5):
        sc = _tiny_scene(rng)
        q = W.random_configs(sc, 4, rng)
        got = oracle_lib.state_margins(sc, q)
        for i in range(4):
            assert got[i] == pytest.approx(_brute_margin(sc, q[i:i + 1]), abs=1e-12)


def test_edge_margin_is_min_over_states(oracle_lib):
    rng = np.random.default_rng(5)
    sc = _tiny_scene(rng)
    qa, qb = W.edge_batch(sc, 6, 0.05, 1, 4, 12)
    n, m = oracle_lib.classify_edges(sc, qa, qb, 0.05)
    for e in range(6):
        t = np.arange(n[e]) / max(1, n[e] - 1)
        qs = qa[e].astype(np.float64) + t[:, None] * (qb[e].astype(np.float64) - qa[e].astype(np.float64))
        qs[-1] = qb[e]
        per = [_brute_margin(sc, qs[k:k + 1].astype(np.float32)) for k in range(n[e])]
        # states are rounded to single precision for the numpy brute force
        assert m[e] == pytest.approx(min(per), abs=1e-6)


def test_monotone_in_obstacles_and_radius(oracle_lib):
    rng = np.random.default_rng(6)
    sc = _tiny_scene(rng)
    qa, qb = W.edge_batch(sc, 32, 0.05, 2, 4, 16)
    _, m0 = oracle_lib.classify_edges(sc, qa, qb, 0.05)
    more = sc.with_env(np.concatenate([sc.env_spheres, [[0, 0, 0.5, 0.1]]]).astype(np.float32), sc.env_boxes)
    _, m1 = oracle_lib.classify_edges(more, qa, qb, 0.05)
    assert np.all(m1 <= m0 + 1e-12)
    grown = sc.env_spheres.copy()
    grown[:, 3] += 0.02
    _, m2 = oracle_lib.classify_edges(sc.with_env(grown, sc.env_boxes), qa, qb, 0.05)
    assert np.all(m2 <= m0 + 1e-12)


def test_robot_permutation_and_reversal(oracle_lib):
    rng = np.random.default_rng(7)
    sc = _tiny_scene(rng, 3, 3)
    qa, qb = W.edge_batch(sc, 16, 0.05, 3, 4, 16)
    n, m = oracle_lib.classify_edges(sc, qa, qb, 0.05)
    perm = [2, 0, 1]
    sp = W.Scene([sc.models[i] for i in perm], sc.base_tf[perm], sc.env_spheres, sc.env_boxes)
    cols = np.concatenate([np.arange(7 * i, 7 * i + 7) for i in perm])
    n2, m2 = oracle_lib.classify_edges(sp, qa[:, cols], qb[:, cols], 0.05)
    assert (n2 == n).all()
    np.testing.assert_allclose(m2, m, atol=1e-12)
    n3, m3 = oracle_lib.classify_edges(sc, qb, qa, 0.05)
    assert (n3 == n).all()
    np.testing.assert_allclose(m3, m, atol=1e-9)


def test_far_apart_robots_decouple(oracle_lib):
    """Bases farther apart than twice the reach plus radii: the composite
    margin is the minimum of each robot's env-only margin."""
    rng = np.random.default_rng(8)
    m = W.panda_like(20)
    b = np.stack([W.base_transform(-3, 0, 0), W.base_transform(3, 0, 0)])
    sph = np.array([[-3.3, 0.1, 0.6, 0.1], [3.2, -0.2, 0.5, 0.12]], np.float32)
    sc = W.Scene([m, m], b, sph, Z6)
    q = W.random_configs(sc, 8, rng)
    both = oracle_lib.state_margins(sc, q)
    one = oracle_lib.state_margins(W.Scene([m], b[:1], sph, Z6), q[:, :7])
    two = oracle_lib.state_margins(W.Scene([m], b[1:], sph, Z6), q[:, 7:])
    np.testing.assert_allclose(both, np.minimum(one, two), atol=1e-12)


def test_fast_checker_matches_classification(oracle_lib):
    rng = np.random.default_rng(9)
    for seed in range(3):
        sc = _tiny_scene(rng, 2, 4)
        qa, qb = W.edge_batch(sc, 64, 0.05, seed, 4, 24)
        n, m = oracle_lib.classify_edges(sc, qa, qb, 0.05)
        v, n2, c = oracle_lib.validate_fast(sc, qa, qb, 0.05)
        v2, _, c2 = oracle_lib.validate_fast(sc, qa, qb, 0.05, early_exit=False)
        assert (n2 == n).all()
        assert ((m >= 0) == (v == 1)).all()
        assert (v2 == v).all()
        assert c2["states"] == n.sum() and c["states"] <= c2["states"]


def test_empty_scene_well_separated_all_valid(oracle_lib):
    m = W.panda_like(20)
    sc = W.Scene([m, m], np.stack([W.base_transform(-3, 0, 0), W.base_transform(3, 0, 0)]), Z4, Z6)
    qa, qb = W.edge_batch(sc, 32, 0.05, 0)
    v, _, _ = oracle_lib.validate_fast(sc, qa, qb, 0.05)
    assert v.all()
