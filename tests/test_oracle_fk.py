"""Pins of the oracle's forward kinematics against closed forms and
invariants that do not come from the oracle itself."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.parametrize("_", [0])  # keep ids short


def _single(model, base=None, env_s=None, env_b=None):
    base = W.base_transform(0, 0, 0) if base is None else base
    return W.Scene([model], base[None], np.zeros((0, 4), np.float32) if env_s is None else env_s,
                   np.zeros((0, 6), np.float32) if env_b is None else env_b)


def _probe_model(links, points):
    """Panda kinematics with probe spheres at given link-local points."""
    m = W.panda_like(59)
    return W.RobotModel("probe", m.dh, m.q_lo, m.q_hi, np.array(links, np.int32),
                        np.array([[*p, 0.01] for p in points], np.float32))


def test_planar_two_link_closed_form(_, oracle_lib):
    l1, l2 = 0.6, 0.4
    sc = _single(W.planar_two_link(l1, l2))
    rng = np.random.default_rng(0)
    q = rng.uniform(-math.pi, math.pi, size=(50, 2)).astype(np.float32)
    out = oracle_lib.fk_spheres(sc, q)
    q64 = q.astype(np.float64)
    tool_x = l1 * np.cos(q64[:, 0]) + l2 * np.cos(q64[:, 0] + q64[:, 1])
    tool_y = l1 * np.sin(q64[:, 0]) + l2 * np.sin(q64[:, 0] + q64[:, 1])
    np.testing.assert_allclose(out[:, 1, 0], tool_x, atol=1e-6)
    np.testing.assert_allclose(out[:, 1, 1], tool_y, atol=1e-6)
    np.testing.assert_allclose(out[:, 1, 2], 0.0, atol=1e-12)
    np.testing.assert_allclose(out[:, 0, 0], 0.5 * l1 * np.cos(q64[:, 0]), atol=1e-6)


def test_panda_zero_pose_by_hand(_, oracle_lib):
    # Joint origins at q = 0, composed by hand from the kinematic table:
    # shoulder (0,0,0.333), elbow (0,0,0.649) then (0.0825,0,0.649),
    # wrist (0,0,1.033), frame 7 at (0.088,0,1.033); flange 0.107 m below it.
    pts = [(0, 0, 0)] * 8 + [(0, 0, 0.107)]
    links = [0, 1, 2, 3, 4, 5, 6, 7, 7]
    sc = _single(_probe_model(links, pts))
    out = oracle_lib.fk_spheres(sc, np.zeros(7, np.float32))[0, :, :3]
    want = [(0, 0, 0), (0, 0, 0.333), (0, 0, 0.333), (0, 0, 0.649), (0.0825, 0, 0.649),
            (0, 0, 1.033), (0, 0, 1.033), (0.088, 0, 1.033), (0.088, 0, 0.926)]
    np.testing.assert_allclose(out, np.array(want), atol=2e-7)


def test_panda_single_joint_rotations(_, oracle_lib):
    sc = _single(_probe_model([7, 3], [(0, 0, 0.107), (0, 0, 0)]))
    # q1 = +pi/2 turns the whole arm about the base z axis.
    q = np.zeros(7, np.float32)
    q[0] = math.pi / 2
    out = oracle_lib.fk_spheres(sc, q)[0, :, :3]
    np.testing.assert_allclose(out[0], (0.0, 0.088, 0.926), atol=2e-7)
    # q2 = +pi/2 pitches the upper arm forward (+x): elbow at (0.316, 0, 0.333).
    q = np.zeros(7, np.float32)
    q[1] = math.pi / 2
    out = oracle_lib.fk_spheres(sc, q)[0, :, :3]
    np.testing.assert_allclose(out[1], (0.316, 0.0, 0.333), atol=2e-7)


def test_rigidity_and_proximal_links_fixed(_, oracle_lib):
    m = W.panda_like(59)
    sc = _single(m)
    rng = np.random.default_rng(1)
    q = W.random_configs(sc, 20, rng)
    out = oracle_lib.fk_spheres(sc, q)[:, :, :3]
    for l in range(8):
        idx = np.nonzero(m.sphere_link == l)[0]
        d = np.linalg.norm(out[:, idx[:, None], :] - out[:, idx[None, :], :], axis=-1)
        np.testing.assert_allclose(d, np.broadcast_to(d[0], d.shape), atol=1e-9)
    # moving joint j leaves links 0..j-1 where they were
    for j in range(7):
        q2 = q.copy()
        q2[:, j] += 0.3
        out2 = oracle_lib.fk_spheres(sc, q2)[:, :, :3]
        prox = m.sphere_link < j + 1
        np.testing.assert_allclose(out2[:, prox], out[:, prox], atol=1e-12)
        if j < 6:  # link 7's spheres lie on joint 7's axis and do not move with it
            assert np.abs(out2[:, ~prox] - out[:, ~prox]).max() > 1e-3


def test_base_equivariance(_, oracle_lib):
    m = W.panda_like(20)
    rng = np.random.default_rng(2)
    q = W.random_configs(_single(m), 10, rng)
    x, y, yaw = 0.7, -0.3, 2.1
    out0 = oracle_lib.fk_spheres(_single(m), q)[:, :, :3]
    out1 = oracle_lib.fk_spheres(_single(m, W.base_transform(x, y, yaw)), q)[:, :, :3]
    c, s = math.cos(yaw), math.sin(yaw)
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    np.testing.assert_allclose(out1, out0 @ Rz.T + np.array([x, y, 0]), atol=1e-6)


def test_composite_is_per_robot(_, oracle_lib):
    m = W.panda_like(20)
    b = np.stack([W.base_transform(-0.5, 0, 0), W.base_transform(0.5, 0, math.pi)])
    sc = W.Scene([m, m], b, np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    rng = np.random.default_rng(3)
    q = W.random_configs(sc, 5, rng)
    both = oracle_lib.fk_spheres(sc, q)
    r0 = oracle_lib.fk_spheres(_single(m, b[0]), q[:, :7])
    r1 = oracle_lib.fk_spheres(_single(m, b[1]), q[:, 7:])
    np.testing.assert_allclose(both[:, :20], r0, atol=1e-12)
    np.testing.assert_allclose(both[:, 20:], r1, atol=1e-12)
