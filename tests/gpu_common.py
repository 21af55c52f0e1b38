"""Helpers shared by the GPU tests: one library context per session, seeded
scenes whose start/goal were checked by the oracle, and parity asserts."""
import functools

import numpy as np

import oracle
import workloads as W

BAND = oracle.BAND


@functools.lru_cache(maxsize=None)
def problem(kind: str, seed: int = 0):
    fn = {"c1": W.scene_c1, "c2": W.scene_c2, "c3": W.scene_c3}[kind]
    return W.make_problem(fn(seed), seed, oracle.states_free)


def assert_bits_match(valid_gpu: np.ndarray, margins: np.ndarray, what: str = "") -> dict:
    """GPU bits must equal the oracle's verdict on every edge outside the
    boundary band |m| < BAND; returns the band count and agreement stats."""
    cls = oracle.classify(margins)
    certain = cls != 0
    want = (cls == 1).astype(np.uint8)
    bad = np.nonzero(certain & (valid_gpu != want))[0]
    assert bad.size == 0, (f"{what}: {bad.size} certain edges disagree, e.g. edge {bad[:5]} "
                           f"margins {margins[bad[:5]]} gpu {valid_gpu[bad[:5]]}")
    return {"edges": int(valid_gpu.size), "band": int((~certain).sum()), "valid": int(want.sum())}


def blocking_obstacle(problem, path):
    """A sphere placed on one arm sphere at a middle waypoint of `path` (so
    the path collides), chosen so that the start and goal stay free."""
    sc = problem.scene
    for k in (len(path) // 2, 1, len(path) - 2):
        centres = oracle.fk_spheres(sc, path[k][None])[0]
        for s in range(len(centres) - 1, -1, -1):
            sph = np.concatenate([sc.env_spheres, [[*centres[s, :3], 0.06]]]).astype(np.float32)
            blocked = sc.with_env(sph, sc.env_boxes)
            if oracle.states_free(blocked, np.stack([problem.q_start, problem.q_goal])).all():
                return blocked
    raise AssertionError("no blocking obstacle that leaves the endpoints free")
