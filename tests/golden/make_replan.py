"""Writes replan_ticks.json: the replanning workload (two arms of the C1 kind
and one sphere moving through the workspace, one position per tick).

The problem is workloads.make_problem on scene_c1(0) with the oracle as the
collision checker.  The moving sphere's straight track crosses, at its
middle tick, the position of an arm sphere at the middle waypoint of the
oracle planner's path (so that the obstacle sweeps through the region the
plans use); its direction is drawn from a seeded generator and kept only when
the oracle finds the start and the goal free at every tick.  The benchmark
needs neither the oracle nor the generator at run time.  Run from the
repository root:

    python tests/golden/make_replan.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_TICKS = 30
RADIUS = 0.1
SPEED = 0.04  # metres per tick


def f32(a):
    """Shortest decimal text of each single-precision value (reads back exactly)."""
    a = np.asarray(a, np.float32)
    return [f32(x) for x in a] if a.ndim else float(str(a))


def main() -> None:
    from oracle import planner as PL
    p = W.make_problem(W.scene_c1(0), 0, oracle.states_free)
    ends = np.stack([p.q_start, p.q_goal])
    r = PL.plan(p.scene, p.q_start, p.q_goal, PL.PlanParams(seed=1, candidates=64, max_rounds=120,
                                                             max_iterations=2, n_roadmap=32, delta=3.0))
    mid = r.path[len(r.path) // 2]
    centres = oracle.fk_spheres(p.scene, mid[None])[0]
    rng = np.random.default_rng([8, 0])
    for attempt in range(200):
        through = centres[rng.integers(len(centres)), :3]
        v = rng.normal(size=3)
        v *= SPEED / np.linalg.norm(v)
        track = [through + v * (t - N_TICKS // 2) for t in range(N_TICKS)]
        ok = True
        for c in track:
            sph = np.concatenate([p.scene.env_spheres, [[*c, RADIUS]]]).astype(np.float32)
            if not oracle.states_free(p.scene.with_env(sph, p.scene.env_boxes), ends).all():
                ok = False
                break
        if ok:
            break
    else:
        raise RuntimeError("no track keeps the endpoints free")
    out = {"scene": "c1/0", "env_spheres": f32(p.scene.env_spheres), "env_boxes": f32(p.scene.env_boxes),
           "q_start": f32(p.q_start), "q_goal": f32(p.q_goal), "radius": RADIUS, "attempt": attempt,
           "ticks": [f32(c) for c in track]}
    with open(os.path.join(HERE, "replan_ticks.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("track attempt", attempt, flush=True)


if __name__ == "__main__":
    main()
