"""Writes c5_served.json: the problems of the served workload (independent
queries with 2-16 arms of 59 spheres and 32-512 sphere or cuboid obstacles;
the served benchmark cycles through them with a new seed per query).

Start/goal are drawn by workloads.make_problem with the oracle as the
collision checker (obstacles touching them are moved or dropped).  A problem
is kept only when the oracle's roadmap growth (the served queries' roadmap
settings: 16 samples per growth round, delta 3 rad, 0.05 rad, at most 16
rounds, seed 0) joins every arm's start and goal, as a start or goal sealed
off from the other makes a query unsolvable; the skipped scene indices are
listed.  The file stores the scenes so that the benchmark needs neither the
oracle nor the generator at run time.  Run from the repository root:

    python tests/golden/make_c5_served.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import planner as PL  # noqa: E402

N_INSTANCES = 32
SEED = 0
RM_PARAMS = dict(seed=0, n_roadmap=16, delta=3.0, max_growth_rounds=16, resolution=0.05)


def roadmaps_connect(p) -> bool:
    """The oracle's ROADMAP (one call) joins every arm's start and goal."""
    sc = p.scene
    R = sc.n_robots
    q_off = np.concatenate([[0], np.cumsum([m.n_joints for m in sc.models])]).astype(int)
    arms = [oracle.OracleScene(PL._arm_scene(sc, r)) for r in range(R)]
    rms = [PL._Roadmap(p.q_start[q_off[r]:q_off[r + 1]], p.q_goal[q_off[r]:q_off[r + 1]]) for r in range(R)]
    return PL.roadmap_step(sc, rms, arms, PL.PlanParams(**RM_PARAMS), 0, q_off)


def f32(a):
    """Shortest decimal text of each single-precision value (reads back exactly)."""
    a = np.asarray(a, np.float32)
    return [f32(x) for x in a] if a.ndim else float(str(a))


def main() -> None:
    out = {"seed": SEED, "roadmap_check": RM_PARAMS, "skipped_indices": [], "instances": []}
    i = 0
    while len(out["instances"]) < N_INSTANCES:
        t0 = time.time()
        sc = W.scene_c5(SEED, i)
        p = W.make_problem(sc, i, oracle.states_free)
        if not roadmaps_connect(p):
            print(i, len(sc.models), "skipped: a roadmap left start and goal apart", flush=True)
            out["skipped_indices"].append(i)
            i += 1
            continue
        out["instances"].append({
            "index": i,
            "n_robots": len(sc.models),
            "bases": f32(p.scene.base_tf),
            "env_spheres": f32(p.scene.env_spheres),
            "env_boxes": f32(p.scene.env_boxes),
            "q_start": f32(p.q_start),
            "q_goal": f32(p.q_goal),
            "dropped_obstacles": p.dropped_obstacles,
        })
        print(i, len(sc.models), len(p.scene.env_spheres) + len(p.scene.env_boxes), f"{time.time() - t0:.1f}s",
              flush=True)
        i += 1
    with open(os.path.join(HERE, "c5_served.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
