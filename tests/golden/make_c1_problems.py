"""Writes c1_problems.json: the 50 two-arm planning problems of the
time-to-solution benchmark (the size of the paper's problem sets): 2 arms x
20 spheres with bases 1 m apart, 16 random spheres, res 0.05 rad.

Start/goal are drawn by workloads.make_problem with the oracle as the
collision checker (obstacles touching them are moved or dropped).  Like the
paper's benchmark sets, every problem is solvable: seeds are taken in order
and a problem is kept when the oracle planner finds a path for it within
SOLVE_CHECK (a start or goal sealed off from the other by obstacles is
dropped); the skipped seeds are listed.  The file stores the resulting
scenes so that the benchmark needs neither the oracle nor the generator at
run time.  Run from the repository root:

    python tests/golden/make_c1_problems.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import planner as PL  # noqa: E402

N_PROBLEMS = 50
# the solvability check: AO-X's initial solve, two roadmap iterations
SOLVE_CHECK = dict(candidates=128, n_roadmap=32, delta=3.0, max_rounds=400, max_iterations=2, stop_at_first=True)


def f32(a):
    """Shortest decimal text of each single-precision value (reads back exactly)."""
    a = np.asarray(a, np.float32)
    return [f32(x) for x in a] if a.ndim else float(str(a))


def main() -> None:
    out = {"what": "C1: 2 arms x 20 spheres, bases 1 m apart, 16 spheres; solvable problems, seeds in order",
           "resolution": 0.05, "solve_check": SOLVE_CHECK, "skipped_seeds": [], "problems": []}
    seed = 0
    while len(out["problems"]) < N_PROBLEMS:
        p = W.make_problem(W.scene_c1(seed), seed, oracle.states_free)
        r = PL.plan(p.scene, p.q_start, p.q_goal, PL.PlanParams(**dict(SOLVE_CHECK, seed=seed, resolution=0.05)))
        if r.status == "OK":
            out["problems"].append({"seed": seed, "env_spheres": f32(p.scene.env_spheres.reshape(-1)),
                                    "env_boxes": f32(p.scene.env_boxes.reshape(-1)), "q_start": f32(p.q_start),
                                    "q_goal": f32(p.q_goal), "dropped_obstacles": int(p.dropped_obstacles)})
        else:
            out["skipped_seeds"].append(seed)
        print(f"seed {seed}: {r.status}", flush=True)
        seed += 1
    with open(os.path.join(HERE, "c1_problems.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {len(out['problems'])} problems, skipped seeds {out['skipped_seeds']}")


if __name__ == "__main__":
    main()
