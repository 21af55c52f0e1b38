"""Writes c1_problems.json: the 50 two-arm planning problems of the
time-to-solution benchmark (seeds 0-49, the size of the paper's problem
sets): 2 arms x 20 spheres with bases 1 m apart, 16 random spheres, res
0.05 rad.

Start/goal are drawn by workloads.make_problem with the oracle as the
collision checker (obstacles touching them are moved or dropped); the file
stores the resulting scenes so that the benchmark needs neither the oracle
nor the generator at run time.  Run from the repository root:

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

N_PROBLEMS = 50


def f32(a):
    """Shortest decimal text of each single-precision value (reads back exactly)."""
    a = np.asarray(a, np.float32)
    return [f32(x) for x in a] if a.ndim else float(str(a))


def main() -> None:
    out = {"what": "C1: 2 arms x 20 spheres, bases 1 m apart, 16 spheres; seeds 0-49", "resolution": 0.05,
           "problems": []}
    for seed in range(N_PROBLEMS):
        p = W.make_problem(W.scene_c1(seed), seed, oracle.states_free)
        out["problems"].append({"seed": seed, "env_spheres": f32(p.scene.env_spheres.reshape(-1)),
                                "env_boxes": f32(p.scene.env_boxes.reshape(-1)), "q_start": f32(p.q_start),
                                "q_goal": f32(p.q_goal), "dropped_obstacles": int(p.dropped_obstacles)})
    with open(os.path.join(HERE, "c1_problems.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {len(out['problems'])} problems")


if __name__ == "__main__":
    main()
