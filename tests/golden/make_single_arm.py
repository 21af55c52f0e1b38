"""Writes single_arm.json: the direct-mode workload (one 59-sphere arm among
12 spheres and 12 cuboids, workloads.scene_single), several scenes with one
start/goal each.

Start/goal are drawn by workloads.make_problem with the oracle as the
collision checker (obstacles touching them are moved or dropped); the file
stores the resulting scenes so that the benchmark needs neither the oracle
nor the generator at run time.  Run from the repository root:

    python tests/golden/make_single_arm.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_PROBLEMS = 16


def f32(a):
    """Shortest decimal text of each single-precision value (reads back exactly)."""
    a = np.asarray(a, np.float32)
    return [f32(x) for x in a] if a.ndim else float(str(a))


def main() -> None:
    out = {"problems": []}
    for i in range(N_PROBLEMS):
        p = W.make_problem(W.scene_single(i), i, oracle.states_free)
        out["problems"].append({
            "scene_seed": i,
            "env_spheres": f32(p.scene.env_spheres),
            "env_boxes": f32(p.scene.env_boxes),
            "q_start": f32(p.q_start),
            "q_goal": f32(p.q_goal),
            "dropped_obstacles": p.dropped_obstacles,
        })
        print(i, len(p.scene.env_spheres) + len(p.scene.env_boxes), p.dropped_obstacles, flush=True)
    with open(os.path.join(HERE, "single_arm.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
