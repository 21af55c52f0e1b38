"""Writes c4_batch.json: planning instances of the batched workload
(independent problems with 2-8 arms of 59 spheres, 16-256 sphere or cuboid
obstacles, per-instance edge resolution delta / (m - 1) with m ~ U{8..256}
states per roadmap-length edge).

Start/goal are drawn by workloads.make_problem with the oracle as the
collision checker (obstacles touching them are moved or dropped); the file
stores the resulting scenes so that the benchmark needs neither the oracle
nor the generator at run time.  Run from the repository root:

    python tests/golden/make_c4_batch.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_INSTANCES = 512
SEED = 0
DELTA = 3.0


def f32(a):
    """Shortest decimal text of each single-precision value (reads back exactly)."""
    a = np.asarray(a, np.float32)
    return [f32(x) for x in a] if a.ndim else float(str(a))


def main() -> None:
    out = {"seed": SEED, "delta": DELTA, "instances": []}
    for i in range(N_INSTANCES):
        sc = W.scene_c4(SEED, i)
        p = W.make_problem(sc, i, oracle.states_free)
        m = int(np.random.default_rng([44, SEED, i]).integers(8, 257))
        out["instances"].append({
            "index": i,
            "n_robots": len(sc.models),
            "bases": f32(p.scene.base_tf),
            "env_spheres": f32(p.scene.env_spheres),
            "env_boxes": f32(p.scene.env_boxes),
            "q_start": f32(p.q_start),
            "q_goal": f32(p.q_goal),
            "resolution": float(np.float32(DELTA / (m - 1))),
            "dropped_obstacles": p.dropped_obstacles,
        })
        print(i, len(sc.models), len(p.scene.env_spheres) + len(p.scene.env_boxes), flush=True)
    with open(os.path.join(HERE, "c4_batch.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
