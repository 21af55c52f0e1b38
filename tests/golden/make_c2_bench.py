"""Write ``c2_bench.json``: the 4-arm validation workload, selected by the oracle.

Calls only ``workloads`` and ``oracle``.  The file holds:
  * the C2 scene (seed 0) after the obstacles touching start or goal were
    redrawn, and the start/goal pair;
  * the seeds and sizes that regenerate the anchor states and the candidate
    edge pool (``workloads.random_configs`` / ``workloads.edge_batch_near``);
  * the indices of the anchors the oracle finds free, and of the first 4096
    pool edges whose minimum margin is at least the 1e-5 m band (certainly
    free: every state must be fully checked, no early exit);
  * the oracle's pair-test counts over those edges (coarse-to-fine checker,
    no early exit), which give the fine-stage work per state;
  * for the first 4096 pool edges (the unselected batch): the oracle's class
    of each (certainly free, certainly colliding, or within the band).

Run:  python tests/golden/make_c2_bench.py
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

OUT = os.path.join(HERE, "c2_bench.json")
RES = 0.05
N_EDGES = 4096
N_ANCHOR_DRAWS = 8000
POOL = 200000
ANCHOR_SEED = 12
POOL_SEED = 13
N_MIN, N_MAX, SPREAD = 8, 64, 0.02


def main():
    t0 = time.time()
    p = W.make_problem(W.scene_c2(0), 0, oracle.states_free)
    sc = p.scene
    anchors_all = W.random_configs(sc, N_ANCHOR_DRAWS, np.random.default_rng([ANCHOR_SEED]))
    free_idx = np.nonzero(oracle.states_free(sc, anchors_all))[0]
    anchors = anchors_all[free_idx]
    qa, qb = W.edge_batch_near(sc, anchors, POOL, RES, POOL_SEED, N_MIN, N_MAX, spread=SPREAD)
    valid, n, _ = oracle.validate_fast(sc, qa, qb, RES, threads=os.cpu_count() or 1)
    cand = np.nonzero(valid)[0]
    print(f"anchors {len(anchors)}, fast-valid {len(cand)} of {POOL} ({time.time() - t0:.1f}s)", flush=True)
    n_c, m_c = oracle.classify_edges(sc, qa[cand], qb[cand], RES)
    certain = cand[m_c >= oracle.BAND]
    if len(certain) < N_EDGES:
        raise SystemExit(f"only {len(certain)} certainly free edges")
    sel = certain[:N_EDGES]
    _, n_sel, counts = oracle.validate_fast(sc, qa[sel], qb[sel], RES, early_exit=False,
                                            threads=os.cpu_count() or 1)
    mixed_valid = valid[:N_EDGES]
    _, m_mixed = oracle.classify_edges(sc, qa[:N_EDGES], qb[:N_EDGES], RES)
    mixed_cls = oracle.classify(m_mixed)
    doc = {
        "what": "C2 validation workload: 4 arms x 59 spheres, 32 spheres + 32 boxes, res 0.05 rad",
        "scene_seed": 0,
        "env_spheres": sc.env_spheres.astype(float).tolist(),
        "env_boxes": sc.env_boxes.astype(float).tolist(),
        "q_start": p.q_start.astype(float).tolist(),
        "q_goal": p.q_goal.astype(float).tolist(),
        "resolution": RES,
        "anchor_draws": N_ANCHOR_DRAWS, "anchor_seed": ANCHOR_SEED,
        "anchor_free_idx": free_idx.tolist(),
        "pool": POOL, "pool_seed": POOL_SEED, "n_min": N_MIN, "n_max": N_MAX, "spread": SPREAD,
        "free_edge_idx": sel.tolist(),
        "free_edge_states": int(n_sel.sum()),
        "oracle_counts_free_edges": counts,
        "mixed_first_4096_valid": int(mixed_valid.sum()),
        "mixed_first_4096_states": int(n[:N_EDGES].sum()),
        "mixed_first_4096_class": mixed_cls.astype(int).tolist(),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT}: {len(sel)} edges, {int(n_sel.sum())} states ({time.time() - t0:.1f}s)")


if __name__ == "__main__":
    main()
