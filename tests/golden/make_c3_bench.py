"""Write ``c3_bench.json``: the 8-arm shelf validation workload, selected by the oracle.

Calls only ``workloads`` and ``oracle``.  The file holds:
  * the C3 scene (seed 0: 8 arms x 59 spheres on a 1.5 m circle around a
    4 x 8 x 8 shelf grid of boxes) and a start/goal pair: each arm's start
    and goal drawn uniformly in its limits among states at least 2 cm clear
    of the boxes, the composite states free of contact between arms, and an
    arm's pair redrawn until the oracle's roadmap growth (the planner's
    random streams for seed 0: 32 samples per growth round, delta 3 rad,
    0.02 rad, at most 12 rounds) joins its start and goal;
  * the seeds and sizes that regenerate the anchor states and the candidate
    edge pool (``workloads.random_configs`` / ``workloads.edge_batch_near``;
    0.02 rad resolution, 8 to 256 states per edge);
  * the indices of the anchors the oracle finds free, and of the first 4096
    pool edges whose minimum margin is at least the 1e-5 m band (certainly
    free: every state must be fully checked);
  * for the first 4096 pool edges (the unselected batch): their state counts
    and the oracle's class of each (certainly free, certainly colliding, or
    within the band).

Run:  python tests/golden/make_c3_bench.py
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

OUT = os.path.join(HERE, "c3_bench.json")
RES = 0.02
N_EDGES = 4096
N_ANCHOR_DRAWS = 20000
POOL = 120000
ANCHOR_SEED = 22
POOL_SEED = 23
N_MIN, N_MAX, SPREAD = 8, 256, 0.02


CLEARANCE = 0.02
RM_ROUNDS = 12
RM_PARAMS = dict(seed=0, n_roadmap=32, delta=3.0, max_growth_rounds=RM_ROUNDS, resolution=RES)


def connectable_problem(sc, seed):
    """Start and goal per arm (see the module docstring)."""
    from oracle import planner as PL
    rng = np.random.default_rng([31, seed])
    R = sc.n_robots
    arms = [oracle.OracleScene(PL._arm_scene(sc, r)) for r in range(R)]
    q_off = np.concatenate([[0], np.cumsum([m.n_joints for m in sc.models])]).astype(int)

    def draw(r):
        m = sc.models[r]
        while True:
            q = (m.q_lo + rng.random((64, m.n_joints)) * (m.q_hi - m.q_lo)).astype(np.float32)
            ok = np.nonzero(oracle.state_margins(arms[r], q) >= CLEARANCE)[0]
            if len(ok) >= 2:
                return q[ok[0]], q[ok[1]]

    qs = np.zeros(sc.dof, np.float32)
    qg = np.zeros(sc.dof, np.float32)
    none4, none6 = np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32)

    def pair_free(r, k):  # arms r and k apart at both the start and the goal
        two = W.Scene([sc.models[r], sc.models[k]], sc.base_tf[[r, k]], none4, none6)
        sl = lambda q, i: q[q_off[i]:q_off[i + 1]]
        q = np.stack([np.concatenate([sl(qs, r), sl(qs, k)]), np.concatenate([sl(qg, r), sl(qg, k)])])
        return bool(oracle.states_free(two, q).all())

    redraw = list(range(R))
    for attempt in range(40):
        placed = [r for r in range(R) if r not in redraw]
        for r in redraw:
            for _ in range(1000):
                qs[q_off[r]:q_off[r + 1]], qg[q_off[r]:q_off[r + 1]] = draw(r)
                if all(pair_free(r, k) for k in placed):
                    break
            else:
                raise SystemExit(f"arm {r}: no start/goal apart from the other arms")
            placed.append(r)
        assert oracle.states_free(sc, np.stack([qs, qg])).all()
        rms = [PL._Roadmap(qs[q_off[r]:q_off[r + 1]], qg[q_off[r]:q_off[r + 1]]) for r in range(R)]
        PL.roadmap_step(sc, rms, arms, PL.PlanParams(**RM_PARAMS), 0, q_off)  # a plan's first iteration
        redraw = [r for r, rm in enumerate(rms) if not rm.connected()]
        print(f"attempt {attempt}: unconnected arms {redraw}", flush=True)
        if not redraw:
            return qs, qg
    raise SystemExit("no connectable start/goal")


def main():
    t0 = time.time()
    th = os.cpu_count() or 1
    sc = W.scene_c3(0)
    q_start, q_goal = connectable_problem(sc, 0)
    print(f"problem ({time.time() - t0:.1f}s)", flush=True)
    anchors_all = W.random_configs(sc, N_ANCHOR_DRAWS, np.random.default_rng([ANCHOR_SEED]))
    free_idx = np.nonzero(oracle.states_free(sc, anchors_all))[0]
    anchors = anchors_all[free_idx]
    print(f"anchors {len(anchors)} of {N_ANCHOR_DRAWS} ({time.time() - t0:.1f}s)", flush=True)
    qa, qb = W.edge_batch_near(sc, anchors, POOL, RES, POOL_SEED, N_MIN, N_MAX, spread=SPREAD)
    valid, n, _ = oracle.validate_fast(sc, qa, qb, RES, threads=th)
    cand = np.nonzero(valid)[0]
    print(f"fast-valid {len(cand)} of {POOL} ({time.time() - t0:.1f}s)", flush=True)
    _, m_c = oracle.classify_edges(sc, qa[cand], qb[cand], RES, threads=th)
    certain = cand[m_c >= oracle.BAND]
    if len(certain) < N_EDGES:
        raise SystemExit(f"only {len(certain)} certainly free edges")
    sel = certain[:N_EDGES]
    _, m_mixed = oracle.classify_edges(sc, qa[:N_EDGES], qb[:N_EDGES], RES, threads=th)
    cls = oracle.classify(m_mixed)
    doc = {
        "what": "C3 validation workload: 8 arms x 59 spheres, 256 shelf boxes, res 0.02 rad",
        "scene_seed": 0,
        "env_spheres": sc.env_spheres.astype(float).tolist(),
        "env_boxes": sc.env_boxes.astype(float).tolist(),
        "q_start": q_start.astype(float).tolist(),
        "q_goal": q_goal.astype(float).tolist(),
        "start_goal_clearance": CLEARANCE, "roadmap_check": RM_PARAMS,
        "resolution": RES,
        "anchor_draws": N_ANCHOR_DRAWS, "anchor_seed": ANCHOR_SEED,
        "anchor_free_idx": free_idx.tolist(),
        "pool": POOL, "pool_seed": POOL_SEED, "n_min": N_MIN, "n_max": N_MAX, "spread": SPREAD,
        "free_edge_idx": sel.tolist(),
        "free_edge_states": int(n[sel].sum()),
        "mixed_first_4096_states": int(n[:N_EDGES].sum()),
        "mixed_first_4096_class": cls.astype(int).tolist(),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT}: {len(sel)} free edges ({int(n[sel].sum())} states), mixed: "
          f"{int((cls == 1).sum())} free, {int((cls == 0).sum())} band ({time.time() - t0:.1f}s)")


if __name__ == "__main__":
    main()
