"""mrpop_plan_batch: many independent instances in shared launches.  Each
instance must return exactly what mrpop_plan returns for it alone (same
parameters, round budgets): the batch changes when work runs, not what it
computes."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import problem

pytestmark = pytest.mark.gpu

PARAMS = dict(candidates=64, max_rounds=60, max_iterations=3, n_roadmap=16, delta=3.0, max_tree_nodes=8192,
              max_roadmap_nodes=1024)

_cache = {}


def _problems():
    if "p" not in _cache:
        ps = [problem("c1"), problem("c2")]
        for s in (1, 2, 3):
            ps.append(W.make_problem(W.scene_c1(s), s, oracle.states_free))
        three = W.Scene([W.panda_like(20)] * 3, W.ring_bases(3, W.ring_radius_for_spacing(3, 1.1)),
                        np.array([[0.0, 0.0, 0.9, 0.12]], np.float32), np.zeros((0, 6), np.float32))
        ps.append(W.make_problem(three, 4, oracle.states_free))
        _cache["p"] = ps
    return _cache["p"]


@pytest.fixture(scope="module")
def ctx():
    import paper_2609_30644_amd as M
    c = M.Context(0)
    yield c
    c.close()


def test_batch_equals_plain(ctx):
    import paper_2609_30644_amd as M
    ps = _problems()
    scenes = [M.Scene(ctx, p.scene) for p in ps]
    jobs = []
    for i, (p, s) in enumerate(zip(ps, scenes)):
        for seed in (0, 7):
            jobs.append((s, p.q_start, p.q_goal, dict(PARAMS, seed=seed + i)))
    print(f"[batch] {len(jobs)} instances", flush=True)
    got, bst = ctx.plan_batch(jobs)
    print(f"  batch stats {bst}", flush=True)
    for k, ((s, qs, qg, prm), g) in enumerate(zip(jobs, got)):
        ref = s.plan(qs, qg, raise_on_error=False, **prm)
        assert g.status == ref.status, (k, g.status, ref.status)
        assert g.stats["rounds"] == ref.stats["rounds"] and g.stats["edge_states"] == ref.stats["edge_states"], k
        assert g.stats["costs"] == ref.stats["costs"], (k, g.stats["costs"], ref.stats["costs"])
        if ref.status == "OK":
            assert np.array_equal(g.path, ref.path) and g.cost == ref.cost, k
    assert sum(g.status == "OK" for g in got) >= len(got) // 2


def test_batch_reports_each_instance(ctx):
    import paper_2609_30644_amd as M
    p = problem("c1")
    s = M.Scene(ctx, p.scene)
    sph = np.concatenate([p.scene.env_spheres, [[-0.5, 0.0, 0.2, 0.2]]]).astype(np.float32)
    blocked = M.Scene(ctx, p.scene.with_env(sph, p.scene.env_boxes))
    bad = p.q_start.copy()
    bad[0] = np.nan
    jobs = [(s, p.q_start, p.q_goal, dict(PARAMS, seed=1)), (blocked, p.q_start, p.q_goal, dict(PARAMS, seed=1)),
            (s, bad, p.q_goal, dict(PARAMS, seed=1)), (s, p.q_start, p.q_goal, dict(PARAMS, seed=1, candidates=0))]
    got, bst = ctx.plan_batch(jobs)
    assert [g.status for g in got] == ["OK", "E_START_INVALID", "E_NONFINITE", "E_INVALID_ARG"]
    assert bst["instances"] == 4 and bst["solved"] == 1
    # tiny path buffer: status and the required length
    got, _ = ctx.plan_batch(jobs[:1], path_cap=1)
    assert got[0].status == "E_BUFFER" and got[0].stats["path_len"] >= 2
    # empty batch
    got, bst = ctx.plan_batch([])
    assert got == [] and bst["instances"] == 0
