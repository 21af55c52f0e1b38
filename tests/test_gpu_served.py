"""Serving with continuous batching: requests admitted into running work give
the same results as alone (round budgets), memory admission and rejection,
and the server's bookkeeping."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import problem

pytestmark = pytest.mark.gpu

PARAMS = dict(candidates=64, max_rounds=60, max_iterations=2, n_roadmap=16, delta=3.0, max_tree_nodes=8192,
              max_roadmap_nodes=1024)


@pytest.fixture(scope="module")
def ctx():
    import paper_2609_30644_amd as M
    c = M.Context(0)
    yield c
    c.close()


def _served_instances(min_arms: int, k: int):
    """The first k queries of the served workload with at least min_arms arms."""
    import json
    import os
    from types import SimpleNamespace
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_served.json")))
    out = []
    for x in d["instances"]:
        R = x["n_robots"]
        if R < min_arms:
            continue
        sc = W.Scene([W.panda_like(59)] * R, np.array(x["bases"], np.float32).reshape(R, 12),
                     np.array(x["env_spheres"], np.float32).reshape(-1, 4),
                     np.array(x["env_boxes"], np.float32).reshape(-1, 6))
        out.append(SimpleNamespace(scene=sc, q_start=np.array(x["q_start"], np.float32),
                                   q_goal=np.array(x["q_goal"], np.float32)))
        if len(out) == k:
            break
    return out


def _queries(ctx):
    """Twelve queries over six problems: two- and four-arm problems, the
    eight-arm shelf, and two served queries with at least eight arms."""
    import paper_2609_30644_amd as M
    ps = [problem("c1"), problem("c2"), problem("c3")] + _served_instances(8, 2) + \
        [W.make_problem(W.scene_c1(5), 5, oracle.states_free)]
    scenes = [M.Scene(ctx, p.scene) for p in ps]
    return [(scenes[i % len(ps)], ps[i % len(ps)], dict(PARAMS, seed=i)) for i in range(12)]


def test_served_results_equal_alone(ctx):
    import paper_2609_30644_amd as M
    qs = _queries(ctx)
    srv = M.Server(ctx, max_slots=5)
    print(f"[served] 12 requests ({sorted(set(s.n_robots for s, _, _ in qs))} arms), 5 slots", flush=True)
    # a first wave, then the rest while the first wave runs
    tickets = [srv.submit(s, p.q_start, p.q_goal, **prm) for s, p, prm in qs[:6]]
    tickets += [srv.submit(s, p.q_start, p.q_goal, **prm) for s, p, prm in qs[6:]]
    got = [srv.wait(t, 120.0) for t in tickets]
    st = srv.stats()
    print(f"  stats {st}", flush=True)
    srv.close()
    assert st["completed"] == 12 and st["max_running"] <= 5 and st["max_running"] >= 2
    for k, ((s, p, prm), g) in enumerate(zip(qs, got)):
        ref = s.plan(p.q_start, p.q_goal, raise_on_error=False, **prm)
        assert g["status"] == ref.status, (k, g["status"], ref.status)
        assert g["stats"]["costs"] == ref.stats["costs"] and g["stats"]["rounds"] == ref.stats["rounds"], k
        if ref.status == "OK":
            assert np.array_equal(g["path"], ref.path) and g["cost"] == ref.cost, k
        assert g["t_submit"] <= g["t_admit"] <= g["t_done"], k


def test_served_memory_admission(ctx):
    import paper_2609_30644_amd as M
    qs = _queries(ctx)[:6]
    one = M.Server(ctx, max_slots=8, mem_budget_bytes=1)
    t = one.submit(qs[0][0], qs[0][1].q_start, qs[0][1].q_goal, **qs[0][2])
    r = one.wait(t, 30.0)
    assert r["status"] == "E_NOMEM" and one.stats()["rejected"] == 1
    one.close()
    # a budget that fits two requests at a time: never more than two run
    need = []
    probe = M.Server(ctx, max_slots=1)
    t = probe.submit(qs[0][0], qs[0][1].q_start, qs[0][1].q_goal, **qs[0][2])
    need.append(probe.wait(t, 60.0)["device_bytes"])
    probe.close()
    srv = M.Server(ctx, max_slots=8, mem_budget_bytes=int(2.5 * need[0]))
    same = [(qs[0][0], qs[0][1], dict(qs[0][2], seed=i)) for i in range(6)]
    tickets = [srv.submit(s, p.q_start, p.q_goal, **prm) for s, p, prm in same]
    got = [srv.wait(t, 120.0) for t in tickets]
    st = srv.stats()
    srv.close()
    assert all(g["status"] in ("OK", "E_NO_SOLUTION") for g in got)
    assert st["max_running"] <= 2 and st["peak_reserved_bytes"] <= int(2.5 * need[0])
    # unknown ticket
    srv = M.Server(ctx, max_slots=1)
    with pytest.raises(M.MrpopError):
        srv.poll(12345)
    srv.close()
