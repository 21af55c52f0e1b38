"""Pins of the oracle planner (Alg. 1 / Alg. 2 in rounds): invariants of
every returned path, the dRRT oracle on hand-built roadmaps, roadmap
invariants checked by independent means, and a closed-form convergence case."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import planner as PL
from gpu_common import blocking_obstacle

PARAMS = dict(seed=1, candidates=64, max_rounds=120, max_iterations=4, n_roadmap=32, delta=3.0)


@pytest.fixture(scope="module")
def c1():
    return W.make_problem(W.scene_c1(0), 0, oracle.states_free)


def test_plan_path_invariants(c1):
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    assert r.status == "OK"
    path = r.path
    assert np.array_equal(path[0], c1.q_start) and np.array_equal(path[-1], c1.q_goal)
    _, m = oracle.classify_edges(c1.scene, path[:-1], path[1:], 0.05)
    assert np.all(m >= 0)
    cost = float(np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1).sum())
    assert cost == pytest.approx(r.cost, rel=1e-12)
    assert cost >= float(np.linalg.norm(c1.q_goal.astype(np.float64) - c1.q_start))
    assert all(b < a for a, b in zip(r.costs, r.costs[1:]))
    assert r.first_round >= 0 and r.edge_states > 0


def test_plan_deterministic(c1):
    a = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    b = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    assert np.array_equal(a.path, b.path) and a.costs == b.costs


def test_plan_start_in_collision(c1):
    sph = np.concatenate([c1.scene.env_spheres, [[-0.5, 0.0, 0.2, 0.2]]]).astype(np.float32)
    r = PL.plan(c1.scene.with_env(sph, c1.scene.env_boxes), c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    assert r.status == "E_START_INVALID"


def test_empty_scene_single_arm_reaches_roadmap_optimum():
    """One arm, no obstacles: every edge is free, so after the last search
    has run out of rounds without improving, the incumbent is the cheapest
    path available, start -> v -> goal over a roadmap neighbour v of the start
    or of the goal (any longer chain is no shorter by the triangle
    inequality)."""
    m = W.panda_like(20)
    sc = W.Scene([m], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    rng = np.random.default_rng(3)
    qs = W.random_configs(sc, 1, rng)[0]
    step = rng.uniform(-1, 1, sc.dof).astype(np.float32)
    step *= 1.0 / np.abs(step).max()
    qg = np.clip(qs + step, sc.q_lo, sc.q_hi).astype(np.float32)
    r = PL.plan(sc, qs, qg, PL.PlanParams(seed=2, candidates=64, max_rounds=300, max_iterations=3, n_roadmap=16,
                                           delta=3.0))
    assert r.status == "OK" and not r.last_search_solved
    rm = r.roadmaps[0]
    s64, g64 = qs.astype(np.float64), qg.astype(np.float64)
    best = min(np.linalg.norm(rm.V[v].astype(np.float64) - s64) + np.linalg.norm(rm.V[v].astype(np.float64) - g64)
               for v in set(rm.adj[0]) | set(rm.adj[1]))
    assert r.cost == pytest.approx(best, rel=1e-6)
    assert r.cost > float(np.linalg.norm(g64 - s64))


def _line_roadmap(points):
    rm = PL._Roadmap(np.asarray(points[0], np.float32), np.asarray(points[1], np.float32))
    for q in points[2:]:
        rm.add_vertex(q)
    return rm


def test_drrt_oracle_best_aligned_and_stay():
    # one planar-ish arm (2 joints): neighbours of vertex 0 in three directions
    rm = _line_roadmap([[0, 0], [1, 0], [0, 1], [-1, 0], [0.7, 0.7]])
    for u in (1, 2, 3, 4):
        rm.add_edge(0, u)
    # sample toward +x: vertex 1 (cos 1)
    assert PL.drrt_oracle([rm], (0,), None, [np.array([3.0, 0.2])]) == [1]
    # sample along the diagonal: vertex 4
    assert PL.drrt_oracle([rm], (0,), None, [np.array([1.0, 1.0])]) == [4]
    # no neighbour with a positive cosine: stay
    rm2 = _line_roadmap([[0, 0], [1, 0]])
    rm2.add_edge(0, 1)
    assert PL.drrt_oracle([rm2], (0,), None, [np.array([-1.0, 0.0])]) == [0]
    # sample at the vertex itself: stay
    assert PL.drrt_oracle([rm2], (0,), None, [np.array([0.0, 0.0])]) == [0]
    # equal cosines: the lower neighbour id
    rm3 = _line_roadmap([[0, 0], [2, 0], [1, 0]])
    rm3.add_edge(0, 1)
    rm3.add_edge(0, 2)
    assert PL.drrt_oracle([rm3], (0,), None, [np.array([5.0, 0.0])]) == [1]


def test_roadmap_invariants(c1):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    sc = c1.scene
    q_off = [0, 7, 14]
    arms = [oracle.OracleScene(PL._arm_scene(sc, r)) for r in range(2)]
    rms = [PL._Roadmap(c1.q_start[q_off[r]:q_off[r + 1]], c1.q_goal[q_off[r]:q_off[r + 1]]) for r in range(2)]
    params = PL.PlanParams(n_roadmap=16, delta=3.0, max_growth_rounds=4)
    PL.roadmap_step(sc, rms, arms, params, 0, q_off)
    sizes = [len(rm.V) for rm in rms]
    PL.roadmap_step(sc, rms, arms, params, 1, q_off)
    for r, rm in enumerate(rms):
        assert len(rm.V) > sizes[r]  # roadmaps persist and grow across calls
        V = np.array(rm.V)
        assert np.all(oracle.state_margins(arms[r], V) >= 0)  # every vertex free of the environment
        edges = [(a, b) for a in range(len(V)) for b in rm.adj[a] if a < b]
        qa = np.array([V[a] for a, _ in edges], np.float32)
        qb = np.array([V[b] for _, b in edges], np.float32)
        assert np.all(np.linalg.norm(qa.astype(np.float64) - qb, axis=1) <= params.delta + 1e-6)
        _, m = oracle.classify_edges(arms[r], qa, qb, params.resolution)
        assert np.all(m >= 0)
        # BFS connectivity agrees with connected components of the same graph
        ii = np.array([a for a, _ in edges] + [b for _, b in edges])
        jj = np.array([b for _, b in edges] + [a for a, _ in edges])
        g = coo_matrix((np.ones(len(ii)), (ii, jj)), shape=(len(V), len(V)))
        _, lab = connected_components(g, directed=False)
        assert rm.connected() == (lab[0] == lab[1])


def test_incumbent_history_ranked_seeds(c1):
    """Seeding (Sec. "Seeding for Multi-Robot Jerk-Free Motion"): every
    improved path is kept with its cost; ranked cheapest first, a prefix of
    that ranking when fewer seeds are wanted.  Each entry is checked by means
    independent of the planner: endpoints, the checker, the FP64 cost of its
    waypoints."""
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    assert r.status == "OK" and len(r.history) == len(r.costs) >= 2
    costs = [c for c, _, _ in r.history]
    assert costs == r.costs and all(b < a for a, b in zip(costs, costs[1:]))
    assert np.array_equal(r.history[-1][1], r.path)
    rounds = [k for _, _, k in r.history]
    assert rounds == sorted(rounds)
    for cost, path, _ in r.history:
        assert np.array_equal(path[0], c1.q_start) and np.array_equal(path[-1], c1.q_goal)
        _, m = oracle.classify_edges(c1.scene, path[:-1], path[1:], 0.05)
        assert np.all(m >= 0)
        assert float(np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1).sum()) == \
            pytest.approx(cost, rel=1e-12)
    ranked = PL.ranked_history(r)
    assert [e[0] for e in ranked] == sorted(costs)
    two = PL.ranked_history(r, 2)
    assert [e[0] for e in two] == sorted(costs)[:2] and np.array_equal(two[0][1], r.path)


def test_steer_closed_form():
    """Direct-mode extension: within `step` the sample itself; beyond it the
    point at distance exactly `step` on the segment toward the sample."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        a = rng.uniform(-2, 2, 7)
        b = a + rng.normal(size=7) * rng.uniform(0.01, 3.0)
        step = float(rng.uniform(0.05, 2.0))
        q = PL.steer(a, b, step)
        dist = float(np.linalg.norm(b - a))
        if dist <= step:
            assert np.array_equal(q, b)
        else:
            assert float(np.linalg.norm(q - a)) == pytest.approx(step, rel=1e-12)
            assert float(np.linalg.norm(b - q)) == pytest.approx(dist - step, rel=1e-9, abs=1e-12)
            assert float(np.dot(q - a, b - a)) == pytest.approx(step * dist, rel=1e-12)
    z = np.ones(7)
    assert np.array_equal(PL.steer(z, z, 0.5), z)


@pytest.fixture(scope="module")
def single():
    return W.make_problem(W.scene_single(0), 0, oracle.states_free)


DIRECT = dict(seed=3, candidates=64, max_rounds=150, max_iterations=4, direct=True, step=1.0)


def test_direct_plan_single_arm(single):
    """Direct mode on one arm: no roadmap grows; the returned path obeys the
    path invariants, and every edge but the one connection is a tree edge no
    longer than `step`."""
    r = PL.plan(single.scene, single.q_start, single.q_goal, PL.PlanParams(**DIRECT))
    assert r.status == "OK"
    assert all(len(rm.V) == 2 for rm in r.roadmaps)
    path = r.path
    assert np.array_equal(path[0], single.q_start) and np.array_equal(path[-1], single.q_goal)
    _, m = oracle.classify_edges(single.scene, path[:-1], path[1:], 0.05)
    assert np.all(m >= 0)
    steps = np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1)
    assert float(steps.sum()) == pytest.approx(r.cost, rel=1e-12)
    assert int((steps > DIRECT["step"] * (1 + 1e-6)).sum()) <= 1
    assert all(b < a for a, b in zip(r.costs, r.costs[1:])) and len(r.costs) >= 2
    again = PL.plan(single.scene, single.q_start, single.q_goal, PL.PlanParams(**DIRECT))
    assert np.array_equal(again.path, r.path)


def test_direct_empty_scene_first_solution_closed_form():
    """One arm, no obstacles: round 0 extends every sample from the start and
    connects it straight to the goal, so the first solution is
    start -> steer(start, q_rand_i) -> goal for the candidate i with the
    least cost (recomputed here from the same streams), and the costs that
    follow stay above the straight line."""
    from oracle import key, u01
    sc = W.Scene([W.panda_like(20)], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32),
                 np.zeros((0, 6), np.float32))
    rng = np.random.default_rng(11)
    qs, qg = W.random_configs(sc, 2, rng)
    prm = dict(seed=4, candidates=32, max_rounds=60, max_iterations=3, direct=True, step=0.7)
    r = PL.plan(sc, qs, qg, PL.PlanParams(**prm))
    assert r.status == "OK" and r.first_round == 0
    lo, hi = sc.q_lo.astype(np.float64), sc.q_hi.astype(np.float64)
    best = None
    for i in range(prm["candidates"]):
        q_rand = lo + u01(key(prm["seed"], PL.PURPOSE_Q, 0, i), sc.dof) * (hi - lo)
        qn = PL.steer(qs.astype(np.float64), q_rand, prm["step"]).astype(np.float32).astype(np.float64)
        tot = float(np.linalg.norm(qn - qs) + np.linalg.norm(qg - qn))
        if best is None or tot < best[0]:
            best = (tot, qn)
    first_cost, first_path, _ = r.history[0]
    assert len(first_path) == 3 and np.array_equal(first_path[1].astype(np.float64), best[1])
    assert first_cost == pytest.approx(best[0], rel=1e-6)
    line = float(np.linalg.norm(qg.astype(np.float64) - qs))
    assert all(c >= line * (1 - 1e-12) for c in r.costs) and r.costs[-1] < first_cost


def test_replan_keeps_free_incumbent_and_drops_blocked(c1):
    """Replanning tick (Sec. "Hardware Deployment"): an unchanged environment
    keeps the previous path as the incumbent (the result is never worse); an
    obstacle on the path discards it and the new path avoids the obstacle; a
    path that does not run start -> goal is not kept."""
    prm = PL.PlanParams(**PARAMS)
    r0 = PL.plan(c1.scene, c1.q_start, c1.q_goal, prm)
    assert r0.status == "OK"
    r1, kept = PL.replan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**dict(PARAMS, seed=7)), r0.path)
    assert kept and r1.status == "OK" and r1.cost <= r0.cost
    if not r1.history:
        assert np.array_equal(r1.path, r0.path)
    blocked = blocking_obstacle(c1, r0.path)
    _, m = oracle.classify_edges(blocked, r0.path[:-1], r0.path[1:], 0.05)
    assert m.min() < 0
    r2, kept2 = PL.replan(blocked, c1.q_start, c1.q_goal, prm, r0.path)
    assert not kept2
    if r2.status == "OK":
        _, m2 = oracle.classify_edges(blocked, r2.path[:-1], r2.path[1:], 0.05)
        assert np.all(m2 >= 0)
    _, kept3 = PL.replan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**dict(PARAMS, max_rounds=1)),
                         r0.path[::-1])
    assert not kept3
