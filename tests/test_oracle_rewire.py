"""Pins of the oracle's ao-dRRT baseline (the paper's asymptotically optimal
multi-robot comparison planner, optimising by rewiring instead of AO-X):
tensor-product adjacency, the cheapest parent, rewiring proposals, cost
refresh, one worked round on a planar arm, tree invariants after whole
plans, and the roadmap optimum on an empty scene."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import planner as PL

PARAMS = dict(seed=1, candidates=64, max_rounds=120, max_iterations=4, n_roadmap=32, delta=3.0, rewire=True)


def _roadmap(points, edges):
    rm = PL._Roadmap(np.asarray(points[0], np.float32), np.asarray(points[1], np.float32))
    for q in points[2:]:
        rm.add_vertex(q)
    for a, b in edges:
        rm.add_edge(a, b)
    return rm


def _tree(rows):
    """rows: (q, g, parent, vid)"""
    t = PL._Tree([], [], [], [])
    for q, g, par, vid in rows:
        t.q.append(np.asarray(q, np.float32))
        t.g.append(np.float32(g))
        t.parent.append(par)
        t.vid.append(tuple(vid))
    return t


def test_tensor_product_adjacency():
    a = _roadmap([[0, 0], [5, 5], [1, 0], [2, 0]], [(0, 2), (2, 3)])
    b = _roadmap([[0, 0], [5, 5], [0, 1]], [(0, 2)])
    assert PL.tp_adjacent([a, b], (0, 0), (2, 0))      # arm 0 moves, arm 1 stays
    assert PL.tp_adjacent([a, b], (0, 0), (2, 2))      # both move along edges
    assert not PL.tp_adjacent([a, b], (0, 0), (0, 0))  # the same vertex
    assert not PL.tp_adjacent([a, b], (0, 0), (3, 0))  # 0 - 3 is no edge
    assert not PL.tp_adjacent([a, b], (2, 0), (2, 1))  # 0 - 1 is no edge of arm 1


# planar two-joint arm: start (0, 0), goal (5, 5); roadmap edges 0-2, 2-3, 0-4, 4-3
RM = [[0, 0], [5, 5], [1, 0], [2, 0], [1, 1]]
EDGES = [(0, 2), (2, 3), (0, 4), (4, 3)]


def test_best_parent_and_proposals_closed_form():
    rm = _roadmap(RM, EDGES)
    s2 = math.sqrt(2.0)
    t = _tree([([0, 0], 0.0, -1, (0,)), ([1, 1], s2, 0, (4,)), ([2, 0], 2 * s2, 1, (3,))])
    g, k = PL.best_parent(t, 3, [rm], (2,), np.array([1.0, 0.0]))
    assert (k, g) == (0, pytest.approx(1.0))   # via the root; vertex 2 costs 2 sqrt2 + 1
    props = PL.rewire_proposals(t, 3, [rm], (2,), np.array([1.0, 0.0]), g, k)
    assert props == [(2, pytest.approx(2.0))]  # (2, 0) drops from 2 sqrt2 to 2 through (1, 0)
    assert PL.best_parent(t, 3, [rm], (1,), np.array([5.0, 5.0])) is None  # the goal has no neighbour in T
    # largest drops first, ties to the lower index, at most RW_SLOTS
    # six neighbours at distance exactly 1 with costs 12, 11, 12, 11, 12, 12:
    # drops 11, 10, 11, 10, 11, 11 -> the four of drop 11, lowest index first
    pts = [[1, 0], [0, 1], [-1, 0], [0, -1], [1, 0], [0, 1]]
    rm2 = _roadmap([[0, 0], [9, 9]] + pts, [(0, 2 + j) for j in range(6)])
    t2 = _tree([([0, 0], 0.0, -1, (0,))] + [(pts[j], [12, 11, 12, 11, 12, 12][j], 0, (2 + j,)) for j in range(6)])
    pr = PL.rewire_proposals(t2, 7, [rm2], (0,), np.array([0.0, 0.0]), 0.0, -1)
    assert [z for z, _ in pr] == [1, 3, 5, 6] and all(c == 1.0 for _, c in pr)


def test_refresh_costs_along_chains():
    s2 = math.sqrt(2.0)
    t = _tree([([0, 0], 0.0, -1, (0,)), ([1, 1], s2, 0, (4,)), ([2, 0], 9.0, 1, (3,)), ([3, 0], 9.0, 2, (5,))])
    PL.refresh_costs(t)
    assert float(t.g[2]) == pytest.approx(2 * s2) and float(t.g[3]) == pytest.approx(2 * s2 + 1)
    t.parent[1] = 3  # a cycle 1 -> 3 -> 2 -> 1
    with pytest.raises(RuntimeError):
        PL.refresh_costs(t)


def test_rewire_round_worked_example():
    """The sample (0.6, -0.9) is nearest to the root; dRRT's oracle moves to
    (1, 0) (cosine 0.55; (1, 1) points away); its cheapest parent is the root
    (cost 1); the tree vertex (2, 0), reached through (1, 1) at 2 sqrt2, is
    rewired through the new vertex at cost 2, and the goal tree's root
    connects at 1 + |(5, 5) - (1, 0)|."""
    m = W.planar_two_link()
    sc = W.Scene([m], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    rm = _roadmap(RM, EDGES)
    s2 = math.sqrt(2.0)
    ta = _tree([([0, 0], 0.0, -1, (0,)), ([1, 1], s2, 0, (4,)), ([2, 0], 2 * s2, 1, (3,))])
    tb = _tree([([5, 5], 0.0, -1, (1,))])
    out = PL.rewire_round(oracle.OracleScene(sc), [rm], ta, tb, [(np.array([0.6, -0.9]), math.inf)], math.inf,
                          PL.PlanParams(candidates=1, resolution=0.05, rewire=True),
                          lambda vid: rm.V[vid[0]].astype(np.float32))
    assert [(c[1], c[2]) for c in out.cands] == [(0, (2,))] and out.cands[0][4] == pytest.approx(1.0)
    assert out.proposals == [(0, 2, pytest.approx(2.0))] and out.pvalid == [True]
    assert out.inserted == [(0, 3)] and out.rewired == [(2, 3)]
    assert ta.parent[2] == 3 and float(ta.g[2]) == pytest.approx(2.0)
    assert out.best[0] == pytest.approx(1.0 + math.hypot(4.0, 5.0)) and out.best[2:] == (3, 0)


@pytest.fixture(scope="module")
def c1():
    return W.make_problem(W.scene_c1(0), 0, oracle.states_free)


def _check_tree(t, roadmaps):
    for v in range(1, len(t)):
        p = t.parent[v]
        assert 0 <= p < len(t) and PL.tp_adjacent(roadmaps, t.vid[p], t.vid[v])
        chain, u = 0, v
        cost = 0.0
        while t.parent[u] >= 0:
            cost += float(np.linalg.norm(t.q[u].astype(np.float64) - t.q[t.parent[u]].astype(np.float64)))
            u = t.parent[u]
            chain += 1
            assert chain <= len(t)
        assert u == 0 and float(t.g[v]) == pytest.approx(cost, rel=1e-6, abs=1e-6)


def test_rewire_plan_invariants(c1):
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    assert r.status == "OK" and len(r.costs) >= 2
    path = r.path
    assert np.array_equal(path[0], c1.q_start) and np.array_equal(path[-1], c1.q_goal)
    _, m = oracle.classify_edges(c1.scene, path[:-1], path[1:], 0.05)
    assert np.all(m >= 0)
    assert float(np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1).sum()) == \
        pytest.approx(r.cost, rel=1e-12)
    assert all(b < a for a, b in zip(r.costs, r.costs[1:]))
    for t in r.trees:
        _check_tree(t, r.roadmaps)
    # the trees persist across searches: the last search's trees hold more
    # vertices than any one search of AO-X's fresh trees would start with
    assert len(r.trees[0]) + len(r.trees[1]) > 2


def test_rewire_empty_scene_reaches_roadmap_optimum():
    """As for AO-X: one arm, no obstacles, the search ends at the cheapest
    path over the roadmap, start -> v -> goal through a neighbour v of the
    start or the goal."""
    sc = W.Scene([W.panda_like(20)], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32),
                 np.zeros((0, 6), np.float32))
    rng = np.random.default_rng(3)
    qs = W.random_configs(sc, 1, rng)[0]
    step = rng.uniform(-1, 1, sc.dof).astype(np.float32)
    step *= 1.0 / np.abs(step).max()
    qg = np.clip(qs + step, sc.q_lo, sc.q_hi).astype(np.float32)
    r = PL.plan(sc, qs, qg, PL.PlanParams(seed=2, candidates=32, max_rounds=80, max_iterations=3, n_roadmap=16,
                                           delta=3.0, rewire=True))
    assert r.status == "OK"
    rm = r.roadmaps[0]
    s64, g64 = qs.astype(np.float64), qg.astype(np.float64)
    best = min(np.linalg.norm(rm.V[v].astype(np.float64) - s64) + np.linalg.norm(rm.V[v].astype(np.float64) - g64)
               for v in set(rm.adj[0]) | set(rm.adj[1]))
    assert r.cost == pytest.approx(best, rel=1e-6)


# the worked example with a second candidate: (1.5, 0.9), a neighbour of the
# root and of (2, 0), also proposes to rewire (2, 0), at 1.749 + 1.030
RM2 = RM + [[1.5, 0.9]]
EDGES2 = EDGES + [(0, 5), (5, 3)]
BLOCK = [-0.0855, 1.0766, 0.0, 0.05]  # a sphere on the sweep of the edge (1, 0) -> (2, 0) only


def _two_candidate_round(env):
    m = W.planar_two_link()
    sc = W.Scene([m], W.base_transform(0, 0, 0)[None], np.array(env, np.float32).reshape(-1, 4),
                 np.zeros((0, 6), np.float32))
    rm = _roadmap(RM2, EDGES2)
    s2 = math.sqrt(2.0)
    ta = _tree([([0, 0], 0.0, -1, (0,)), ([1, 1], s2, 0, (4,)), ([2, 0], 2 * s2, 1, (3,))])
    tb = _tree([([5, 5], 0.0, -1, (1,))])
    draws = [(np.array([0.6, -0.9]), math.inf), (np.array([0.3, 0.18]), math.inf)]
    out = PL.rewire_round(oracle.OracleScene(sc), [rm], ta, tb, draws, math.inf,
                          PL.PlanParams(candidates=2, resolution=0.05, rewire=True),
                          lambda vid: rm.V[vid[0]].astype(np.float32))
    return sc, out, ta


def test_rewire_keeps_the_cheapest_proposal():
    """Both new vertices propose (2, 0): candidate 0 at 2.0, candidate 1 at
    |(1.5, 0.9)| + |(0.5, -0.9)|; the later, dearer proposal must not
    replace the earlier one."""
    _, out, ta = _two_candidate_round(np.zeros((0, 4)))
    c1 = math.hypot(1.5, 0.9) + math.hypot(0.5, 0.9)
    assert [(i, z) for i, z, _ in out.proposals] == [(0, 2), (1, 2)]
    assert out.proposals[1][2] == pytest.approx(c1) and c1 < 2 * math.sqrt(2.0)
    assert out.inserted == [(0, 3), (1, 4)] and out.rewired == [(2, 3)]
    assert ta.parent[2] == 3 and float(ta.g[2]) == pytest.approx(2.0)


def test_rewire_needs_a_free_edge():
    """With a sphere on the sweep of (1, 0) -> (2, 0), candidate 0's proposal
    fails its edge check, and (2, 0) is rewired through candidate 1."""
    sc, out, ta = _two_candidate_round([BLOCK])
    qa = np.array([[0, 0], [1, 1], [0, 0], [0, 0], [1.5, 0.9], [1, 0]], np.float32)
    qb = np.array([[1, 1], [2, 0], [1, 0], [1.5, 0.9], [2, 0], [2, 0]], np.float32)
    _, m = oracle.classify_edges(sc, qa, qb, 0.05)
    assert np.all(m[:-1] > 1e-3) and m[-1] < -1e-3  # only the last edge collides
    assert out.pvalid == [False, True] and out.rewired == [(2, 4)]
    assert ta.parent[2] == 4 and float(ta.g[2]) == pytest.approx(math.hypot(1.5, 0.9) + math.hypot(0.5, 0.9))


def test_parent_is_cheapest_neighbour_not_nearest():
    """The sample lies next to (1, -1), which the tree reaches at cost 5, so
    that vertex is the nearest; the extension to (2, 0) takes (1, 1), cost
    sqrt2, as its parent instead."""
    m = W.planar_two_link()
    sc = W.Scene([m], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    rm = _roadmap([[0, 0], [5, 5], [1, 1], [1, -1], [2, 0]], [(0, 2), (0, 3), (2, 4), (3, 4)])
    s2 = math.sqrt(2.0)
    ta = _tree([([0, 0], 0.0, -1, (0,)), ([1, 1], s2, 0, (2,)), ([1, -1], 5.0, 0, (3,))])
    tb = _tree([([5, 5], 0.0, -1, (1,))])
    out = PL.rewire_round(oracle.OracleScene(sc), [rm], ta, tb, [(np.array([1.3, -0.7]), math.inf)], math.inf,
                          PL.PlanParams(candidates=1, resolution=0.05, rewire=True),
                          lambda vid: rm.V[vid[0]].astype(np.float32))
    assert oracle.nearest(np.array(ta.q[:3]), np.array(ta.g[:3]), np.array([1.3, -0.7], np.float32), math.inf) == 2
    assert [(c[1], c[2]) for c in out.cands] == [(1, (4,))] and out.cands[0][4] == pytest.approx(2 * s2)


def test_trees_persist_across_searches(c1):
    """After each improvement the next search starts from the grown trees
    (AO-X would start from the two roots)."""
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**PARAMS))
    solves = [k for _, _, k in r.history][:-1]
    assert solves
    by_round = {rnd: na + nb for rnd, _, na, nb in r.trace}
    assert all(by_round[k + 1] > 2 for k in solves if k + 1 in by_round)
    fresh = PL.plan(c1.scene, c1.q_start, c1.q_goal, PL.PlanParams(**dict(PARAMS, rewire=False)))
    by_round_f = {rnd: na + nb for rnd, _, na, nb in fresh.trace}
    assert all(by_round_f[k + 1] == 2 for _, _, k in fresh.history[:-1] if k + 1 in by_round_f)
