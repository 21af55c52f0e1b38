"""Pins of the oracle planner's AO-X steps (Alg. 2; Sec. "Converge to
Global Optimality"): the cost coordinate c_rand, the informed draw clamped
onto the joint box, ORACLE_AOX's admissible-first choice, the connection
budget c_best - g_new, and the smaller-tree rule.  Each pin is a closed form,
a distribution test or a hand-built tree/roadmap whose answer is worked out
by hand in the test."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W
from oracle import planner as PL


@pytest.fixture(scope="module")
def c1():
    return W.make_problem(W.scene_c1(0), 0, oracle.states_free)


# --------------------------------------------------------------------------
# c_rand ~ U[g(q_rand), c_best]
# --------------------------------------------------------------------------

def test_cost_coordinate_closed_form():
    assert PL.cost_coordinate(1.0, 3.0, 0.0) == 1.0
    assert PL.cost_coordinate(1.0, 3.0, 0.5) == 2.0
    assert PL.cost_coordinate(1.0, 3.0, 0.75) == 2.5
    assert PL.cost_coordinate(4.0, 3.0, 0.3) == 3.0  # lower bound above c_best: c_best itself


@pytest.mark.parametrize("root_is_goal", [False, True])
def test_cost_coordinate_uniform_between_bound_and_incumbent(c1, root_is_goal):
    """Over the candidates of a round, c_rand lies in [|q_rand - root|,
    c_best] and (c_rand - lb) / (c_best - lb) is uniform on [0, 1); the bound
    is measured to the root of the extended tree (the goal after a swap)."""
    sc = c1.scene
    lo, hi = sc.q_lo.astype(np.float64), sc.q_hi.astype(np.float64)
    qs, qg = c1.q_start, c1.q_goal
    cmin = float(np.linalg.norm(qg.astype(np.float64) - qs))
    c_best = 1.6 * cmin
    root = (qg if root_is_goal else qs).astype(np.float64)
    t = []
    for i in range(3000):
        q, c = PL.draw_candidate(5, 3, i, c_best, lo, hi, qs, qg, root)
        lb = float(np.linalg.norm(q - root))
        assert lb <= c_best * (1 + 1e-12)
        assert lb - 1e-12 <= c <= c_best
        t.append((c - lb) / (c_best - lb))
    assert stats.kstest(np.array(t), "uniform").pvalue > 1e-3


def test_initial_solve_draw_is_uniform_in_box_with_infinite_budget(c1):
    sc = c1.scene
    lo, hi = sc.q_lo.astype(np.float64), sc.q_hi.astype(np.float64)
    q = np.array([PL.draw_candidate(2, 0, i, math.inf, lo, hi, c1.q_start, c1.q_goal, c1.q_start)[0]
                  for i in range(2000)])
    cs = {PL.draw_candidate(2, 0, i, math.inf, lo, hi, c1.q_start, c1.q_goal, c1.q_start)[1] for i in range(5)}
    assert cs == {math.inf}
    u = (q - lo) / (hi - lo)
    assert u.min() >= 0 and u.max() < 1
    for j in (0, 5, 13):
        assert stats.kstest(u[:, j], "uniform").pvalue > 1e-3


# --------------------------------------------------------------------------
# informed draw clamped onto the joint box
# --------------------------------------------------------------------------

def test_informed_draw_stays_in_box_and_focal_set(c1):
    sc = c1.scene
    lo, hi = sc.q_lo.astype(np.float64), sc.q_hi.astype(np.float64)
    qs, qg = c1.q_start.astype(np.float64), c1.q_goal.astype(np.float64)
    c_best = 2.5 * float(np.linalg.norm(qg - qs))
    clamped = 0
    for i in range(1000):
        q, _ = PL.draw_candidate(7, 1, i, c_best, lo, hi, c1.q_start, c1.q_goal, qs)
        assert np.all(q >= lo) and np.all(q <= hi)
        assert np.linalg.norm(q - qs) + np.linalg.norm(q - qg) <= c_best * (1 + 1e-9)
        clamped += int(np.any(q == lo) or np.any(q == hi))
    assert clamped > 0  # the hyperspheroid sticks out of the box here


def test_informed_draw_clamp_2d_closed_form():
    """Box [-1, 1] x [-0.5, 0.5], foci (-0.5, 0) and (0.5, 0), c_best = 2: the
    ellipse has semi-axes a = 1, b = sqrt(3)/2, so only y can leave the box.
    Points inside the strip |y| < 0.5 are kept as drawn (a share
    2 (tau sqrt(1 - tau^2) + asin tau) / pi of the ellipse's area,
    tau = 0.5 / b), the others land on y = +-0.5 with x unchanged."""
    lo, hi = np.array([-1.0, -0.5]), np.array([1.0, 0.5])
    qs, qg = np.array([-0.5, 0.0], np.float32), np.array([0.5, 0.0], np.float32)
    b = math.sqrt(3.0) / 2.0
    tau = 0.5 / b
    share = 2.0 * (tau * math.sqrt(1 - tau * tau) + math.asin(tau)) / math.pi
    n, inside, on_face = 20000, 0, 0
    for i in range(n):
        q, _ = PL.draw_candidate(11, 0, i, 2.0, lo, hi, qs, qg, qs.astype(np.float64))
        if abs(q[1]) < 0.5:
            inside += 1
        else:
            assert abs(q[1]) == 0.5
            on_face += 1
        assert abs(q[0]) <= 1.0 and (q[0] / 1.0) ** 2 + (min(abs(q[1]), b) / b) ** 2 <= 1 + 1e-9
    sigma = math.sqrt(share * (1 - share) / n)
    assert abs(inside / n - share) < 5 * sigma
    assert on_face == n - inside > 0


# --------------------------------------------------------------------------
# ORACLE_AOX: admissible neighbours first, then the best aligned
# --------------------------------------------------------------------------

def _roadmap(points, edges):
    rm = PL._Roadmap(np.asarray(points[0], np.float32), np.asarray(points[1], np.float32))
    for q in points[2:]:
        rm.add_vertex(q)
    for a, b in edges:
        rm.add_edge(a, b)
    return rm


def test_aox_oracle_picks_best_aligned_admissible_neighbour():
    """Vertex 0 at the origin; neighbour 1 at (2, 0) is the best aligned with
    the sample (5, 0.5) but costs 2 to reach, neighbour 2 at (0.5, 0.5)
    costs sqrt(0.5).  Budget 1: only vertex 2 is admissible and is taken
    (choosing the best aligned first and then dropping the candidate as
    inadmissible would give no extension at all).  No budget: vertex 1.
    Budget 0.5: nothing admissible, the arm stays."""
    rm = _roadmap([[0, 0], [2, 0], [0.5, 0.5]], [(0, 1), (0, 2)])
    s = [np.array([5.0, 0.5])]
    assert PL.aox_oracle([rm], (0,), s, 0.0, 1.0) == [2]
    assert PL.aox_oracle([rm], (0,), s) == [1]
    assert PL.aox_oracle([rm], (0,), s, 0.0, 0.5) == [0]
    # the cost-to-come of the near vertex counts: g_near 0.4 + sqrt(0.5) >= 1.1
    assert PL.aox_oracle([rm], (0,), s, 0.4, 1.1) == [0]
    assert PL.aox_oracle([rm], (0,), s, 0.3, 1.1) == [2]
    # strict: g_near + |u - v| == c_rand is not admissible
    assert PL.aox_oracle([rm], (0,), s, 0.0, 2.0) == [2]
    assert PL.aox_oracle([rm], (0,), s, 0.0, 2.0000001) == [1]


def test_aox_oracle_composite_budget_reverts_least_aligned_arm():
    """Two arms, each with one neighbour at distance 1 from the origin; arm 0
    is better aligned (cos 0.995) than arm 1 (cos 0.894).  Each move fits a
    budget of 1.2 alone but together they cost sqrt(2): arm 1 goes back to
    staying.  A budget of 1.5 keeps both; equal cosines revert the higher arm
    first."""
    a0 = _roadmap([[0, 0], [9, 9], [1, 0]], [(0, 2)])
    a1 = _roadmap([[0, 0], [9, 9], [0, 1]], [(0, 2)])
    s = [np.array([1.0, 0.1]), np.array([0.5, 1.0])]
    assert PL.aox_oracle([a0, a1], (0, 0), s, 0.0, 1.2) == [2, 0]
    assert PL.aox_oracle([a0, a1], (0, 0), s, 0.0, 1.5) == [2, 2]
    assert PL.aox_oracle([a0, a1], (0, 0), s) == [2, 2]
    eq = [np.array([1.0, 0.5]), np.array([0.5, 1.0])]
    assert PL.aox_oracle([a0, a1], (0, 0), eq, 0.0, 1.2) == [2, 0]
    # the reverted set never leaves the candidate inadmissible
    for c in np.linspace(1.01, 1.6, 25):
        vid = PL.aox_oracle([a0, a1], (0, 0), s, 0.0, float(c))
        moved = sum(1 for r in range(2) if vid[r] != 0)
        assert moved >= 1 and math.sqrt(moved) < c


def test_drrt_oracle_is_aox_without_budget():
    rm = _roadmap([[0, 0], [1, 0], [0, 1], [-1, 0], [0.7, 0.7]], [(0, 1), (0, 2), (0, 3), (0, 4)])
    rng = np.random.default_rng(0)
    for _ in range(50):
        q = rng.normal(size=2)
        assert PL.drrt_oracle([rm], (0,), None, [q]) == PL.aox_oracle([rm], (0,), [q], 0.0, math.inf)


# --------------------------------------------------------------------------
# connection budget and the round
# --------------------------------------------------------------------------

def _planar_round(c_best, draw):
    """One search round on a planar two-link arm in an empty scene: T_a = {the
    start (0, 0)}, T_b = {the goal (2, 0)}, roadmap edge start - (0, 1)."""
    m = W.planar_two_link()
    sc = W.Scene([m], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    rm = _roadmap([[0, 0], [2, 0], [0, 1]], [(0, 2)])
    ta = PL._new_tree(np.array([0, 0], np.float32), (0,))
    tb = PL._new_tree(np.array([2, 0], np.float32), (1,))
    params = PL.PlanParams(candidates=1, resolution=0.05)
    out = PL.search_round(oracle.OracleScene(sc), [rm], ta, tb, [draw], c_best, params,
                          lambda vid: rm.V[vid[0]].astype(np.float32))
    return out, ta


def test_connection_budget_excludes_paths_not_cheaper():
    """The sample (0, 2) with c_rand 2.4 extends the start tree to (0, 1)
    (g_new = 1).  With c_best 2.5 the connection budget is 1.5 < |(0, 1) -
    (2, 0)| = sqrt(5): no connection is even tried.  With c_best 3.3 the
    budget 2.3 admits the goal and the connection of total cost 1 + sqrt(5)
    is the round's result."""
    assert PL.connect_budget(2.5, 1.0) == 1.5 and PL.connect_budget(math.inf, 1.0) == math.inf
    draw = (np.array([0.0, 2.0]), 2.4)
    out, ta = _planar_round(2.5, draw)
    assert [c[2] for c in out.cands] == [(2,)] and out.valid == [True]
    assert out.inserted == [(0, 1)] and float(ta.g[1]) == pytest.approx(1.0)
    assert out.conns == [] and out.best is None
    out, _ = _planar_round(3.3, draw)
    assert out.conns == [(0, 1, 0)] and out.cvalid == [True]
    assert out.best[0] == pytest.approx(1.0 + math.sqrt(5.0), rel=1e-9)


def test_round_nearest_respects_sample_budget():
    """NEAREST is bounded by c_rand as well: the sample (0, 2) with c_rand
    1.9 admits no vertex (0 + 2 >= 1.9), so nothing is extended."""
    out, ta = _planar_round(2.5, (np.array([0.0, 2.0]), 1.9))
    assert out.cands == [] and len(ta) == 1


def test_smaller_tree_is_extended(c1):
    """needs_swap, and its trace through a plan: every round extends a tree
    no larger than the other, and the start tree is not always the one
    extended."""
    t1, t2 = PL._new_tree(np.zeros(2, np.float32), (0,)), PL._new_tree(np.ones(2, np.float32), (1,))
    assert not PL.needs_swap(t1, t2)
    t1.q.append(np.zeros(2, np.float32))
    assert PL.needs_swap(t1, t2) and not PL.needs_swap(t2, t1)
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal,
                PL.PlanParams(seed=1, candidates=64, max_rounds=60, max_iterations=2, n_roadmap=32, delta=3.0))
    assert r.trace and all(na <= nb for _, _, na, nb in r.trace)
    assert any(not a_is_start for _, a_is_start, _, _ in r.trace)
    assert any(na < nb for _, _, na, nb in r.trace)


# --------------------------------------------------------------------------
# the outer loop (Alg. 1) around ROADMAP and the searches
# --------------------------------------------------------------------------

def test_no_search_until_roadmaps_connect(c1):
    """Two samples per growth round, one growth round per iteration: the
    roadmaps stay unconnected for four iterations, so no search round runs,
    and every iteration grows each arm by two vertices."""
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal,
                PL.PlanParams(seed=1, candidates=64, max_rounds=40, max_iterations=4, n_roadmap=2, delta=3.0,
                              max_growth_rounds=1))
    assert not any(m.connected() for m in r.roadmaps)
    assert (r.status, r.rounds, r.iterations, r.trace) == ("E_NO_SOLUTION", 0, 4, [])
    assert [len(m.V) for m in r.roadmaps] == [2 + 4 * 2] * 2


def test_full_tree_restarts_the_search(c1):
    """With room for three vertices per tree, the first round's free
    extensions overflow T_a: the search ends there and every further
    iteration starts over from the two roots; no path is found and the
    result says the capacity was the limit."""
    r = PL.plan(c1.scene, c1.q_start, c1.q_goal,
                PL.PlanParams(seed=1, candidates=64, max_rounds=12, max_iterations=6, n_roadmap=32, delta=3.0,
                              max_tree_nodes=3))
    assert (r.status, r.rounds, r.iterations) == ("E_CAPACITY", 6, 6)
    assert [(na, nb) for _, _, na, nb in r.trace] == [(1, 1)] * 6
