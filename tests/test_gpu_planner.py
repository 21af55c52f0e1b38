"""HIP planner and search primitives through the C ABI, checked against the
oracle: NEAREST and the samples element by element, plans by re-validation
of every returned edge, recomputed costs and the invariants of Alg. 1/2."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import BAND, assert_bits_match, blocking_obstacle, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2609_30644_amd as M
    c = M.Context(0)
    yield c
    c.close()


def _scene(ctx, sc):
    import paper_2609_30644_amd as M
    return M.Scene(ctx, sc)


# --------------------------------------------------------------------------
# NEAREST
# --------------------------------------------------------------------------

def test_nearest_matches_oracle(ctx):
    print("[nearest] random", flush=True)
    rng = np.random.default_rng(0)
    for N, D, M in ((1, 3, 5), (17, 7, 64), (3000, 28, 300), (5000, 56, 100)):
        V = rng.normal(size=(N, D)).astype(np.float32)
        g = rng.uniform(0, 4, N).astype(np.float32)
        Q = rng.normal(size=(M, D)).astype(np.float32)
        c = rng.uniform(1, 12, M).astype(np.float32)
        c[::7] = np.inf
        got = ctx.nearest(V, g, Q, c).cpu().numpy()
        want = oracle.nearest_batch(V, g, Q, c.astype(np.float64))
        # exact equality except where the best and second-best candidates are
        # within single-precision rounding of each other
        for i in np.nonzero(got != want)[0]:
            d = np.sqrt(((Q[i].astype(np.float64) - V.astype(np.float64)) ** 2).sum(1))
            ok = g.astype(np.float64) + d < c[i]
            assert got[i] >= 0 and want[i] >= 0, (i, got[i], want[i])
            assert abs(d[got[i]] - d[want[i]]) < 1e-5 * max(1.0, d[want[i]]), (i, d[got[i]], d[want[i]])
            assert ok[got[i]] or abs(g[got[i]] + d[got[i]] - c[i]) < 1e-5 * c[i]


def test_nearest_ties_budget_and_empty(ctx):
    V = np.array([[1, 0], [1, 0], [0, 1], [5, 5]], np.float32)
    g = np.array([2.0, 1.0, 1.0, 0.0], np.float32)
    Q = np.zeros((4, 2), np.float32)
    c = np.array([np.inf, 2.0, 2.1, 7.1], np.float32)
    got = ctx.nearest(V, g, Q, c).cpu().numpy().tolist()
    assert got == [1, -1, 1, 1]
    assert ctx.nearest(V[3:], g[3:], Q[:1], np.array([7.0], np.float32)).cpu().numpy().tolist() == [-1]
    assert ctx.nearest(np.zeros((0, 2), np.float32), None, Q[:2], None).cpu().numpy().tolist() == [-1, -1]
    # no costs means all zero: the plain nearest vertex (ties to lower index)
    assert ctx.nearest(V, None, Q[:1], None).cpu().numpy().tolist() == [0]


# --------------------------------------------------------------------------
# Samples (INFORMED_SAMPLE and c_rand)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("informed", [False, True])
def test_sample_matches_oracle(ctx, informed):
    print(f"[sample] informed={informed}", flush=True)
    p = problem("c2")
    sc = p.scene
    s = _scene(ctx, sc)
    straight = float(np.linalg.norm(p.q_goal.astype(np.float64) - p.q_start))
    c_best = 1.4 * straight if informed else math.inf
    root = p.q_goal if informed else p.q_start
    n = 257
    q, c = s.sample(p.q_start, p.q_goal, root, c_best, seed=11, round_=5, n=n, first=3)
    q, c = q.cpu().numpy().astype(np.float64), c.cpu().numpy().astype(np.float64)
    from oracle.planner import draw_candidate  # the oracle's candidate draw, pinned on the CPU
    lo, hi = sc.q_lo.astype(np.float64), sc.q_hi.astype(np.float64)
    for i in range(n):
        wq, wc = draw_candidate(11, 5, 3 + i, c_best, lo, hi, p.q_start, p.q_goal, root.astype(np.float64))
        np.testing.assert_allclose(q[i], wq, atol=2e-5 * max(1.0, c_best if informed else 1.0), rtol=0)
        if informed:
            assert abs(c[i] - wc) <= 2e-5 * c_best
            lb = np.linalg.norm(q[i] - root)
            assert lb - 1e-4 <= c[i] <= c_best * (1 + 1e-6)
            assert (np.linalg.norm(q[i] - p.q_start) + np.linalg.norm(q[i] - p.q_goal)) <= c_best * (1 + 1e-5)
        else:
            assert math.isinf(c[i])
        assert np.all(q[i] >= sc.q_lo - 1e-6) and np.all(q[i] <= sc.q_hi + 1e-6)


# --------------------------------------------------------------------------
# Plans
# --------------------------------------------------------------------------

PARAMS = dict(seed=1, candidates=64, max_rounds=150, max_iterations=4, n_roadmap=32, delta=3.0)


class PlanResultLike:
    """A path with its cost in the shape _check_path reads."""

    def __init__(self, path, cost, stats):
        self.path, self.cost, self.stats = path, cost, stats


def _check_path(sc, res, q_start, q_goal, params):
    path = res.path
    assert path is not None and len(path) >= 2
    assert np.array_equal(path[0], q_start) and np.array_equal(path[-1], q_goal)
    _, m = oracle.classify_edges(sc, path[:-1], path[1:], params["resolution"] if "resolution" in params else 0.05)
    cls = oracle.classify(m)
    assert np.all(cls >= 0), f"path edge certainly colliding, margins {m}"
    cost = float(np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1).sum())
    assert abs(cost - res.cost) <= 1e-5 * cost
    assert cost >= float(np.linalg.norm(q_goal.astype(np.float64) - q_start)) * (1 - 1e-6)
    costs = res.stats["costs"]
    assert all(b < a for a, b in zip(costs, costs[1:])), costs
    assert abs(costs[-1] - res.cost) <= 1e-6 * res.cost
    return m


def _check_roadmap_moves(sc, hist, roadmaps, delta, res, sample=200):
    """Every incumbent path lies on the roadmaps' tensor product (Sec.
    "Problem Setup"): each waypoint is the composite of its arms' roadmap
    vertices, and each step moves every arm along one of its roadmap edges
    or keeps it in place, except at most one step (the straight connection
    of the two trees).  The exported roadmaps themselves: vertices free of
    the environment, edges no longer than delta and free for their arm."""
    from oracle.planner import _arm_scene
    R = sc.n_robots
    q_off = np.concatenate([[0], np.cumsum([m.n_joints for m in sc.models])])
    edges = [set(map(tuple, np.sort(E, axis=1).tolist())) for _, E in roadmaps]
    for h in hist:
        vid = h.vertex_ids
        assert vid.shape == (len(h.path), R)
        for k in range(len(h.path)):
            want = np.concatenate([roadmaps[r][0][vid[k, r], :sc.models[r].n_joints] for r in range(R)])
            np.testing.assert_array_equal(h.path[k], want)
        jumps = 0
        for k in range(len(h.path) - 1):
            ok = all(vid[k, r] == vid[k + 1, r] or tuple(sorted((vid[k, r], vid[k + 1, r]))) in edges[r]
                     for r in range(R))
            jumps += 0 if ok else 1
        assert jumps <= 1, f"{jumps} path steps are not roadmap moves"
    rng = np.random.default_rng(0)
    for r, (V, E) in enumerate(roadmaps):
        arm = _arm_scene(sc, r)
        assert np.all(oracle.classify(oracle.state_margins(arm, V)) >= 0)
        if len(E):
            pick = E[rng.choice(len(E), min(sample, len(E)), replace=False)]
            qa, qb = V[pick[:, 0]], V[pick[:, 1]]
            assert np.all(np.linalg.norm(qa.astype(np.float64) - qb, axis=1) <= delta * (1 + 1e-6))
            _, m = oracle.classify_edges(arm, qa, qb, res)
            assert np.all(oracle.classify(m) >= 0)


@pytest.mark.parametrize("kind", ["c1", "c2"])
def test_plan_returns_valid_improving_path(ctx, kind):
    print(f"[plan] {kind}", flush=True)
    p = problem(kind)
    s = _scene(ctx, p.scene)
    res, hist, n = s.plan_with_history(p.q_start, p.q_goal, roadmaps=True, **PARAMS)
    print(f"  cost {res.cost:.4f} stats { {k: v for k, v in res.stats.items() if k != 'roadmaps'} }", flush=True)
    assert res.status == "OK" and n == len(hist) >= 1
    _check_path(p.scene, res, p.q_start, p.q_goal, PARAMS)
    assert res.stats["first_round"] >= 0 and res.stats["edge_states"] > 0
    _check_roadmap_moves(p.scene, hist, res.stats["roadmaps"], PARAMS["delta"], 0.05)
    assert [len(V) for V, _ in res.stats["roadmaps"]] and \
        sum(len(V) for V, _ in res.stats["roadmaps"]) == res.stats["roadmap_vertices"]
    # finer re-validation (the method checks discrete states only): reported
    _, m4 = oracle.classify_edges(p.scene, res.path[:-1], res.path[1:], 0.05 / 4)
    print(f"  min margin at res/4: {m4.min():.3e}", flush=True)


def _tiny_scene():
    """Two 20-sphere arms 1 m apart facing each other, four obstacle spheres."""
    sph = np.array([[0.0, 0.45, 0.55, 0.12], [0.0, -0.45, 0.6, 0.1], [0.15, 0.0, 1.25, 0.1],
                    [-0.2, 0.3, 0.2, 0.08]], np.float32)
    m = W.panda_like(20)
    sc = W.Scene([m, m], np.stack([W.base_transform(-0.5, 0, 0), W.base_transform(0.5, 0, np.pi)]), sph,
                 np.zeros((0, 6), np.float32), name="tiny two-arm scene")
    return W.make_problem(sc, 5, oracle.states_free)


def test_plan_tiny_scene_passes_quarter_resolution(ctx):
    """On a pinned tiny scene every incumbent, checked at a quarter of the
    planning resolution by the oracle, has no certainly colliding edge."""
    p = _tiny_scene()
    s = _scene(ctx, p.scene)
    res, hist, n = s.plan_with_history(p.q_start, p.q_goal, roadmaps=True, **PARAMS)
    assert res.status == "OK" and n >= 1
    _check_path(p.scene, res, p.q_start, p.q_goal, PARAMS)
    _check_roadmap_moves(p.scene, hist, res.stats["roadmaps"], PARAMS["delta"], 0.05)
    for h in hist:
        _, m4 = oracle.classify_edges(p.scene, h.path[:-1], h.path[1:], 0.05 / 4)
        assert np.all(oracle.classify(m4) >= 0), f"res/4 margins {m4.min():.3e}"
        print(f"  cost {h.cost:.4f}: min margin at res/4 {m4.min():.3e}", flush=True)


C3_PARAMS = dict(seed=0, candidates=256, max_rounds=200, max_iterations=2, n_roadmap=32, delta=3.0,
                 resolution=0.02, max_growth_rounds=24, time_budget_s=60.0)


def _c3_problem():
    """The 8-arm shelf problem of the benchmark fixture: start and goal drawn
    with 2 cm clearance and kept when the oracle's roadmap growth (seed 0)
    joins each arm's pair."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_bench.json")))
    sc = W.scene_c3(d["scene_seed"]).with_env(np.array(d["env_spheres"], np.float32).reshape(-1, 4),
                                              np.array(d["env_boxes"], np.float32).reshape(-1, 6))
    return sc, np.array(d["q_start"], np.float32), np.array(d["q_goal"], np.float32)


def test_plan_c3_eight_arms(ctx):
    """The 56-DoF shelf workload (8 arms x 59 spheres, 256 boxes, 0.02 rad):
    the path passes the oracle's re-validation with its FP64 cost and lies on
    the roadmaps' tensor product."""
    print("[plan] c3", flush=True)
    sc, qs, qg = _c3_problem()
    s = _scene(ctx, sc)
    res, hist, n = s.plan_with_history(qs, qg, roadmaps=True, **C3_PARAMS)
    print(f"  status {res.status} cost {res.cost:.4f} rounds {res.stats['rounds']} "
          f"first round {res.stats['first_round']} tts {res.stats['time_to_first_s']:.3f}s "
          f"edge states {res.stats['edge_states']} roadmap connected {res.stats['roadmap_connected']}", flush=True)
    assert res.status == "OK" and n >= 1
    _check_path(sc, res, qs, qg, C3_PARAMS)
    _check_roadmap_moves(sc, hist, res.stats["roadmaps"], C3_PARAMS["delta"], 0.02, sample=60)


def test_plan_ten_arms_grouped_launches(ctx):
    """Ten planar arms: each roadmap step's per-arm commands exceed one
    launch group (eight records) and the arms' validations exceed the
    one-workgroup segment table, so the chunked and the general paths run.
    The plan must be valid, repeatable and equal to its batched run."""
    rng = np.random.default_rng(31)
    sph = np.concatenate([rng.uniform([-0.5, -0.5, -0.05], [0.5, 0.5, 0.05], (6, 3)),
                          rng.uniform(0.05, 0.1, (6, 1))], axis=1).astype(np.float32)
    sc = W.Scene([W.planar_two_link()] * 10, W.ring_bases(10, 1.3), sph, np.zeros((0, 6), np.float32),
                 name="ten planar arms")
    p = W.make_problem(sc, 3, oracle.states_free)
    s = _scene(ctx, p.scene)
    params = dict(PARAMS, max_iterations=2)
    a = s.plan(p.q_start, p.q_goal, **params)
    print(f"  cost {a.cost:.4f} stats {a.stats}", flush=True)
    assert a.status == "OK"
    _check_path(p.scene, a, p.q_start, p.q_goal, params)
    b = s.plan(p.q_start, p.q_goal, **params)
    assert np.array_equal(a.path, b.path) and a.cost == b.cost
    got, _ = ctx.plan_batch([(s, p.q_start, p.q_goal, dict(params, seed=k)) for k in (1, 2)])
    for k, g in zip((1, 2), got):
        ref = s.plan(p.q_start, p.q_goal, raise_on_error=False, **dict(params, seed=k))
        assert g.status == ref.status
        if ref.status == "OK":
            assert np.array_equal(g.path, ref.path) and g.cost == ref.cost


def test_plan_deterministic(ctx):
    p = problem("c1")
    s = _scene(ctx, p.scene)
    a = s.plan(p.q_start, p.q_goal, **PARAMS)
    b = s.plan(p.q_start, p.q_goal, **PARAMS)
    assert np.array_equal(a.path, b.path) and a.cost == b.cost and a.stats["costs"] == b.stats["costs"]


def test_plan_empty_scene_single_arm_reaches_roadmap_optimum(ctx):
    """One arm, no obstacles: every edge is free and the roadmap samples come
    from the same streams on both sides, so both planners end at the
    cheapest path available over the roadmap, start -> v -> goal through a
    roadmap neighbour v of the start or the goal (closed form below)."""
    from oracle.planner import plan as oplan, PlanParams
    m = W.panda_like(20)
    sc = W.Scene([m], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    rng = np.random.default_rng(3)
    qs = W.random_configs(sc, 1, rng)[0]
    step = rng.uniform(-1, 1, sc.dof).astype(np.float32)
    step *= 1.0 / np.abs(step).max()
    qg = np.clip(qs + step, sc.q_lo, sc.q_hi).astype(np.float32)
    kw = dict(seed=2, candidates=64, max_rounds=300, max_iterations=3, n_roadmap=16, delta=3.0)
    o = oplan(sc, qs, qg, PlanParams(**kw))
    assert o.status == "OK" and not o.last_search_solved
    rm = o.roadmaps[0]
    s64, g64 = qs.astype(np.float64), qg.astype(np.float64)
    best = min(np.linalg.norm(rm.V[v].astype(np.float64) - s64) + np.linalg.norm(rm.V[v].astype(np.float64) - g64)
               for v in set(rm.adj[0]) | set(rm.adj[1]))
    res = _scene(ctx, sc).plan(qs, qg, **kw)
    assert res.status == "OK"
    assert res.stats["roadmap_vertices"] == len(rm.V)
    assert abs(res.cost - best) <= 1e-5 * best, (res.cost, best, res.stats)


@pytest.mark.parametrize("case", ["roadmaps_unconnected", "tree_full"])
def test_plan_outer_loop_matches_oracle(ctx, case):
    """Alg. 1's outer loop: an iteration that leaves an arm's start and goal
    unconnected runs no search (the next one grows on), and a search whose
    tree fills up ends and the next iteration starts afresh.  Both planners
    draw the same streams, so they agree on the outcome, the rounds, the
    iterations and the roadmap sizes."""
    from oracle.planner import plan as oplan, PlanParams
    kw = {"roadmaps_unconnected": dict(seed=1, candidates=64, max_rounds=40, max_iterations=4, n_roadmap=2,
                                       delta=3.0, max_growth_rounds=1),
          "tree_full": dict(seed=1, candidates=64, max_rounds=12, max_iterations=6, n_roadmap=32, delta=3.0,
                            max_tree_nodes=3)}[case]
    p = problem("c1")
    o = oplan(p.scene, p.q_start, p.q_goal, PlanParams(**kw))
    g, _, _ = _scene(ctx, p.scene).plan_with_history(p.q_start, p.q_goal, raise_on_error=False, roadmaps=True, **kw)
    print(f"  {case}: oracle {o.status} rounds {o.rounds} iterations {o.iterations}; "
          f"gpu {g.status} rounds {g.stats['rounds']} iterations {g.stats['iterations']}", flush=True)
    assert o.status == {"roadmaps_unconnected": "E_NO_SOLUTION", "tree_full": "E_CAPACITY"}[case]
    assert (g.status, g.stats["rounds"], g.stats["iterations"]) == (o.status, o.rounds, o.iterations)
    assert g.stats["roadmap_vertices"] == sum(len(m.V) for m in o.roadmaps)
    for (V, _), m in zip(g.stats["roadmaps"], o.roadmaps):
        mv = np.asarray(m.V, np.float32)  # the samples' affine map rounds once on each side
        assert V.shape[0] == mv.shape[0] and np.abs(V[:, :mv.shape[1]] - mv).max() <= 4e-6


def test_plan_error_paths(ctx):
    import paper_2609_30644_amd as M
    p = problem("c1")
    s = _scene(ctx, p.scene)
    bad = p.q_start.copy()
    bad[0] = np.nan
    with pytest.raises(M.MrpopError) as e:
        s.plan(bad, p.q_goal, **PARAMS)
    assert e.value.name == "E_NONFINITE"
    # a start inside an obstacle
    sph = np.concatenate([p.scene.env_spheres, [[-0.5, 0.0, 0.2, 0.2]]]).astype(np.float32)
    blocked = p.scene.with_env(sph, p.scene.env_boxes)
    with pytest.raises(M.MrpopError) as e:
        _scene(ctx, blocked).plan(p.q_start, p.q_goal, **PARAMS)
    assert e.value.name == "E_START_INVALID"
    # path buffer too small: status and the required length
    r = s.plan(p.q_start, p.q_goal, path_cap=1, raise_on_error=False, **PARAMS)
    assert r.status == "E_BUFFER" and r.stats["path_len"] >= 2
    with pytest.raises(M.MrpopError) as e:
        s.plan(p.q_start, p.q_goal, candidates=0)
    assert e.value.name == "E_INVALID_ARG"


def test_plan_trajectory_matches_oracle_c1(ctx):
    """The oracle planner follows the same rounds and random streams, so on
    a problem without near-ties (the C1 problem of seed 0: checked once, the
    trajectories then agreed to the last incumbent) the two planners find
    the same incumbents in the same rounds and end on the same path; a
    near-tie elsewhere could make them part (FP32 against FP64)."""
    from oracle.planner import plan as oplan, PlanParams
    p = problem("c1")
    s = _scene(ctx, p.scene)
    g = s.plan(p.q_start, p.q_goal, **PARAMS)
    o = oplan(p.scene, p.q_start, p.q_goal, PlanParams(**PARAMS))
    print(f"  gpu costs {[round(c, 4) for c in g.stats['costs']]} first round {g.stats['first_round']}")
    print(f"  cpu costs {[round(c, 4) for c in o.costs]} first round {o.first_round}", flush=True)
    assert g.status == o.status == "OK" and g.stats["first_round"] == o.first_round
    assert len(g.stats["costs"]) == len(o.costs)
    for a, b in zip(g.stats["costs"], o.costs):
        assert abs(a - b) <= 1e-5 * b, (g.stats["costs"], o.costs)
    assert g.path.shape == o.path.shape and np.abs(g.path - o.path).max() < 1e-4


def test_plan_history_ranked_and_valid(ctx):
    """mrpop_plan_with_history: every incumbent of the call, cheapest first;
    the plan itself is the one mrpop_plan returns; each entry re-validated by
    the oracle with its FP64 cost; smaller buffers keep the cheapest ones."""
    print("[plan history] c2", flush=True)
    p = problem("c2")
    s = _scene(ctx, p.scene)
    ref = s.plan(p.q_start, p.q_goal, **PARAMS)
    res, hist, n = s.plan_with_history(p.q_start, p.q_goal, **PARAMS)
    print(f"  {n} incumbents, costs {[h.cost for h in hist]}", flush=True)
    assert res.status == "OK" and np.array_equal(res.path, ref.path) and res.cost == ref.cost
    assert n == res.stats["solutions"] == len(hist) >= 1
    assert np.array_equal(hist[0].path, res.path) and hist[0].cost == res.cost
    costs = [h.cost for h in hist]
    assert all(a < b for a, b in zip(costs, costs[1:]))
    assert costs == [float(c) for c in reversed(res.stats["costs"][:n])]
    assert all(a.found_round >= b.found_round and a.found_s >= b.found_s for a, b in zip(hist, hist[1:]))
    for h in hist:
        _check_path(p.scene, PlanResultLike(h.path, h.cost, {"costs": [h.cost]}), p.q_start, p.q_goal, PARAMS)
    one = s.plan_with_history(p.q_start, p.q_goal, max_entries=1, **PARAMS)
    assert one[2] == n and len(one[1]) == 1 and np.array_equal(one[1][0].path, hist[0].path)
    if n >= 2:
        rows = len(hist[0].path) + len(hist[1].path) - 1  # room for the cheapest only
        cut = s.plan_with_history(p.q_start, p.q_goal, max_waypoints=rows, **PARAMS)
        assert cut[2] == n and len(cut[1]) == 1 and cut[1][0].cost == hist[0].cost
    none = s.plan_with_history(p.q_start, p.q_goal, max_entries=0, max_waypoints=0, **PARAMS)
    assert none[2] == n and none[1] == [] and np.array_equal(none[0].path, res.path)


DIRECT = dict(seed=3, candidates=64, max_rounds=150, max_iterations=4, n_roadmap=32, delta=3.0, direct=1, step=1.0)


def test_plan_direct_single_arm(ctx):
    """Direct mode through the C ABI: no roadmap; the path passes the oracle's
    re-validation with its FP64 cost; every edge but the connection is a tree
    edge no longer than `step`; deterministic."""
    print("[plan direct] single arm", flush=True)
    p = W.make_problem(W.scene_single(0), 0, oracle.states_free)
    s = _scene(ctx, p.scene)
    res = s.plan(p.q_start, p.q_goal, **DIRECT)
    assert res.status == "OK" and res.stats["roadmap_vertices"] == 0 and res.stats["roadmap_edge_states"] == 0
    _check_path(p.scene, res, p.q_start, p.q_goal, DIRECT)
    steps = np.linalg.norm(np.diff(res.path.astype(np.float64), axis=0), axis=1)
    assert int((steps > DIRECT["step"] * (1 + 1e-5)).sum()) <= 1
    again = s.plan(p.q_start, p.q_goal, **DIRECT)
    assert np.array_equal(again.path, res.path) and again.cost == res.cost


def test_plan_direct_first_solution_matches_oracle(ctx):
    """One arm, no obstacles: the first solution is start -> steer(start,
    q_rand_i) -> goal for the cheapest candidate of round 0 on both sides
    (the same random streams); the GPU's equals the oracle's within FP32
    rounding."""
    from oracle.planner import plan as oplan, PlanParams
    sc = W.Scene([W.panda_like(20)], W.base_transform(0, 0, 0)[None], np.zeros((0, 4), np.float32),
                 np.zeros((0, 6), np.float32))
    qs, qg = W.random_configs(sc, 2, np.random.default_rng(11))
    prm = dict(seed=4, candidates=32, max_rounds=60, max_iterations=3, direct=1, step=0.7)
    o = oplan(sc, qs, qg, PlanParams(**dict(prm, direct=True)))
    s = _scene(ctx, sc)
    res, hist, n = s.plan_with_history(qs, qg, **prm)
    assert res.status == "OK" and res.stats["first_round"] == 0 and n >= 1
    first = hist[-1]  # ranked cheapest first: the first one found is the last
    o_cost, o_path, _ = o.history[0]
    print(f"  gpu first {first.cost:.6f} oracle first {o_cost:.6f}", flush=True)
    assert first.path.shape == o_path.shape == (3, sc.dof)
    assert np.allclose(first.path, o_path, atol=1e-5, rtol=0)
    assert abs(first.cost - o_cost) <= 1e-5 * o_cost


def test_plan_direct_batch_equals_plain(ctx):
    """Direct-mode instances in one mrpop_plan_batch equal their plain runs."""
    p = W.make_problem(W.scene_single(0), 0, oracle.states_free)
    s = _scene(ctx, p.scene)
    jobs = [(s, p.q_start, p.q_goal, dict(DIRECT, seed=k)) for k in range(4)]
    got, _ = ctx.plan_batch(jobs)
    for k, g in enumerate(got):
        ref = s.plan(p.q_start, p.q_goal, raise_on_error=False, **dict(DIRECT, seed=k))
        assert g.status == ref.status
        if ref.status == "OK":
            assert np.array_equal(g.path, ref.path) and g.cost == ref.cost


def test_scene_set_env_parity(ctx):
    """mrpop_scene_set_env: after replacing the obstacles, edge bits match
    the oracle on the new environment (and a fresh scene built from it)."""
    print("[set_env] c1 -> new obstacles", flush=True)
    p = problem("c1")
    s = _scene(ctx, p.scene)
    other = W.scene_c1(5)
    new = p.scene.with_env(other.env_spheres, p.scene.env_boxes)
    s.set_env(new.env_spheres, new.env_boxes)
    qa, qb = W.edge_batch(new, 512, 0.05, seed=3)[:2]
    got = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    _, m = oracle.classify_edges(new, qa, qb, 0.05)
    stats = assert_bits_match(got, m, "set_env")
    fresh = _scene(ctx, new).validate_edges(qa, qb, 0.05).cpu().numpy()
    assert np.array_equal(got, fresh)
    print(f"  {stats}", flush=True)


def test_plans_reuse_buffers_and_sub_scenes(ctx):
    """Plans take their buffers from the context's pool and the roadmaps'
    one-arm sub-scenes from the scene: a plan repeated after plans of other
    sizes (stale pooled contents) is identical, and after set_env a plan on
    the same scene equals one on a fresh scene of the new environment (the
    sub-scenes are rebuilt)."""
    p1, p2 = problem("c1"), problem("c2")
    s1, s2 = _scene(ctx, p1.scene), _scene(ctx, p2.scene)
    a = s1.plan(p1.q_start, p1.q_goal, **PARAMS)
    s2.plan(p2.q_start, p2.q_goal, raise_on_error=False, **PARAMS)
    b = s1.plan(p1.q_start, p1.q_goal, **PARAMS)
    assert a.status == b.status == "OK"
    assert np.array_equal(a.path, b.path) and a.cost == b.cost and a.stats["costs"] == b.stats["costs"]
    for key in ("rounds", "edge_states", "roadmap_edge_states", "roadmap_vertices"):
        assert a.stats[key] == b.stats[key], key
    other = W.scene_c1(5)
    new = p1.scene.with_env(other.env_spheres, p1.scene.env_boxes)
    ok = oracle.states_free(new, np.stack([p1.q_start, p1.q_goal]))
    if not ok.all():
        pytest.skip("the new obstacles cover an endpoint")
    s1.set_env(new.env_spheres, new.env_boxes)
    c = s1.plan(p1.q_start, p1.q_goal, raise_on_error=False, **PARAMS)
    d = _scene(ctx, new).plan(p1.q_start, p1.q_goal, raise_on_error=False, **PARAMS)
    assert c.status == d.status
    if c.status == "OK":
        assert np.array_equal(c.path, d.path) and c.cost == d.cost
        _check_path(new, c, p1.q_start, p1.q_goal, PARAMS)


def test_replan_tick(ctx):
    """mrpop_replan through the C ABI: an unchanged environment keeps the
    previous path (never worse); an obstacle placed on it (set_env) discards
    it -- the same decision as the oracle's -- and the new path is free in
    the new environment."""
    print("[replan] c1", flush=True)
    p = problem("c1")
    s = _scene(ctx, p.scene)
    r0 = s.plan(p.q_start, p.q_goal, **PARAMS)
    r1, kept = s.replan(p.q_start, p.q_goal, r0.path, **dict(PARAMS, seed=7))
    assert kept and r1.status == "OK" and r1.cost <= r0.cost
    _check_path(p.scene, r1, p.q_start, p.q_goal, {})
    if r1.stats["solutions"] == 0:
        assert np.array_equal(r1.path, r0.path)
    blocked = blocking_obstacle(p, r0.path)
    s.set_env(blocked.env_spheres, blocked.env_boxes)
    r2, kept2 = s.replan(p.q_start, p.q_goal, r0.path, raise_on_error=False, **PARAMS)
    valid, _, _ = oracle.validate_fast(blocked, r0.path[:-1], r0.path[1:], 0.05)
    assert kept2 == bool(np.all(valid)) and not kept2
    if r2.status == "OK":
        _, m2 = oracle.classify_edges(blocked, r2.path[:-1], r2.path[1:], 0.05)
        assert np.all(oracle.classify(m2) >= 0)
    s.set_env(p.scene.env_spheres, p.scene.env_boxes)
