"""Plain CPU planner: MR. POP as bulk-synchronous rounds (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Follows Alg. 1 (the
outer anytime loop) and Alg. 2 (ROADMAP, AO-X with the dRRT oracle, NEAREST)
step by step, in double precision, with Python loops over candidates.  It
uses the oracle's C primitives for the collision check, NEAREST, the random
stream and the informed sample.

Readings where the paper is silent (each is also a GPU-side rule):
  * Rounds: every round draws P candidates against the round-start trees;
    the valid ones are inserted in candidate order; a round that connects
    keeps the cheapest connection (ties: lowest candidate index).
  * Random numbers: counter-based SplitMix64 streams keyed by
    (seed, purpose, round, candidate) -- purpose 1: configuration sample,
    2: unit-ball sample, 3: cost sample, 4: roadmap samples.
  * ROADMAP adds the start and goal as vertices 0 and 1 and connects only new
    samples to their neighbours (as Alg. 2 reads), so start and goal are
    never adjacent to each other.
  * ROADMAP: each call resets the connected flags; every unconnected arm gets
    n samples (uniform in its limits, kept when free of the environment,
    first n free in draw order), then every pair (new vertex i, any vertex
    j < i) closer than delta becomes an edge when its single-arm motion is
    free; BFS from the start vertex (0) to the goal vertex (1).  Roadmaps
    persist across calls.  A call grows for at most max_growth_rounds
    rounds; if an arm is still unconnected then, the iteration runs no
    search (the tensor product has no start-goal path) and the next
    iteration's call grows on, so that over the iterations ROADMAP loops
    until every arm is connected, as Alg. 2 has it.
  * ORACLE_AOX (the dRRT oracle with AO-X's admissibility; Sec. "Converge to
    Global Optimality"): per arm, a roadmap neighbour u of the arm's vertex
    in z_near is admissible when the composite neighbour that moves this arm
    alone to u stays within the budget, g_near + |u - q_near^i| < c_rand; among
    the admissible ones the arm takes the one best aligned with the sample
    direction (largest cosine, ties to the lowest neighbour id), and stays if
    no admissible neighbour has a positive cosine.  When the composite of
    these per-arm moves exceeds the budget, arms go back to staying, least
    aligned first (ties: the higher arm index first), until it fits; the last
    moving arm always fits on its own.  A candidate where every arm stays is
    dropped.  With c_rand = +inf (the initial solve) this is the plain dRRT
    oracle.
  * Informed samples outside the joint limits are clamped onto them (the
    Euclidean projection onto the box).  The projection cannot move a point
    farther from either focus (it is non-expansive and both foci are inside
    the box), so the clamped point is still inside the prolate hyperspheroid;
    points already inside the box are unchanged, so the draw has a positive
    density on the whole informed set within the limits.
  * The cost lower bound g(q) of a sample is its distance to the root of the
    tree being extended (the start, or the goal after a swap).
  * Connection: NEAREST in the other tree with budget c_best - g_new (the
    initial solve uses an infinite budget); accepted only if the new path is
    strictly cheaper than the incumbent.
  * Tree capacity: a search whose round finds T_a full (a free extension
    that max_tree_nodes leaves out) ends after that round, and the next outer
    iteration starts afresh (roadmaps grow, new trees): Alg. 1 loops until
    the time budget, so the memory bound restarts a search rather than
    ending the plan.  ao-dRRT, whose trees persist, ends there.
  * Direct mode (single-robot planning without the roadmap layer): no
    ROADMAP; an extension steers from q_near toward q_rand, all the way when
    q_rand is within `step` (Euclidean), else by exactly `step` along the
    segment (RRT-Connect's extend, the connection being its greedy connect);
    a sample equal to q_near is dropped; the AO-X admissibility rule is
    unchanged.  Every outer iteration is one search with fresh trees.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import (OracleScene, classify_edges, edge_nstates, ellipsoid_map, key, nearest, u01, unit_ball,
               validate_fast)

PURPOSE_Q, PURPOSE_BALL, PURPOSE_C, PURPOSE_ROADMAP = 1, 2, 3, 4
ROADMAP_BATCH = 4  # candidates drawn per needed sample in one roadmap draw


@dataclass
class PlanParams:
    seed: int = 0
    delta: float = 1.0
    n_roadmap: int = 32
    candidates: int = 64
    resolution: float = 0.05
    max_rounds: int = 200
    max_iterations: int = 4
    max_growth_rounds: int = 16
    max_tree_nodes: int = 100000
    stop_at_first: bool = False
    # direct mode: no roadmaps; extensions steer toward the sample by at most
    # `step` (Sec. "Single-Robot Simulation Benchmarks & Ablations")
    direct: bool = False
    step: float = 1.0
    # ao-dRRT: persistent trees improved by rewiring instead of AO-X's
    # cost-bounded searches on fresh trees (Sec. "Methodology": the paper's
    # asymptotically optimal multi-robot baseline)
    rewire: bool = False
    # wall-clock bound on plan() (0: none), checked between rounds; it stops
    # the run, it changes no result of a round
    time_budget_s: float = 0.0


@dataclass
class PlanResult:
    status: str
    path: Optional[np.ndarray]
    cost: float
    rounds: int
    iterations: int
    first_round: int = -1
    costs: List[float] = field(default_factory=list)
    edge_states: int = 0
    roadmaps: list = field(default_factory=list)
    last_search_solved: bool = False
    # every incumbent in discovery order: (cost, path start to goal, round)
    history: list = field(default_factory=list)
    # per search round: (round, extended tree is the start tree, |T_a|, |T_b|)
    trace: list = field(default_factory=list)
    # the last search's trees (start tree, goal tree)
    trees: tuple = ()


class _Roadmap:
    def __init__(self, q_start: np.ndarray, q_goal: np.ndarray):
        self.V: List[np.ndarray] = [q_start.astype(np.float32), q_goal.astype(np.float32)]
        self.adj: List[set] = [set(), set()]

    def add_vertex(self, q):
        self.V.append(np.asarray(q, np.float32))
        self.adj.append(set())
        return len(self.V) - 1

    def add_edge(self, i, j):
        self.adj[i].add(j)
        self.adj[j].add(i)

    def connected(self) -> bool:
        seen, frontier = {0}, [0]
        while frontier:
            nxt = []
            for v in frontier:
                for u in self.adj[v]:
                    if u not in seen:
                        seen.add(u)
                        nxt.append(u)
            frontier = nxt
        return 1 in seen


def _arm_scene(scene, r):
    from workloads import Scene
    return Scene([scene.models[r]], scene.base_tf[r:r + 1], scene.env_spheres, scene.env_boxes)


def roadmap_step(scene, roadmaps, arm_scenes, params: PlanParams, iteration: int, q_off):
    """ROADMAP (Alg. 2): grow every arm's roadmap until start and goal are
    connected (at most max_growth_rounds rounds).  Returns True if all are
    connected."""
    connected = [False] * scene.n_robots
    for g in range(params.max_growth_rounds):
        for r, rm in enumerate(roadmaps):
            if connected[r]:
                continue
            m = scene.models[r]
            lo, hi = m.q_lo.astype(np.float64), m.q_hi.astype(np.float64)
            k = key(params.seed, PURPOSE_ROADMAP, iteration * 1024 + g, r)
            accepted, j = [], 0
            while len(accepted) < params.n_roadmap:
                batch = ROADMAP_BATCH * params.n_roadmap
                u = u01(k, (j + batch) * 8)
                cand = np.array([lo + u[(j + b) * 8:(j + b) * 8 + m.n_joints] * (hi - lo) for b in range(batch)],
                                np.float32)
                _, mm = classify_edges(arm_scenes[r], cand, cand, 1.0)
                for b in range(batch):
                    if mm[b] >= 0 and len(accepted) < params.n_roadmap:
                        accepted.append(cand[b])
                j += batch
            n0 = len(rm.V)
            for q in accepted:
                rm.add_vertex(q)
            pairs = []
            for i in range(n0, len(rm.V)):
                for jj in range(i):
                    if np.linalg.norm(rm.V[i].astype(np.float64) - rm.V[jj].astype(np.float64)) <= params.delta:
                        pairs.append((jj, i))
            if pairs:
                qa = np.array([rm.V[a] for a, _ in pairs], np.float32)
                qb = np.array([rm.V[b] for _, b in pairs], np.float32)
                valid, _, _ = validate_fast(arm_scenes[r], qa, qb, params.resolution)
                for (a, b), v in zip(pairs, valid):
                    if v:
                        rm.add_edge(a, b)
            connected[r] = rm.connected()
        if all(connected):
            return True
    return all(connected)


@dataclass
class _Tree:
    q: List[np.ndarray]
    g: List[float]
    parent: List[int]
    vid: List[tuple]

    def __len__(self):
        return len(self.q)


def _new_tree(q, vid):
    return _Tree([np.asarray(q, np.float32)], [0.0], [-1], [vid])


def _path_to_root(t: _Tree, i: int):
    out = []
    while i >= 0:
        out.append(t.q[i])
        i = t.parent[i]
    return out[::-1]


def _cost(path) -> float:
    p = np.asarray(path, np.float64)
    return float(np.linalg.norm(np.diff(p, axis=0), axis=1).sum()) if len(p) > 1 else 0.0


def aox_oracle(roadmaps, vid_near, q_rand_arms, g_near: float = 0.0, c_rand: float = math.inf):
    """ORACLE_AOX (Alg. 2; Sec. "Converge to Global Optimality"): the vertex
    ids of q_new, one per arm (equal to vid_near when no arm moves).

    Per arm i, with v = vid_near[i] and the sample direction d = q_rand^i - V_v:
    a neighbour u of v in the arm's roadmap is admissible when moving arm i
    alone to it stays within the budget, g_near + |V_u - V_v| < c_rand, and
    the arm takes the admissible neighbour of largest cosine with d (ties:
    lowest id), or stays when none has a positive cosine (or d = 0).  If the
    composite move then costs g_near + |q_new - q_near| >= c_rand, moving arms
    go back to staying, least aligned first (ties: higher arm index first),
    until it fits.  With c_rand = +inf this is dRRT's oracle."""
    best, cosv, d2 = [], [], []
    for r, rm in enumerate(roadmaps):
        v = vid_near[r]
        base = rm.V[v].astype(np.float64)
        d = np.asarray(q_rand_arms[r], np.float64) - base
        nd = float(np.linalg.norm(d))
        b, b_cos, b_d2 = v, 0.0, 0.0
        if nd > 0:
            for u in sorted(rm.adj[v]):
                e = rm.V[u].astype(np.float64) - base
                ne = float(np.linalg.norm(e))
                if ne == 0 or not (g_near + ne < c_rand):
                    continue
                cos = float(np.dot(e, d) / (ne * nd))
                if cos > b_cos:
                    b, b_cos, b_d2 = u, cos, ne * ne
        best.append(b)
        cosv.append(b_cos)
        d2.append(b_d2)
    moving = [r for r in range(len(roadmaps)) if best[r] != vid_near[r]]
    while moving and not (g_near + math.sqrt(sum(d2[r] for r in moving)) < c_rand):
        moving.remove(min(moving, key=lambda r: (cosv[r], -r)))
    return [best[r] if r in moving else vid_near[r] for r in range(len(roadmaps))]


def drrt_oracle(roadmaps, vid_near, q_near_arms, q_rand_arms):
    """dRRT's oracle (no cost budget): ORACLE_AOX with c_rand = +inf."""
    return aox_oracle(roadmaps, vid_near, q_rand_arms)


def cost_coordinate(lb: float, c_best: float, u: float) -> float:
    """The cost coordinate c_rand ~ U[lb, c_best] of an AO-X sample (Alg. 2:
    the budgets under which q_rand is reachable, lb = g(q_rand)) from a
    uniform u in [0, 1); c_best itself when lb >= c_best."""
    return lb + u * (c_best - lb) if lb < c_best else c_best


def draw_candidate(seed: int, rnd: int, i: int, c_best: float, lo, hi, q_start, q_goal, root):
    """Candidate i of round rnd: (q_rand, c_rand), FP64 (Alg. 2).

    c_best = +inf: q_rand uniform in the joint box, c_rand = +inf.  Otherwise
    INFORMED_SAMPLE: a uniform point of the unit D-ball mapped into the
    prolate hyperspheroid with foci q_start, q_goal and transverse diameter
    c_best, clamped onto the joint box; c_rand from cost_coordinate with
    lb = |q_rand - root|, root being the root of the tree this candidate
    extends."""
    D = lo.shape[0]
    if math.isinf(c_best):
        u = u01(key(seed, PURPOSE_Q, rnd, i), D)
        return lo + u * (hi - lo), math.inf
    x = unit_ball(key(seed, PURPOSE_BALL, rnd, i), D)
    q_rand = np.clip(ellipsoid_map(q_start, q_goal, c_best, x), lo, hi)
    lb = float(np.linalg.norm(q_rand - np.asarray(root, np.float64)))
    return q_rand, cost_coordinate(lb, c_best, u01(key(seed, PURPOSE_C, rnd, i), 1)[0])


def needs_swap(ta, tb) -> bool:
    """Alg. 2 extends the smaller tree: swap when |V_a| > |V_b| (equal sizes
    keep the current order)."""
    return len(ta) > len(tb)


def connect_budget(c_best: float, g_new: float) -> float:
    """Budget of the connection search from a new vertex (Alg. 2, AO-X): only
    vertices z of the other tree with g_z + |q_new - q_z| < c_best - g_new,
    so that any connection makes a path cheaper than c_best; +inf in the
    initial solve."""
    return c_best - g_new if not math.isinf(c_best) else math.inf


@dataclass
class RoundOutcome:
    """What one search round did, in candidate order."""
    cands: list = field(default_factory=list)     # (i, k_near, vid_new, q_new, g_new): extensions to validate
    valid: list = field(default_factory=list)     # their edge bits
    inserted: list = field(default_factory=list)  # (i, index in T_a)
    conns: list = field(default_factory=list)     # (i, index in T_a, index in T_b): connection edges tried
    cvalid: list = field(default_factory=list)    # their edge bits
    best: Optional[tuple] = None                  # (total cost, i, index in T_a, index in T_b)
    edge_states: int = 0
    overflow: bool = False                        # a free extension found T_a full


def search_round(osc, roadmaps, ta, tb, draws, c_best: float, params: PlanParams, composite) -> RoundOutcome:
    """One round of P candidate iterations against the round-start trees
    (Alg. 2, AO-X; dRRT_SEARCH when c_best = +inf): for each draw (q_rand,
    c_rand): NEAREST in T_a under c_rand, the extension (ORACLE_AOX, or a
    steer in direct mode), then the edge checks; survivors enter T_a in
    candidate order, each searches T_b under connect_budget, and the free
    connection of least total cost (ties: lowest candidate) is the round's
    result.  T_a grows in place."""
    out = RoundOutcome()
    R = len(roadmaps)
    na, nb = len(ta), len(tb)
    Va, ga = np.array(ta.q[:na], np.float32), np.array(ta.g[:na], np.float32)
    Vb, gb = np.array(tb.q[:nb], np.float32), np.array(tb.g[:nb], np.float32)
    q_off = np.concatenate([[0], np.cumsum([len(rm.V[0]) for rm in roadmaps])]).astype(int)
    for i, (q_rand, c_rand) in enumerate(draws):
        k_near = nearest(Va, ga, np.asarray(q_rand, np.float32), c_rand)
        if k_near < 0:
            continue
        q_near = ta.q[k_near].astype(np.float64)
        g_near = float(ta.g[k_near])
        if params.direct:
            if not np.any(np.asarray(q_rand, np.float64) != q_near):  # nothing to extend toward
                continue
            q_new = steer(q_near, q_rand, params.step).astype(np.float32)
            vid_new = ta.vid[k_near]
            g_new = g_near + float(np.linalg.norm(q_new.astype(np.float64) - q_near))
            if not math.isinf(c_best) and not (g_new < c_rand):
                continue
        else:
            arms = [np.asarray(q_rand, np.float64)[q_off[r]:q_off[r + 1]] for r in range(R)]
            vid_new = tuple(aox_oracle(roadmaps, ta.vid[k_near], arms, g_near, c_rand))
            if vid_new == ta.vid[k_near]:
                continue
            q_new = composite(vid_new)
            g_new = g_near + float(np.linalg.norm(q_new.astype(np.float64) - q_near))
        out.cands.append((i, k_near, vid_new, q_new, g_new))
    if out.cands:
        qa = np.array([ta.q[c[1]] for c in out.cands], np.float32)
        qb = np.array([c[3] for c in out.cands], np.float32)
        valid, n, _ = validate_fast(osc, qa, qb, params.resolution)
        out.valid = [bool(v) for v in valid]
        out.edge_states += int(n.sum())
    for c, v in zip(out.cands, out.valid):
        out.overflow |= v and len(ta) >= params.max_tree_nodes
        if v and len(ta) < params.max_tree_nodes:
            ta.q.append(c[3])
            ta.g.append(np.float32(c[4]))
            ta.parent.append(c[1])
            ta.vid.append(c[2])
            out.inserted.append((c[0], len(ta) - 1))
    for ci, idx in out.inserted:
        kc = nearest(Vb, gb, ta.q[idx], connect_budget(c_best, float(ta.g[idx])))
        if kc >= 0:
            out.conns.append((ci, idx, kc))
    if out.conns:
        qa = np.array([ta.q[c[1]] for c in out.conns], np.float32)
        qb = np.array([tb.q[c[2]] for c in out.conns], np.float32)
        valid, n, _ = validate_fast(osc, qa, qb, params.resolution)
        out.cvalid = [bool(v) for v in valid]
        out.edge_states += int(n.sum())
        for (ci, idx, kc), v in zip(out.conns, out.cvalid):
            if not v:
                continue
            tot = float(ta.g[idx]) + float(np.linalg.norm(ta.q[idx].astype(np.float64) -
                                                          tb.q[kc].astype(np.float64))) + float(tb.g[kc])
            if out.best is None or tot < out.best[0]:
                out.best = (tot, ci, idx, kc)
    return out


# ---------------------------------------------------------------------------
# ao-dRRT: the rewiring baseline
# ---------------------------------------------------------------------------

RW_SLOTS = 4  # rewiring proposals kept per candidate


def tp_adjacent(roadmaps, u, v) -> bool:
    """Composite vertices u and v (tuples of roadmap vertex ids) are adjacent
    in the tensor product of the roadmaps (Sec. "Problem Setup"): they differ,
    and every arm either stays or moves along one of its roadmap edges."""
    return tuple(u) != tuple(v) and all(a == b or b in rm.adj[a] for rm, a, b in zip(roadmaps, u, v))


def _adjacent_mask(tree, n: int, roadmaps, vid_new) -> np.ndarray:
    """tp_adjacent(tree.vid[k], vid_new) for k < n, as a boolean array: per
    arm, the vertex is vid_new's or one of its roadmap neighbours."""
    if n == 0:
        return np.zeros(0, bool)
    V = np.array(tree.vid[:n], np.int64).reshape(n, -1)
    ok = np.ones(n, bool)
    same = np.ones(n, bool)
    for r, rm in enumerate(roadmaps):
        v = vid_new[r]
        ok &= np.isin(V[:, r], list(rm.adj[v]) + [v])
        same &= V[:, r] == v
    return ok & ~same


def best_parent(tree, n: int, roadmaps, vid_new, q_new):
    """The parent of a new vertex: among the first n tree vertices adjacent to
    it in the tensor product, the one of least g_z + |q_new - q_z| (ties: the
    lowest index).  Returns (g_new, index), or None when there is none."""
    ks = np.nonzero(_adjacent_mask(tree, n, roadmaps, vid_new))[0]
    if ks.size == 0:
        return None
    Q = np.array([tree.q[k] for k in ks], np.float64)
    c = np.array([float(tree.g[k]) for k in ks]) + np.linalg.norm(Q - np.asarray(q_new, np.float64), axis=1)
    j = int(np.argmin(c))  # the first of equal minima: the lowest index
    return float(c[j]), int(ks[j])


def rewire_proposals(tree, n: int, roadmaps, vid_new, q_new, g_new: float, parent: int, slots: int = RW_SLOTS):
    """Tree vertices z (among the first n, adjacent to the new vertex, not its
    parent) whose cost would drop through it, g_new + |q_z - q_new| < g_z:
    the `slots` of largest drop (ties: lowest index), as (z, new cost)."""
    mask = _adjacent_mask(tree, n, roadmaps, vid_new)
    if 0 <= parent < n:
        mask[parent] = False
    ks = np.nonzero(mask)[0]
    if ks.size == 0:
        return []
    Q = np.array([tree.q[k] for k in ks], np.float64)
    c = g_new + np.linalg.norm(Q - np.asarray(q_new, np.float64), axis=1)
    g = np.array([float(tree.g[k]) for k in ks])
    out = [(float(g[j] - c[j]), int(ks[j]), float(c[j])) for j in np.nonzero(c < g)[0]]
    out.sort(key=lambda t: (-t[0], t[1]))
    return [(k, c) for _, k, c in out[:slots]]


def refresh_costs(tree):
    """Cost-to-come of every vertex recomputed along its parent chain (sum of
    the edge lengths from the root), after rewiring changed parents."""
    for v in range(len(tree)):
        chain, u = [], v
        while u >= 0:
            chain.append(u)
            u = tree.parent[u]
            if len(chain) > len(tree):
                raise RuntimeError("cycle in the tree")
        chain.reverse()
        g = 0.0
        for a, b in zip(chain, chain[1:]):
            g += float(np.linalg.norm(tree.q[b].astype(np.float64) - tree.q[a].astype(np.float64)))
        tree.g[v] = np.float32(g)


@dataclass
class RewireOutcome(RoundOutcome):
    proposals: list = field(default_factory=list)  # (i, z, new cost): rewiring edges checked, candidate order
    pvalid: list = field(default_factory=list)     # their edge bits
    rewired: list = field(default_factory=list)    # (z, index of its new parent) applied, in order


def rewire_round(osc, roadmaps, ta, tb, draws, c_best: float, params: PlanParams, composite) -> RewireOutcome:
    """One round of the ao-dRRT baseline against the round-start trees: for
    each draw, NEAREST in T_a (no budget), dRRT's oracle, the cheapest parent
    among T_a's tensor-product neighbours of q_new, and up to RW_SLOTS
    rewiring proposals; then the checks of the extension edges (parent ->
    q_new), the connections (budget c_best - g_new) and the proposals;
    insertion in candidate order; the cheapest free connection; the
    proposals of inserted candidates applied in candidate and slot order
    when still cheaper; costs refreshed along the parent chains."""
    out = RewireOutcome()
    R = len(roadmaps)
    na, nb = len(ta), len(tb)
    Va, ga = np.array(ta.q[:na], np.float32), np.array(ta.g[:na], np.float32)
    Vb, gb = np.array(tb.q[:nb], np.float32), np.array(tb.g[:nb], np.float32)
    q_off = np.concatenate([[0], np.cumsum([len(rm.V[0]) for rm in roadmaps])]).astype(int)
    props = []
    for i, (q_rand, _) in enumerate(draws):
        k_near = nearest(Va, ga, np.asarray(q_rand, np.float32), math.inf)
        if k_near < 0:
            continue
        arms = [np.asarray(q_rand, np.float64)[q_off[r]:q_off[r + 1]] for r in range(R)]
        vid_new = tuple(aox_oracle(roadmaps, ta.vid[k_near], arms))
        if vid_new == ta.vid[k_near]:
            continue
        q_new = composite(vid_new)
        g_new, parent = best_parent(ta, na, roadmaps, vid_new, q_new)
        out.cands.append((i, parent, vid_new, q_new, g_new))
        props.append(rewire_proposals(ta, na, roadmaps, vid_new, q_new, g_new, parent))
    if out.cands:
        qa = np.array([ta.q[c[1]] for c in out.cands], np.float32)
        qb = np.array([c[3] for c in out.cands], np.float32)
        valid, n, _ = validate_fast(osc, qa, qb, params.resolution)
        out.valid = [bool(v) for v in valid]
        out.edge_states += int(n.sum())
    # connections, searched for every candidate before its extension edge is
    # known to be free (the other tree does not change in the round)
    conn = [nearest(Vb, gb, c[3], connect_budget(c_best, c[4])) for c in out.cands]
    for c, ps in zip(out.cands, props):
        for z, cost in ps:
            out.proposals.append((c[0], z, cost))
    if out.proposals:
        qa = np.array([out.cands[[c[0] for c in out.cands].index(i)][3] for i, _, _ in out.proposals], np.float32)
        qb = np.array([ta.q[z] for _, z, _ in out.proposals], np.float32)
        valid, _, _ = validate_fast(osc, qa, qb, params.resolution)
        out.pvalid = [bool(v) for v in valid]
    slot = {}
    for c, v in zip(out.cands, out.valid):
        out.overflow |= v and len(ta) >= params.max_tree_nodes
        if v and len(ta) < params.max_tree_nodes:
            ta.q.append(c[3])
            ta.g.append(np.float32(c[4]))
            ta.parent.append(c[1])
            ta.vid.append(c[2])
            out.inserted.append((c[0], len(ta) - 1))
            slot[c[0]] = len(ta) - 1
    cand_conn = {c[0]: kc for c, kc in zip(out.cands, conn)}
    for ci, idx in out.inserted:
        if cand_conn[ci] >= 0:
            out.conns.append((ci, idx, cand_conn[ci]))
    if out.conns:
        qa = np.array([ta.q[c[1]] for c in out.conns], np.float32)
        qb = np.array([tb.q[c[2]] for c in out.conns], np.float32)
        valid, n, _ = validate_fast(osc, qa, qb, params.resolution)
        out.cvalid = [bool(v) for v in valid]
        out.edge_states += int(n.sum())
        for (ci, idx, kc), v in zip(out.conns, out.cvalid):
            if not v:
                continue
            tot = float(ta.g[idx]) + float(np.linalg.norm(ta.q[idx].astype(np.float64) -
                                                          tb.q[kc].astype(np.float64))) + float(tb.g[kc])
            if out.best is None or tot < out.best[0]:
                out.best = (tot, ci, idx, kc)
    for (i, z, cost), v in zip(out.proposals, out.pvalid):
        if v and i in slot and cost < float(ta.g[z]):
            ta.parent[z] = slot[i]
            ta.g[z] = np.float32(cost)
            out.rewired.append((z, slot[i]))
    if out.rewired:
        refresh_costs(ta)
    return out


def steer(q_near: np.ndarray, q_rand: np.ndarray, step: float) -> np.ndarray:
    """Direct-mode extension (no roadmap layer): q_rand itself when it lies
    within `step` of q_near (Euclidean), else the point at distance `step`
    from q_near on the segment toward q_rand.  FP64."""
    q_near = np.asarray(q_near, np.float64)
    q_rand = np.asarray(q_rand, np.float64)
    d = q_rand - q_near
    dist = float(np.linalg.norm(d))
    if dist <= step:
        return q_rand.copy()
    return q_near + (step / dist) * d


def plan(scene, q_start, q_goal, params: PlanParams, warm_path=None) -> PlanResult:
    """Alg. 1 with the subroutines of Alg. 2, in rounds of P candidates.
    warm_path: a collision-free path (start to goal) to improve on; it is the
    result when no strictly cheaper path is found."""
    osc = OracleScene(scene)
    R, D = scene.n_robots, scene.dof
    q_off = np.concatenate([[0], np.cumsum([m.n_joints for m in scene.models])]).astype(int)
    q_start = np.asarray(q_start, np.float32)
    q_goal = np.asarray(q_goal, np.float32)
    _, m_ends = classify_edges(osc, np.stack([q_start, q_goal]), np.stack([q_start, q_goal]), 1.0)
    if m_ends[0] < 0:
        return PlanResult("E_START_INVALID", None, math.inf, 0, 0)
    if m_ends[1] < 0:
        return PlanResult("E_GOAL_INVALID", None, math.inf, 0, 0)
    lo, hi = scene.q_lo.astype(np.float64), scene.q_hi.astype(np.float64)
    arm_scenes = [OracleScene(_arm_scene(scene, r)) for r in range(R)]
    roadmaps = [_Roadmap(q_start[q_off[r]:q_off[r + 1]], q_goal[q_off[r]:q_off[r + 1]]) for r in range(R)]
    c_best, best_path, costs, history, trace = math.inf, None, [], [], []
    if warm_path is not None:
        best_path = np.asarray(warm_path, np.float32)
        c_best = _cost(best_path)
    rnd, it, first_round, edge_states = 0, 0, -1, 0
    solved = overflow = False

    def composite(vid):
        return np.concatenate([roadmaps[r].V[vid[r]] for r in range(R)]).astype(np.float32)

    t0 = time.perf_counter()
    out_of_time = lambda: params.time_budget_s > 0 and time.perf_counter() - t0 >= params.time_budget_s
    ta = tb = None
    while it < params.max_iterations and rnd < params.max_rounds and not out_of_time():
        if not params.direct and not roadmap_step(scene, roadmaps, arm_scenes, params, it, q_off):
            # ROADMAP (Alg. 2) grows until every arm connects its start and
            # goal; until then the tensor product holds no start-goal path
            it += 1
            continue
        if ta is None or not params.rewire:  # ao-dRRT keeps its trees across searches
            ta, tb = _new_tree(q_start, tuple([0] * R)), _new_tree(q_goal, tuple([1] * R))
            a_is_start = True
        solved = False
        while not solved and rnd < params.max_rounds and not out_of_time():
            if needs_swap(ta, tb):
                ta, tb = tb, ta
                a_is_start = not a_is_start
            trace.append((rnd, a_is_start, len(ta), len(tb)))
            root_a = ta.q[0].astype(np.float64)
            draws = [draw_candidate(params.seed, rnd, i, c_best, lo, hi, q_start, q_goal, root_a)
                     for i in range(params.candidates)]
            if params.rewire:
                out = rewire_round(osc, roadmaps, ta, tb, draws, c_best, params, composite)
            else:
                out = search_round(osc, roadmaps, ta, tb, draws, c_best, params, composite)
            edge_states += out.edge_states
            if out.best is not None:
                _, _, ia, ib = out.best
                path = _path_to_root(ta, ia) + _path_to_root(tb, ib)[::-1]
                if not a_is_start:
                    path = path[::-1]
                cost = _cost(path)
                if cost < c_best:
                    c_best, best_path = cost, np.array(path, np.float32)
                    costs.append(cost)
                    history.append((cost, best_path, rnd))
                    if first_round < 0:
                        first_round = rnd
                    solved = True
            rnd += 1
            if out.overflow and not solved:  # the tree is full: this search is over
                overflow = True
                break
        it += 1
        if solved and params.stop_at_first:
            break
        if overflow and not solved and params.rewire:  # its trees persist, full
            break
    status = "OK" if best_path is not None else ("E_CAPACITY" if overflow else "E_NO_SOLUTION")
    trees = () if ta is None else ((ta, tb) if a_is_start else (tb, ta))
    return PlanResult(status, best_path, c_best, rnd, it, first_round, costs, edge_states, roadmaps, solved, history,
                      trace, trees)


def ranked_history(result: PlanResult, max_entries: int = 64):
    """The incumbents as optimiser seeds (Sec. "Seeding for Multi-Robot
    Jerk-Free Motion"): cheapest first, at most max_entries of them -- when
    there are more paths than seeds, the cheaper ones are kept."""
    return sorted(result.history, key=lambda e: e[0])[:max_entries]


def replan(scene, q_start, q_goal, params: PlanParams, prev_path):
    """One replanning tick (Sec. "Hardware Deployment": replanning amid moving
    obstacles): the previous path is kept as the incumbent when it runs
    exactly from q_start to q_goal and every edge of it is free in the
    current environment; then only strictly cheaper paths replace it.
    Otherwise the planner starts from scratch.  Returns (result, kept)."""
    kept = False
    if prev_path is not None and len(prev_path) >= 2:
        prev = np.asarray(prev_path, np.float32)
        if np.array_equal(prev[0], np.asarray(q_start, np.float32)) and \
                np.array_equal(prev[-1], np.asarray(q_goal, np.float32)):
            valid, _, _ = validate_fast(OracleScene(scene), prev[:-1], prev[1:], params.resolution)
            kept = bool(np.all(valid))
    return plan(scene, q_start, q_goal, params, warm_path=prev_path if kept else None), kept
