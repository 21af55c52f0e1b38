"""Parity of the extension step (ORACLE_AOX of Alg. 2, through mrpop_extend)
with the oracle's aox_oracle, candidate by candidate: the chosen roadmap
vertex of every arm, survival, q_new, g_new and the edge's state count.

Roadmaps and trees are random (vertices in the joint limits, random
adjacency with duplicated vertices, so that zero-length edges and exact
cosine ties occur), with budgets chosen so that admissibility and the
composite revert often decide.  A candidate counts as a near-tie, and is only
reported, when the oracle's own answer changes under tiny perturbations of
its budget, its cost-to-come or its sample (the GPU decides in single
precision)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import planner as PL

pytestmark = pytest.mark.gpu

RES = 0.05


@pytest.fixture(scope="module")
def ctx():
    import paper_2609_30644_amd as M
    c = M.Context(0)
    yield c
    c.close()


def _fixture(R, seed, n_rm=40, deg=6, n_tree=96, P=384):
    rng = np.random.default_rng([seed, R])
    model = W.panda_like(20)
    sc = W.Scene([model] * R, W.ring_bases(R, 0.6 + 0.25 * R), np.zeros((0, 4), np.float32),
                 np.zeros((0, 6), np.float32))
    lo, hi = model.q_lo.astype(np.float64), model.q_hi.astype(np.float64)
    roadmaps, rows = [], np.zeros((R, n_rm, 8), np.float32)
    for r in range(R):
        mid = lo + rng.random(7) * (hi - lo)
        V = np.clip(mid + (rng.random((n_rm, 7)) - 0.5) * 0.4 * (hi - lo), lo, hi).astype(np.float32)
        V[n_rm - 1] = V[5]  # duplicates: equal cosines, and a zero-length edge 3 - (n_rm - 2)
        V[n_rm - 2] = V[3]
        rm = PL._Roadmap(V[0], V[1])
        for q in V[2:]:
            rm.add_vertex(q)
        for i in range(n_rm):
            for j in rng.choice(n_rm, deg, replace=False):
                if j != i:
                    rm.add_edge(i, int(j))
        for i in range(n_rm):
            if 5 in rm.adj[i] and i != n_rm - 1:
                rm.add_edge(i, n_rm - 1)
        rm.add_edge(3, n_rm - 2)
        roadmaps.append(rm)
        rows[r, :, :7] = V
    col_cap = max(sum(len(rm.adj[i]) for i in range(n_rm)) for rm in roadmaps)
    rowptr = np.zeros((R, n_rm + 1), np.int32)
    col = np.full((R, col_cap), -1, np.int32)
    for r, rm in enumerate(roadmaps):
        k = 0
        for i in range(n_rm):
            nb = list(rm.adj[i])
            rng.shuffle(nb)  # the result must not depend on the order of a row
            col[r, k:k + len(nb)] = nb
            k += len(nb)
            rowptr[r, i + 1] = k
    vids = rng.integers(0, n_rm, (n_tree, R))
    tree_q = np.stack([np.concatenate([rows[r, vids[t, r], :7] for r in range(R)]) for t in range(n_tree)]).T.copy()
    tree_g = rng.uniform(0.0, 4.0, n_tree).astype(np.float32)
    near = rng.integers(0, n_tree, P).astype(np.int32)
    near[rng.random(P) < 0.05] = -1
    q_rand = np.concatenate([lo + rng.random((P, 7)) * (hi - lo) for _ in range(R)], axis=1).astype(np.float32)
    c_rand = (tree_g[np.maximum(near, 0)] + rng.uniform(0.3, 1.2, P) * math.sqrt(R)).astype(np.float32)
    c_rand[rng.random(P) < 0.3] = np.inf
    return dict(sc=sc, roadmaps=roadmaps, rows=rows, rowptr=rowptr, col=col, vids=vids, tree_q=tree_q,
                tree_g=tree_g, near=near, q_rand=q_rand, c_rand=c_rand)


def _oracle_one(f, i, g_shift=0.0, c_scale=1.0, q_shift=None):
    R = len(f["roadmaps"])
    k = f["near"][i]
    vid_near = tuple(int(x) for x in f["vids"][k])
    q = f["q_rand"][i].astype(np.float64) + (0 if q_shift is None else q_shift)
    arms = [q[7 * r:7 * r + 7] for r in range(R)]
    c = float(f["c_rand"][i]) * c_scale
    return tuple(PL.aox_oracle(f["roadmaps"], vid_near, arms, float(f["tree_g"][k]) * (1 + g_shift), c))


@pytest.mark.parametrize("R", [1, 2, 4, 8, 16])
def test_extend_matches_oracle(ctx, R):
    import paper_2609_30644_amd as M
    f = _fixture(R, 7)
    print(f"[extend] {R} arms, {len(f['near'])} candidates", flush=True)
    s = M.Scene(ctx, f["sc"])
    got = s.extend(f["near"], f["q_rand"], f["c_rand"], f["tree_q"], f["tree_g"], f["vids"].T.astype(np.int32),
                   f["rows"], f["rowptr"], f["col"], RES)
    rng = np.random.default_rng(99)
    D = 7 * R
    ties = differs_from_plain = reverted = compared = 0
    for i, k in enumerate(f["near"]):
        if k < 0:
            assert got["alive"][i] == 0 and np.all(got["vid_new"][:, i] == -1) and math.isinf(got["g_new"][i])
            continue
        want = _oracle_one(f, i)
        perturbed = {_oracle_one(f, i, c_scale=1 + e) for e in (-1e-5, 1e-5)}
        perturbed |= {_oracle_one(f, i, g_shift=e) for e in (-1e-5, 1e-5)}
        perturbed |= {_oracle_one(f, i, q_shift=rng.uniform(-2e-5, 2e-5, D)) for _ in range(3)}
        if perturbed != {want}:
            ties += 1
            continue
        compared += 1
        vid_near = tuple(int(x) for x in f["vids"][k])
        alive = want != vid_near
        assert tuple(got["vid_new"][:, i]) == want, (i, want, got["vid_new"][:, i])
        assert bool(got["alive"][i]) == alive
        q_near = f["tree_q"][:, k]
        q_new = np.concatenate([f["rows"][r, want[r], :7] for r in range(R)])
        np.testing.assert_array_equal(got["q_new"][i], q_new)
        g_want = float(f["tree_g"][k]) + float(np.linalg.norm(q_new.astype(np.float64) - q_near))
        assert abs(got["g_new"][i] - g_want) <= 2e-5 * max(1.0, g_want)
        if alive and math.isfinite(f["c_rand"][i]):
            assert got["g_new"][i] < f["c_rand"][i]
        np.testing.assert_array_equal(got["edge_a"][i], q_near)
        np.testing.assert_array_equal(got["edge_b"][i], q_new if alive else q_near)
        assert got["n_states"][i] == oracle.edge_nstates(q_near, got["edge_b"][i], RES)[0]
        # where the admissible-first rule decided
        plain = tuple(PL.aox_oracle(f["roadmaps"], vid_near,
                                    [f["q_rand"][i, 7 * r:7 * r + 7].astype(np.float64) for r in range(R)]))
        differs_from_plain += int(plain != want)
        for r in range(R):
            alone = PL.aox_oracle([f["roadmaps"][r]], (vid_near[r],),
                                  [f["q_rand"][i, 7 * r:7 * r + 7].astype(np.float64)], float(f["tree_g"][k]),
                                  float(f["c_rand"][i]))
            if want[r] == vid_near[r] and alone[0] != vid_near[r]:
                reverted += 1
                break
    print(f"  compared {compared}, near-ties {ties}, budget changed the choice {differs_from_plain}, "
          f"composite reverts {reverted}", flush=True)
    assert ties <= 0.05 * len(f["near"])
    assert differs_from_plain > 0
    if R >= 2:
        assert reverted > 0


def test_extend_rejects_bad_arguments(ctx):
    import ctypes as C
    import paper_2609_30644_amd as M
    f = _fixture(2, 1, P=8)
    s = M.Scene(ctx, f["sc"])
    st = ctx._lib.mrpop_extend(ctx.handle, s.handle, None, ctx.stream())
    assert M.STATUS_NAMES[st] == "E_INVALID_ARG"
    from paper_2609_30644_amd._binding import _ExtendBatch
    b = _ExtendBatch()
    b.n = 4  # buffers left NULL
    b.tree_cap = b.rm_cap = 1
    assert M.STATUS_NAMES[ctx._lib.mrpop_extend(ctx.handle, s.handle, C.byref(b), ctx.stream())] == "E_INVALID_ARG"
    b.n = 0
    assert ctx._lib.mrpop_extend(ctx.handle, s.handle, C.byref(b), ctx.stream()) == 0
