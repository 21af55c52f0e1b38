"""Parity of the HIP path (through the C ABI) against the FP64 oracle:
forward kinematics to 4e-6 m, edge bits exact outside the 1e-5 m band."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import BAND, assert_bits_match, problem

pytestmark = pytest.mark.gpu

FK_TOL = 4e-6  # metres; half the boundary band minus rounding of the tests


@pytest.fixture(scope="module")
def ctx():
    import paper_2609_30644_amd as M
    c = M.Context(0)
    yield c
    c.close()


def _scene(ctx, sc):
    import paper_2609_30644_amd as M
    return M.Scene(ctx, sc)


def _fk_err(ctx, sc, q):
    got = _scene(ctx, sc).fk_spheres(q).cpu().numpy().astype(np.float64)
    want = oracle.fk_spheres(sc, q)
    assert got.shape == want.shape
    np.testing.assert_array_equal(got[..., 3], want[..., 3].astype(np.float32))
    return np.abs(got[..., :3] - want[..., :3]).max()


@pytest.mark.parametrize("kind", ["c1", "c2", "c3"])
def test_fk_parity(ctx, kind):
    print(f"[fk_parity] {kind}", flush=True)
    sc = problem(kind).scene
    q = W.random_configs(sc, 512, np.random.default_rng(11))
    assert _fk_err(ctx, sc, q) <= FK_TOL


def test_fk_planar_closed_form(ctx):
    sc = W.Scene([W.planar_two_link(0.6, 0.4)], W.base_transform(0.2, -0.1, 0.3)[None],
                 np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    q = np.random.default_rng(0).uniform(-3, 3, (257, 2)).astype(np.float32)
    out = _scene(ctx, sc).fk_spheres(q).cpu().numpy().astype(np.float64)
    q64 = q.astype(np.float64)
    f = lambda v: float(np.float32(v))
    a = q64[:, 0] + 0.3
    x = f(0.6) * np.cos(a) + f(0.4) * np.cos(a + q64[:, 1])
    y = f(0.6) * np.sin(a) + f(0.4) * np.sin(a + q64[:, 1])
    np.testing.assert_allclose(out[:, 1, 0], f(0.2) + x, atol=FK_TOL)
    np.testing.assert_allclose(out[:, 1, 1], f(-0.1) + y, atol=FK_TOL)


def test_fk_empty_and_order(ctx):
    sc = problem("c1").scene
    s = _scene(ctx, sc)
    assert s.fk_spheres(np.zeros((0, sc.dof), np.float32)).shape == (0, sc.n_robots * 20, 4)
    # spheres come back in input order: radii match the model per robot
    out = s.fk_spheres(np.zeros((1, sc.dof), np.float32)).cpu().numpy()
    np.testing.assert_array_equal(out[0, :20, 3], sc.models[0].sphere_xyzr[:, 3])


def _parity(ctx, sc, qa, qb, res, what, n_states=None):
    print(f"[validate_parity] {what}: {qa.shape[0]} edges", flush=True)
    valid, st = _scene(ctx, sc).validate_edges(qa, qb, res, n_states=n_states, stats=True)
    valid = valid.cpu().numpy()
    n, m = oracle.classify_edges(sc, qa, qb, res, nstates=n_states)
    info = assert_bits_match(valid, m, what)
    assert st.edge_states == int(n.sum())
    assert st.edges_invalid == int((valid == 0).sum())
    if valid.all():  # no early exit: every state is evaluated (the kernels' work sums)
        assert st.states_checked == st.edge_states
    print(f"  {info} states={st.edge_states} checked={st.states_checked}", flush=True)
    return valid, m, st


@pytest.mark.parametrize("kind,res", [("c1", 0.05), ("c2", 0.05), ("c3", 0.02)])
def test_validate_random_edges(ctx, kind, res):
    sc = problem(kind).scene
    E = 1024 if kind != "c3" else 256
    qa, qb = W.edge_batch(sc, E, res, 100, 8, 64)
    _parity(ctx, sc, qa, qb, res, f"{kind}/random")


@pytest.mark.parametrize("kind,res", [("c1", 0.05), ("c2", 0.05), ("c3", 0.02)])
def test_validate_near_free_edges(ctx, kind, res):
    """Edges anchored at oracle-free states: a real mix of free and colliding
    edges, so both bit values are exercised."""
    p = problem(kind)
    sc = p.scene
    rng = np.random.default_rng(5)
    anchors = W.random_configs(sc, 4000 if kind != "c3" else 1500, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    anchors = np.concatenate([anchors, p.q_start[None], p.q_goal[None]])
    E = 1024 if kind != "c3" else 256
    qa, qb = W.edge_batch_near(sc, anchors, E, res, 101, 2, 40, spread=0.02)
    valid, m, _ = _parity(ctx, sc, qa, qb, res, f"{kind}/near")
    assert 0 < valid.sum() < E, "batch should mix free and colliding edges"


def test_validate_c2_full_batch(ctx):
    """4096 edges at the workload's full batch size, every edge checked."""
    p = problem("c2")
    sc = p.scene
    rng = np.random.default_rng(6)
    anchors = W.random_configs(sc, 6000, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    qa, qb = W.edge_batch_near(sc, anchors, 4096, 0.05, 102, 8, 64, spread=0.02)
    _parity(ctx, sc, qa, qb, 0.05, "c2/full")


@pytest.mark.parametrize("kind", ["c2", "c3"])
def test_validate_certainly_free_batch_work_sums(ctx, kind):
    """The benchmark's certainly-free batch (4096 edges the oracle found free
    away from the boundary band): every edge is valid, so no state exits
    early, and the kernels' summed work counters obey their invariants:
    every state is checked, every arm's chain runs at every state, and every
    link with spheres is placed once per chain."""
    import bench
    sc, batches, fx = bench.load_workload(*((bench.FIXTURE, "scene_c2") if kind == "c2" else
                                            (bench.C3_FIXTURE, "scene_c3")))
    qa, qb = batches["free"]
    res = float(fx["resolution"])
    print(f"[free_batch] {kind}: {qa.shape[0]} edges", flush=True)
    valid, st = _scene(ctx, sc).validate_edges(qa, qb, res, stats=True)
    assert valid.cpu().numpy().all()
    n = oracle.edge_nstates(qa, qb, res)
    assert st.edge_states == int(n.sum()) == st.states_checked
    links_per_arm = sum(1 for l in range(sc.models[0].n_joints + 1) if (sc.models[0].sphere_link == l).any())
    w = st.work
    assert w["chains"] == sc.n_robots * st.edge_states
    assert w["links"] == links_per_arm * w["chains"]


def test_validate_degenerate_edges(ctx):
    p = problem("c2")
    sc = p.scene
    q = np.stack([p.q_start, p.q_goal])
    # null edges (n = 1), an explicit state count, and a NaN endpoint
    valid, st = _scene(ctx, sc).validate_edges(q, q, 0.05, stats=True)
    assert valid.cpu().numpy().tolist() == [1, 1] and st.edge_states == 2
    qa = np.stack([p.q_start, p.q_start, p.q_start])
    qb = np.stack([p.q_goal, p.q_goal, p.q_goal])
    qb[2, 3] = np.nan
    ns = np.array([1, 7, 5], np.int32)
    valid, st = _scene(ctx, sc).validate_edges(qa, qb, 0.05, n_states=ns, stats=True)
    v = valid.cpu().numpy()
    assert v[2] == 0 and st.nonfinite_edges == 1
    n, m = oracle.classify_edges(sc, qa[:2], qb[:2], 0.05, nstates=ns[:2])
    assert_bits_match(v[:2], m, "explicit n")
    assert st.edge_states == 1 + 7


def test_validate_empty_batch(ctx):
    sc = problem("c1").scene
    z = np.zeros((0, sc.dof), np.float32)
    valid, st = _scene(ctx, sc).validate_edges(z, z, 0.05, stats=True)
    assert valid.numel() == 0 and st.edge_states == 0


def test_validate_long_edges_span_many_tiles(ctx):
    p = problem("c1")
    sc = p.scene
    rng = np.random.default_rng(7)
    anchors = W.random_configs(sc, 3000, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    qa, qb = W.edge_batch_near(sc, anchors, 64, 0.002, 103, 300, 700, spread=0.0)
    _parity(ctx, sc, qa, qb, 0.002, "c1/long")


def test_validate_single_arm_and_mixed_models(ctx):
    rng = np.random.default_rng(8)
    one = W.Scene([W.panda_like(59)], W.base_transform(0, 0, 0)[None],
                  np.array([[0.4, 0.2, 0.5, 0.1], [-0.3, -0.4, 0.8, 0.12]], np.float32),
                  np.array([[0.3, -0.5, 0.0, 0.6, -0.2, 0.4]], np.float32))
    qa, qb = W.edge_batch(one, 512, 0.05, 104, 2, 30)
    _parity(ctx, one, qa, qb, 0.05, "single arm")
    mixed = W.Scene([W.panda_like(20), W.panda_like(59), W.planar_two_link()],
                    np.stack([W.base_transform(-0.5, 0, 0), W.base_transform(0.5, 0, math.pi),
                              W.base_transform(0.0, 0.6, -math.pi / 2, 0.4)]),
                    np.array([[0.0, 0.0, 0.6, 0.1]], np.float32), np.array([[0.1, 0.3, 0.0, 0.3, 0.5, 0.2]], np.float32))
    qa, qb = W.edge_batch(mixed, 512, 0.05, 105, 2, 30)
    _parity(ctx, mixed, qa, qb, 0.05, "mixed models")


def test_validate_deterministic(ctx):
    sc = problem("c2").scene
    qa, qb = W.edge_batch(sc, 2048, 0.05, 106, 8, 64)
    s = _scene(ctx, sc)
    a = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    b = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    assert (a == b).all()


def test_validate_scene_too_large_for_lds_staging(ctx):
    """Thousands of small obstacles: the scene's filter rows exceed the LDS
    budget, so the tile kernel reads them from global memory instead."""
    rng = np.random.default_rng(9)
    base = problem("c1").scene
    ns, nb = 700, 700  # 8 links x 1400 rows x 16 B: beyond the staging budget
    cs = rng.uniform([-1.5, -1.5, 0.0], [1.5, 1.5, 1.6], (ns, 3))
    sph = np.concatenate([cs, rng.uniform(0.005, 0.02, (ns, 1))], 1).astype(np.float32)
    lo = rng.uniform([-1.5, -1.5, 0.0], [1.5, 1.5, 1.6], (nb, 3))
    box = np.concatenate([lo, lo + rng.uniform(0.005, 0.03, (nb, 3))], 1).astype(np.float32)
    sc = base.with_env(sph, box)
    anchors = W.random_configs(sc, 4000, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    assert len(anchors) > 64
    qa, qb = W.edge_batch_near(sc, anchors, 384, 0.05, 107, 2, 8, spread=0.0)
    _parity(ctx, sc, qa, qb, 0.05, "large env (global rows)")


def _shelf_mix(ns, nb, seed):
    """The 8-arm shelf scene with its first nb boxes and ns small spheres on
    the shelves of one quarter of the grid."""
    sc = problem("c3").scene
    rng = np.random.default_rng(seed)
    mid = 0.5 * (sc.env_boxes[:, :3] + sc.env_boxes[:, 3:])
    corner = np.nonzero((mid[:, 0] < 0) & (mid[:, 1] < 0))[0]
    c = mid[rng.choice(corner, ns, replace=ns > len(corner))] + rng.uniform(-0.1, 0.1, (ns, 3))
    sph = np.concatenate([c, rng.uniform(0.02, 0.06, (ns, 1))], 1).astype(np.float32)
    return sc.with_env(sph, sc.env_boxes[:nb].copy())


def _sparse_mix(ns, nb, seed):
    """The 4-arm scene with ns spheres and nb boxes scattered over 3.6 m."""
    rng = np.random.default_rng(seed)
    cs = rng.uniform([-1.8, -1.8, 0.0], [1.8, 1.8, 1.5], (ns, 3))
    sph = np.concatenate([cs, rng.uniform(0.01, 0.04, (ns, 1))], 1).astype(np.float32)
    lo = rng.uniform([-1.8, -1.8, 0.0], [1.8, 1.8, 1.5], (nb, 3))
    box = np.concatenate([lo, lo + rng.uniform(0.02, 0.08, (nb, 3))], 1).astype(np.float32)
    return problem("c2").scene.with_env(sph, box)


@pytest.mark.parametrize("kind,ns,nb,clusters", [("shelf", 37, 210, True), ("shelf", 200, 0, True),
                                                  ("shelf", 0, 256, True), ("sparse", 50, 47, False)])
def test_validate_obstacle_lists(ctx, kind, ns, nb, clusters):
    """Each link tests only the obstacles within its reach of its arm's base,
    and a long list of dense obstacles first tests clusters of eight (in
    Morton order: here spheres and boxes mixed in one list, ragged last
    clusters, and the full shelf grid), while a sparse scene keeps one level.
    The bits equal the oracle's either way, and fewer coarse tests run than
    one per link and obstacle."""
    seed = ns * 1000 + nb
    sc = _shelf_mix(ns, nb, seed) if kind == "shelf" else _sparse_mix(ns, nb, seed)
    res = 0.02 if kind == "shelf" else 0.05
    rng = np.random.default_rng(seed)
    anchors = W.random_configs(sc, 1500 if kind == "shelf" else 3000, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    assert len(anchors) > 8
    qa, qb = W.edge_batch_near(sc, anchors, 256, res, 110, 2, 40 if kind == "shelf" else 24,
                               spread=0.02 if kind == "shelf" else 0.3)
    n_clusters = _scene(ctx, sc).obstacle_clusters
    print(f"[clusters] {kind} {ns}+{nb}: {n_clusters} clusters", flush=True)
    assert (n_clusters > 0) == clusters
    valid, m, st = _parity(ctx, sc, qa, qb, res, f"{kind} env {ns}+{nb}")
    assert (m < -BAND).any() and (m > BAND).any()
    w = st.work
    print(f"  coarse tests {w['env_tests']} links {w['links']} per link {w['env_tests'] / w['links']:.1f}", flush=True)
    assert w["env_tests"] < w["links"] * (ns + nb)


def test_validate_no_obstacles_arm_pairs_only(ctx):
    sc = problem("c2").scene
    empty = sc.with_env(np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    qa, qb = W.edge_batch(empty, 1024, 0.05, 108, 8, 64)
    valid, m, _ = _parity(ctx, empty, qa, qb, 0.05, "no obstacles")
    assert (m < -BAND).any() and (m > BAND).any()  # both outcomes present


@pytest.mark.parametrize("mode", ["lds", "scalar"])
def test_validate_tile_modes(ctx, mode):
    """Both places the tile kernel can read its coarse rows from give the
    oracle's bits (and the same bits as each other)."""
    p = problem("c2")
    sc = p.scene
    rng = np.random.default_rng(10)
    anchors = W.random_configs(sc, 3000, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    qa, qb = W.edge_batch_near(sc, anchors, 1024, 0.05, 109, 2, 48)
    s = _scene(ctx, sc)
    s.set_tile_mode(mode)
    assert s.tile_mode == mode
    print(f"[validate_parity] tile mode {mode}", flush=True)
    got = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    _, m = oracle.classify_edges(sc, qa, qb, 0.05)
    print(f"  {assert_bits_match(got, m, f'tile mode {mode}')}", flush=True)
    s.set_tile_mode("auto")
    assert np.array_equal(got, s.validate_edges(qa, qb, 0.05).cpu().numpy())


@pytest.mark.parametrize("case", ["single3000", "c2_1025"])
def test_validate_one_workgroup_count_in_chunks(ctx, case):
    """Batches above 1024 edges whose endpoint coordinates (edges x dof) stay
    within 32768 are counted and scanned by one workgroup, 1024 edges at a
    time: a one-arm batch of three chunks (the last one ragged) and a
    composite batch whose second chunk holds a single edge."""
    if case == "single3000":
        sc = W.Scene([W.panda_like(59)], W.base_transform(0, 0, 0)[None],
                     np.array([[0.4, 0.2, 0.5, 0.1], [-0.3, -0.4, 0.8, 0.12]], np.float32),
                     np.array([[0.3, -0.5, 0.0, 0.6, -0.2, 0.4]], np.float32))
        qa, qb = W.edge_batch(sc, 3000, 0.05, 111, 2, 30)
    else:
        sc = problem("c2").scene
        qa, qb = W.edge_batch(sc, 1025, 0.05, 112, 2, 40)
    assert 1024 < qa.shape[0] and qa.shape[0] * sc.dof <= 32768
    _parity(ctx, sc, qa, qb, 0.05, case)


def test_validate_more_edges_than_one_scan_block(ctx):
    """More than 4096 edges take the multi-block count and scan path."""
    sc = problem("c1").scene
    qa, qb = W.edge_batch(sc, 6000, 0.05, 110, 1, 40)
    _parity(ctx, sc, qa, qb, 0.05, "c1/6000 edges")


@pytest.mark.parametrize("spheres", [20, 59])
def test_validate_sixteen_arms(ctx, spheres):
    """Sixteen arms (the largest served queries): the joint sine/cosine cache
    no longer fits next to the published centres, so the arm-pair stage
    rebuilds frames from the joint values."""
    m = W.panda_like(spheres)
    R = 16
    sc = W.Scene([m] * R, W.ring_bases(R, W.ring_radius_for_spacing(R, 1.0)),
                 np.array([[0.0, 0.0, 0.5, 0.2]], np.float32), np.zeros((0, 6), np.float32))
    qa, qb = W.edge_batch(sc, 256, 0.05, 111, 2, 24)
    _, m_, _ = _parity(ctx, sc, qa, qb, 0.05, f"16 arms x {spheres} spheres")
    assert (m_ < -BAND).any() and (m_ > BAND).any()


def _long_link_arm(n_tool: int) -> "W.RobotModel":
    """Planar 2R arm whose second link carries n_tool small spheres."""
    dh = np.array([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0]], np.float32)
    xs = np.linspace(0.02, 0.45, n_tool)
    xyzr = [[0.25, 0.0, 0.0, 0.05]] + [[x, 0.0, 0.0, 0.012] for x in xs]
    return W.RobotModel("planar_long_link", dh, np.array([-math.pi] * 2, np.float32), np.array([math.pi] * 2, np.float32),
                        np.array([1] + [2] * n_tool, np.int32), np.array(xyzr, np.float32))


@pytest.mark.parametrize("n_tool", [40, 100])
def test_validate_arm_pairs_with_many_spheres_per_link(ctx, n_tool):
    """Arm-pair fine tests where a link has fewer or more than 64 spheres."""
    m = _long_link_arm(n_tool)
    sc = W.Scene([m, m], np.stack([W.base_transform(-0.35, 0, 0), W.base_transform(0.35, 0, math.pi)]),
                 np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))
    qa, qb = W.edge_batch(sc, 512, 0.05, 112, 2, 30)
    _, m_, _ = _parity(ctx, sc, qa, qb, 0.05, f"pairs, {n_tool} spheres on a link")
    assert (m_ < -BAND).any() and (m_ > BAND).any()


@pytest.mark.parametrize("kind,res,E,n_min,n_max", [("c1", 0.05, 40, 2, 30), ("c2", 0.05, 1024, 2, 40),
                                                   ("c2", 0.05, 1024, 20, 120), ("c3", 0.02, 600, 20, 60)])
def test_validate_counted_matches_oracle_and_general_path(ctx, kind, res, E, n_min, n_max):
    """mrpop_validate_counted (one launch from the caller's state counts; more
    tiles than workgroups run the two-pass state order) against the oracle
    outside the band, and bit for bit against mrpop_validate_edges with the
    same counts.  Sizes: a batch of fewer tiles than workgroups (plain order),
    the planner's round size, edges of up to 120 states (several tiles per
    edge), and the 8-arm shelf scene."""
    p = problem(kind)
    sc = p.scene
    anchors = W.random_configs(sc, 4000 if kind != "c3" else 1500, np.random.default_rng(7))
    anchors = np.concatenate([anchors[oracle.states_free(sc, anchors)], p.q_start[None], p.q_goal[None]])
    qa, qb = W.edge_batch_near(sc, anchors, E, res, 103, n_min, n_max, spread=0.02)
    n = oracle.edge_nstates(qa, qb, res)
    print(f"[validate_counted] {kind}: {E} edges, {int(n.sum())} states", flush=True)
    s = _scene(ctx, sc)
    valid, st = s.validate_counted(qa, qb, n, stats=True)
    valid = valid.cpu().numpy()
    plain, st_plain = s.validate_edges(qa, qb, res, n_states=n, stats=True)
    _, m = oracle.classify_edges(sc, qa, qb, res, nstates=n)
    info = assert_bits_match(valid, m, f"{kind}/counted")
    np.testing.assert_array_equal(valid, plain.cpu().numpy())
    assert st.edge_states == st_plain.edge_states == int(n.sum())
    assert st.edges_invalid == int((valid == 0).sum())
    assert 0 < st.states_checked <= st.edge_states
    if valid.all():
        assert st.states_checked == st.edge_states
    print(f"  {info} checked {st.states_checked} of {st.edge_states} (general path {st_plain.states_checked})",
          flush=True)


def test_validate_counted_codes_and_limits(ctx):
    """Counts <= 0 report the edge invalid unchecked (the extension kernel
    writes -1 for a non-finite endpoint, -2 for an edge too long); a free
    batch is wholly evaluated; more than MRPOP_COUNTED_MAX_EDGES edges and a
    missing count array are rejected."""
    import paper_2609_30644_amd as M
    p = problem("c2")
    sc = p.scene
    anchors = W.random_configs(sc, 4000, np.random.default_rng(8))
    anchors = anchors[oracle.states_free(sc, anchors)]
    qa = np.resize(anchors, (1024, anchors.shape[1]))  # free states, repeated
    n = np.ones(1024, np.int32)  # each edge its free start state alone
    n[[3, 500]] = [0, -1]
    s = _scene(ctx, sc)
    valid, st = s.validate_counted(qa, qa, n, stats=True)
    valid = valid.cpu().numpy()
    want = (n > 0) & (oracle.state_margins(sc, qa) >= BAND)
    np.testing.assert_array_equal(valid.astype(bool), want)
    assert st.edge_states == st.states_checked == int((n > 0).sum())
    assert st.nonfinite_edges == 1 and st.edges_invalid == 2
    # a too-long edge: its bit is 0; with stats the call reports it as
    # mrpop_validate_edges does
    n[1023] = -2
    valid = s.validate_counted(qa, qa, n).cpu().numpy()
    np.testing.assert_array_equal(valid.astype(bool), (n > 0) & want)
    with pytest.raises(M.MrpopError) as e:
        s.validate_counted(qa, qa, n, stats=True)
    assert e.value.name == "E_INVALID_ARG"
    with pytest.raises(M.MrpopError) as e:
        s.validate_counted(np.concatenate([qa, qa[:1]]), np.concatenate([qa, qa[:1]]), np.ones(1025, np.int32))
    assert e.value.name == "E_INVALID_ARG"
    with pytest.raises(M.MrpopError) as e:
        s.validate_counted(qa, qa, None)
    assert e.value.name == "E_INVALID_ARG"


def test_validate_counted_sixteen_arms(ctx):
    """The counted path on sixteen 20-sphere arms: the sine/cosine cache does
    not fit, so the two-pass order runs in the kernel variant that composes
    whole chains; bits against the oracle and against the general path."""
    m = W.panda_like(20)
    R = 16
    sc = W.Scene([m] * R, W.ring_bases(R, W.ring_radius_for_spacing(R, 1.0)),
                 np.array([[0.0, 0.0, 0.5, 0.2]], np.float32), np.zeros((0, 6), np.float32))
    qa, qb = W.edge_batch(sc, 1024, 0.05, 112, 20, 50)
    n = oracle.edge_nstates(qa, qb, 0.05)
    print(f"[validate_counted] 16 arms: {int(n.sum())} states", flush=True)
    s = _scene(ctx, sc)
    valid, st = s.validate_counted(qa, qb, n, stats=True)
    valid = valid.cpu().numpy()
    plain = s.validate_edges(qa, qb, 0.05, n_states=n).cpu().numpy()
    _, marg = oracle.classify_edges(sc, qa, qb, 0.05, nstates=n)
    info = assert_bits_match(valid, marg, "16 arms/counted")
    np.testing.assert_array_equal(valid, plain)
    assert st.edge_states == int(n.sum()) and 0 < st.states_checked <= st.edge_states
    print(f"  {info} checked {st.states_checked} of {st.edge_states}", flush=True)
