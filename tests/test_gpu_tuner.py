"""The tile-shape autotuner through the C ABI: the first launch of a kind is
measured at several shapes and the fastest is kept (in memory and in the
JSON cache file); later launches of that kind are not measured again; a
cached choice is used as written; and the bits never depend on the shape."""
import json

import numpy as np
import pytest

import workloads as W
from gpu_common import problem

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    import paper_2609_30644_amd as M
    c = M.Context(0)
    yield c
    c.tuner_configure(None, True)  # the process defaults again: no file, measuring on
    c.close()


def _lines(path):
    return [json.loads(x) for x in open(path).read().splitlines() if x.strip()] if path.exists() else []


def test_tuner_measures_once_and_bits_do_not_change(ctx, tmp_path):
    import paper_2609_30644_amd as M
    p = problem("c2")
    s = M.Scene(ctx, p.scene)
    qa, qb = W.edge_batch(p.scene, 700, 0.05, 5, 8, 64)
    ctx.tuner_configure(None, False)
    rule = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    f = tmp_path / "tiles.json"
    ctx.tuner_configure(str(f), True)
    assert ctx.tuner_entries() == 0
    print("[tuner] first launch (measured)", flush=True)
    first = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    rows = _lines(f)
    assert len(rows) == 1 and ctx.tuner_entries() == 1
    r = rows[0]
    assert (r["path"], r["arms"], r["obstacles"]) == ("general", 4, 64)
    assert len(r["measured_us"]) >= 2 and str(r["waves"]) in r["measured_us"]
    assert r["measured_us"][str(r["waves"])] == min(r["measured_us"].values())
    again = s.validate_edges(qa, qb, 0.05).cpu().numpy()
    assert len(_lines(f)) == 1  # known kind: not measured again
    np.testing.assert_array_equal(first, rule)
    np.testing.assert_array_equal(again, rule)
    # the planner's one-launch batches are another kind, measured once each
    res = s.plan(p.q_start, p.q_goal, raise_on_error=False, seed=1, candidates=64, max_rounds=20, max_iterations=1,
                 n_roadmap=16, delta=3.0)
    kinds = {(x["path"], x["arms"], x["bucket"]) for x in _lines(f)}
    assert any(k[0] == "small" for k in kinds) and len(kinds) == len(_lines(f))
    # a later process loads the file: same choices, nothing measured
    ctx.tuner_configure(str(f), False)
    assert ctx.tuner_entries() == len(_lines(f))
    res2 = s.plan(p.q_start, p.q_goal, raise_on_error=False, seed=1, candidates=64, max_rounds=20,
                  max_iterations=1, n_roadmap=16, delta=3.0)
    assert res2.status == res.status and res2.cost == res.cost


def test_tuner_uses_cached_choice(ctx, tmp_path):
    import paper_2609_30644_amd as M
    p = problem("c2")
    s = M.Scene(ctx, p.scene)
    qa, qb = W.edge_batch(p.scene, 1500, 0.05, 6, 8, 64)
    bucket = int(np.ceil(np.log2(1500)))
    f = tmp_path / "tiles.json"
    for waves in (4, 16):
        f.write_text(json.dumps({"path": "general", "arms": 4, "spheres": 59, "obstacles": 64, "bucket": bucket,
                                 "waves": waves}) + "\n")
        ctx.tuner_configure(str(f), False)
        assert ctx.tuner_entries() == 1
        ctx.profile_enable(True)
        v = s.validate_edges(qa, qb, 0.05).cpu().numpy()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        assert prof.block_threads == 64 * waves
        if waves == 4:
            v4 = v
    np.testing.assert_array_equal(v, v4)


def test_tuner_rejects_bad_flag(ctx):
    import paper_2609_30644_amd as M
    with pytest.raises(M.MrpopError):
        ctx._check(ctx._lib.mrpop_tuner_configure(None, 3), None)


def test_profile_times_every_kth_launch(ctx):
    """With a stride k, the first tile launch and then every k-th carry the
    timing events, while the work totals still cover every launch."""
    import paper_2609_30644_amd as M
    p = problem("c2")
    s = M.Scene(ctx, p.scene)
    qa, qb = W.edge_batch(p.scene, 600, 0.05, 7, 8, 64)
    s.validate_edges(qa, qb, 0.05)  # warm (and tuned) before the counted launches
    totals = []
    for stride in (1, 3):
        ctx.profile_enable(stride)
        for _ in range(7):
            s.validate_edges(qa, qb, 0.05)
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        assert prof.launches == 7 and prof.timed_launches == (7 if stride == 1 else 3)
        assert prof.kernel_ms > 0.0
        totals.append(prof.edge_states)
    assert totals[0] == totals[1] > 0
    with pytest.raises(M.MrpopError):
        ctx.profile_enable(-1)
