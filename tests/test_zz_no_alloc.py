"""The allocation-free validation entry point (mrpop_validate_edges_noalloc)
against mrpop_validate_edges, through the C ABI: identical bits and counters
on two calls in a row (the second smaller, so stale words of the first call
sit in the shared device array), the oracle's verdict outside the band, and
the size limit rejected on the host."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import assert_bits_match, problem

pytestmark = pytest.mark.gpu

MAX_EDGES = 65536  # MRPOP_NOALLOC_MAX_EDGES


@pytest.fixture(scope="module")
def c2():
    import paper_2609_30644_amd as M
    ctx = M.Context(0)
    p = problem("c2")
    yield M, ctx, M.Scene(ctx, p.scene), p
    ctx.close()


def _batch(p, n, seed):
    sc = p.scene
    rng = np.random.default_rng(seed)
    qa, qb = W.edge_batch(sc, n // 2, 0.05, seed, 8, 64)
    anchors = W.random_configs(sc, 3000, rng)
    anchors = anchors[oracle.states_free(sc, anchors)]
    na, nb = W.edge_batch_near(sc, anchors, n - n // 2, 0.05, seed + 1, 4, 40, spread=0.02)
    return np.concatenate([qa, na]), np.concatenate([qb, nb])


@pytest.mark.parametrize("sizes", [(1500, 333)])
def test_noalloc_equals_validate_two_calls(c2, sizes):
    import torch
    M, ctx, s, p = c2
    for k, n in enumerate(sizes):
        print(f"[noalloc] call {k}: {n} edges (C2 scene)", flush=True)
        qa, qb = _batch(p, n, 40 + k)
        ref, st_ref = s.validate_edges(qa, qb, 0.05, stats=True)
        got, st_got = s.validate_edges_noalloc(qa, qb, 0.05, stats=True)
        torch.cuda.synchronize()
        ref, got = ref.cpu().numpy(), got.cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        # (the executed-work counters depend on timing: lanes skip link jobs
        # once another wave has marked their edge colliding)
        assert (st_got.edge_states, st_got.edges_invalid, st_got.tiles) == \
            (st_ref.edge_states, st_ref.edges_invalid, st_ref.tiles)
        _, m = oracle.classify_edges(p.scene, qa, qb, 0.05)
        info = assert_bits_match(got, m, f"noalloc call {k}")
        assert 0 < info["valid"] < n
        # without stats, on the current stream, with explicit state counts
        ns = oracle.edge_nstates(qa, qb, 0.05)
        got2 = s.validate_edges_noalloc(qa, qb, 0.05, n_states=ns).cpu().numpy()
        np.testing.assert_array_equal(got2, ref)


def test_noalloc_rejects_more_than_the_limit(c2):
    import torch
    M, ctx, s, p = c2
    D = p.scene.dof
    a = torch.zeros((1, D), dtype=torch.float32, device=ctx.device)
    out = torch.zeros(1, dtype=torch.uint8, device=ctx.device)
    st = ctx._lib.mrpop_validate_edges_noalloc(ctx.handle, s.handle, a.data_ptr(), a.data_ptr(), MAX_EDGES + 1,
                                               C.c_float(0.05), None, out.data_ptr(), None, ctx.stream())
    assert M.STATUS_NAMES[st] == "E_INVALID_ARG"
    assert b"MRPOP_NOALLOC_MAX_EDGES" in ctx._lib.mrpop_last_error(ctx.handle)
    # an empty batch is a no-op
    assert s.validate_edges_noalloc(np.zeros((0, D), np.float32), np.zeros((0, D), np.float32), 0.05).numel() == 0
