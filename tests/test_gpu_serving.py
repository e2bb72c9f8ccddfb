"""Request loop with continuous batching: results are bit-identical alone and in the mix."""
import sys
import time

import numpy as np
import pytest

from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    from paper_2604_11659_amd import fhe
    ctx = fhe.Context(12, 5, 2, 2, 2)
    sk = ctx.keygen(42)
    reqs = []
    for t, (m, k, n, sa, sb) in enumerate([(6, 8, 5, 0.5, 0.5), (3, 3, 3, 0.2, 0.2), (8, 5, 8, 0.7, 0.4),
                                           (2, 9, 4, 0.0, 0.5), (7, 7, 7, 0.6, 0.6), (5, 4, 6, 0.3, 0.8)]):
        a = synth.sparse_dense(m, k, sa, "uniform", 500 + t, 600 + t)
        b = synth.sparse_dense(k, n, sb, "halfnormal", 700 + t, 800 + t)
        A = ctx.encrypt_csr(sk, m, k, *synth.to_csr(a), seed=1000 + t)
        B = ctx.encrypt_csc(sk, k, n, *synth.to_csc(b), seed=2000 + t)
        reqs.append((a, b, A, B))
    alone = []
    for (a, b, A, B) in reqs:
        C = ctx.spmspm(A, B)
        alone.append([ctx.export(C, c) for c in range(C.info()["chunks"])])
    return fhe, ctx, sk, reqs, alone


def _same(ctx, C, ref):
    return all((ctx.export(C, c) == r).all() for c, r in enumerate(ref))


def test_mixed_arrivals_bit_identical(env):
    fhe, ctx, sk, reqs, alone = env
    srv = fhe.Server(ctx, hbm_budget=1 << 34, max_inflight=4, slice_products=3)
    _say("[serve] staggered submissions")
    tickets = []
    for i, (a, b, A, B) in enumerate(reqs):
        tickets.append(srv.submit(A, B))
        time.sleep(0.002 * i)  # later requests arrive while earlier ones run
    for i, t in enumerate(tickets):
        res = srv.poll(t, wait_ms=60000)
        assert res is not None
        C, lat = res
        assert lat > 0
        assert _same(ctx, C, alone[i]), i
        a, b = reqs[i][0], reqs[i][1]
        assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["inflight"] == 0 and st["queued"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"]
    srv.close()


def test_budget_admission_and_rejection(env):
    fhe, ctx, sk, reqs, alone = env
    one = 2 * (5 - 2) * (1 << 12) * 8  # one result chunk at two levels below the top
    srv = fhe.Server(ctx, hbm_budget=one, max_inflight=8, slice_products=2)
    _say("[serve] budget of one result")
    tickets = [srv.submit(A, B) for (_, _, A, B) in reqs[:3]]
    for i, t in enumerate(tickets):
        C, _ = srv.poll(t, wait_ms=60000)
        assert _same(ctx, C, alone[i])
    srv.close()
    srv = fhe.Server(ctx, hbm_budget=one - 1, max_inflight=2, slice_products=2)
    t = srv.submit(reqs[0][2], reqs[0][3])
    with pytest.raises(fhe.FheError) as ei:
        srv.poll(t, wait_ms=60000)
    assert ei.value.code == -5
    srv.close()


def test_mixed_arrivals_tree_hoisted_bit_identical(env):
    """The request loop in the digit-tree plan with hoisted alignment rotations: every request runs
    whole in a step shared with the others, and its result equals the standalone call in that mode."""
    fhe, ctx, sk, reqs, alone = env
    srv = fhe.Server(ctx, hbm_budget=1 << 34, max_inflight=4, tree=True, hoist=True)
    _say("[serve] tree + hoisted, staggered submissions")
    tickets = []
    for i, (a, b, A, B) in enumerate(reqs):
        tickets.append(srv.submit(A, B))
        time.sleep(0.002 * i)
    with pytest.raises(fhe.FheError):  # the plan is fixed once requests have been submitted
        _lib_set = fhe._lib.fhe_server_set_plan
        fhe._check(_lib_set(srv._ptr, 0))
    for i, t in enumerate(tickets):
        res = srv.poll(t, wait_ms=60000)
        assert res is not None
        C, _ = res
        A, B = reqs[i][2], reqs[i][3]
        ref = ctx.spmspm(A, B, tree=True, hoist=True)
        assert all((ctx.export(C, c) == ctx.export(ref, c)).all() for c in range(C.info()["chunks"])), i
        assert np.abs(ctx.decrypt_decode(sk, C) - reqs[i][0] @ reqs[i][1]).max() < 1e-5
    srv.close()
