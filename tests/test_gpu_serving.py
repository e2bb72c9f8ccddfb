"""Request loop with continuous batching over two parameter sets sharing one HBM budget.

Every served result is compared limb by limb with the oracle's Algorithm 1 + 2 on the same seeded
keys, noise and operands (the per-pair plan, and the digit-tree plan with hoisted alignment rotations
against the oracle's tree + hoisted form). The budget tests check that a budget for one request at a
time admits one request at a time, that a request that can never fit is refused at submission, and
that closing the server cancels the requests still queued (their pollers get FHE_ECANCELED).
"""
import sys
import threading
import time

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu
WORKERS = 8

# (log_n, n_q, n_p, alpha, rotation digits): two parameter sets served by one server
PARAMS = [(12, 5, 2, 2, 2), (13, 4, 1, 1, 2)]
SHAPES = [(6, 8, 5, 0.5, 0.5), (3, 3, 3, 0.2, 0.2), (8, 5, 8, 0.7, 0.4), (2, 9, 4, 0.0, 0.5), (7, 7, 7, 0.6, 0.6),
          (5, 4, 6, 0.3, 0.8)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    from paper_2604_11659_amd import fhe
    ctxs, sks, ops, okeys = [], [], [], []
    for prm in PARAMS:
        log_n, n_q, n_p, alpha, D = prm
        _say(f"[serve] context {prm}")
        ctxs.append(fhe.Context(log_n, n_q, n_p, alpha, D))
        sks.append(ctxs[-1].keygen(42))
        ops.append(ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D))
        okeys.append(ckks.Keys(ops[-1], 42))
    reqs = []  # (ctx id, a, b, A, B, oracle A, oracle B)
    for t, (m, k, n, sa, sb) in enumerate(SHAPES):
        ci = t % 2
        a = synth.sparse_dense(m, k, sa, "uniform", 500 + t, 600 + t)
        b = synth.sparse_dense(k, n, sb, "halfnormal", 700 + t, 800 + t)
        ipa, ixa, va = synth.to_csr(a)
        ipb, ixb, vb = synth.to_csc(b)
        A = ctxs[ci].encrypt_csr(sks[ci], m, k, ipa, ixa, va, seed=1000 + t)
        B = ctxs[ci].encrypt_csc(sks[ci], k, n, ipb, ixb, vb, seed=2000 + t)
        OA = spmspm.encrypt_csr(ops[ci], okeys[ci], m, k, ipa, ixa, va, seed=1000 + t)
        OB = spmspm.encrypt_csc(ops[ci], okeys[ci], k, n, ipb, ixb, vb, seed=2000 + t)
        reqs.append((ci, a, b, A, B, OA, OB))
    oracle = {}

    def expected(i, tree=False):
        """Oracle result limbs of request i (per pair, or digit tree + hoisted), computed once."""
        if (i, tree) not in oracle:
            ci, _, _, _, _, OA, OB = reqs[i]
            _say(f"[serve] oracle request {i} tree={tree}")
            res = spmspm.spmspm(ops[ci], okeys[ci], OA, OB, workers=WORKERS, tree=tree, hoist=tree)
            oracle[(i, tree)] = [r.data for r in res]
        return oracle[(i, tree)]

    return fhe, ctxs, sks, reqs, expected


def _check(env, i, C, tree=False):
    fhe, ctxs, sks, reqs, expected = env
    ci, a, b = reqs[i][0], reqs[i][1], reqs[i][2]
    ref = expected(i, tree)
    assert C.info()["chunks"] == len(ref)
    for c, r in enumerate(ref):
        assert (ctxs[ci].export(C, c) == r).all(), (i, c)
    assert np.abs(ctxs[ci].decrypt_decode(sks[ci], C) - a @ b).max() < 1e-5


def test_mixed_arrivals_two_contexts_match_oracle(env):
    fhe, ctxs, sks, reqs, _ = env
    srv = fhe.Server(ctxs, hbm_budget=1 << 36, max_inflight=4, slice_products=3)
    _say("[serve] staggered submissions over two parameter sets")
    tickets = []
    for i, (ci, _, _, A, B, _, _) in enumerate(reqs):
        tickets.append(srv.submit(A, B, ctx_id=ci))
        if i >= 3:
            time.sleep(0.002 * i)  # later requests arrive while earlier ones run
    served = []
    for t in tickets:
        res = srv.poll(t, wait_ms=120000)
        assert res is not None
        assert res[1] > 0
        served.append(res[0])
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["inflight"] == 0 and st["queued"] == 0 and st["failed"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"]
    assert st["max_merged"] >= 2  # requests of one context shared a launch stream
    assert st["steps"] >= 2
    srv.close()
    for i, C in enumerate(served):
        _check(env, i, C)


def _charges(fhe, ctxs, reqs):
    """Result bytes of each request (its per-request charge in the per-pair plan)."""
    out = []
    for (ci, _, _, A, B, _, _) in reqs:
        c = ctxs[ci]
        out.append(c.plan_stats(A, B).result_chunks * 2 * (c.n_q - 2) * c.N * 8)
    return out


def test_budget_for_one_request_admits_one_at_a_time(env):
    fhe, ctxs, sks, reqs, _ = env
    ws = 64 << 20
    probe = fhe.Server(ctxs, hbm_budget=1 << 40, workspace_bytes=ws)
    fixed = probe.stats()["fixed_bytes"]
    probe.close()
    charges = _charges(fhe, ctxs, reqs)
    # room for the largest request alone: no two requests (of any context) fit together
    assert min(charges) * 2 > max(charges)
    budget = fixed + max(charges)
    srv = fhe.Server(ctxs, hbm_budget=budget, workspace_bytes=ws, max_inflight=8, slice_products=2)
    _say(f"[serve] budget {budget} = fixed {fixed} + one request")
    tickets = [srv.submit(A, B, ctx_id=ci) for (ci, _, _, A, B, _, _) in reqs]
    st0 = srv.stats()
    assert st0["fixed_bytes"] == fixed and st0["inflight_bytes"] <= max(charges)
    served = [srv.poll(t, wait_ms=120000)[0] for t in tickets]
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["max_step_requests"] == 1
    srv.close()
    for i, C in enumerate(served):
        _check(env, i, C)
    # a request whose own charge exceeds what the budget leaves is refused at submission
    srv = fhe.Server(ctxs, hbm_budget=fixed + min(charges) - 1, workspace_bytes=ws)
    with pytest.raises(fhe.FheError) as ei:
        srv.submit(reqs[0][3], reqs[0][4], ctx_id=reqs[0][0])
    assert ei.value.code == -5
    with pytest.raises(fhe.FheError) as ei:  # a context id the server does not have
        srv.submit(reqs[0][3], reqs[0][4], ctx_id=2)
    assert ei.value.code == -1
    srv.close()
    # a budget below the fixed part cannot start a server
    with pytest.raises(fhe.FheError) as ei:
        fhe.Server(ctxs, hbm_budget=fixed - 1, workspace_bytes=ws)
    assert ei.value.code == -5


def test_close_cancels_queued_requests(env):
    fhe, ctxs, sks, reqs, _ = env
    srv = fhe.Server(ctxs, hbm_budget=1 << 36, max_inflight=1, slice_products=1)
    _say("[serve] close with queued requests")
    tickets = [(i, srv.submit(A, B, ctx_id=ci)) for i, (ci, _, _, A, B, _, _) in enumerate(reqs)]
    outcome = {}

    def wait_last():
        try:
            outcome["res"] = srv.poll(tickets[-1][1], wait_ms=120000)
        except fhe.FheError as e:
            outcome["code"] = e.code

    th = threading.Thread(target=wait_last)
    th.start()
    time.sleep(0.05)
    st = srv.stats()
    srv.close()  # cancels what is still queued, wakes the waiting poller, waits for it to leave
    th.join(timeout=60)
    assert not th.is_alive()
    if st["queued"] >= 1:  # the last request was still waiting for admission when the server closed
        assert outcome.get("code") == -8, outcome
    else:
        assert "res" in outcome or outcome.get("code") == -8


def test_mixed_arrivals_tree_hoisted_match_oracle(env):
    """The request loop in the digit-tree plan with hoisted alignment rotations: every request runs
    whole in a step shared with the requests of its context, and its limbs equal the oracle's tree +
    hoisted form."""
    fhe, ctxs, sks, reqs, _ = env
    srv = fhe.Server(ctxs, hbm_budget=1 << 36, max_inflight=4, tree=True, hoist=True)
    _say("[serve] tree + hoisted, staggered submissions")
    tickets = []
    for i, (ci, _, _, A, B, _, _) in enumerate(reqs):
        tickets.append(srv.submit(A, B, ctx_id=ci))
        time.sleep(0.002 * i)
    with pytest.raises(fhe.FheError):  # the plan is fixed once requests have been submitted
        fhe._check(fhe._lib.fhe_server_set_plan(srv._ptr, 0))
    served = []
    for t in tickets:
        res = srv.poll(t, wait_ms=120000)
        assert res is not None
        served.append(res[0])
    srv.close()
    for i, C in enumerate(served):
        _check(env, i, C, tree=True)


def test_missing_rotation_key_fails_request(env):
    """FHE_EKEY: with one rotation digit (per-amount keys) and no keys generated, a matmul that needs
    a rotation fails, directly and through the server."""
    fhe = env[0]
    ctx = fhe.Context(12, 4, 1, 1, 1)
    sk = ctx.keygen(42)
    a = np.array([[0.5, -0.25]])
    b = np.array([[0.0], [0.75]])  # a_pos 1, b_pos 0: an alignment rotation by 1
    A = ctx.encrypt_csr(sk, 1, 2, *synth.to_csr(a), seed=1)
    B = ctx.encrypt_csc(sk, 2, 1, *synth.to_csc(b), seed=2)
    with pytest.raises(fhe.FheError) as ei:
        ctx.spmspm(A, B)
    assert ei.value.code == -4
    srv = fhe.Server(ctx, hbm_budget=1 << 34)
    t = srv.submit(A, B)
    with pytest.raises(fhe.FheError) as ei:
        srv.poll(t, wait_ms=60000)
    assert ei.value.code == -4
    assert srv.stats()["failed"] == 1
    srv.close()
    ctx.keygen_rotations(sk, ctx.plan_rotations(A, B))
    C = ctx.spmspm(A, B)
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    ctx.close()
