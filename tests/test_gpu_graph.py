"""HIP-graph form of the matmul (FHE_PLAN_GRAPH): the recorded launch stream, replayed several times
with eager work in between, gives the eager form's limbs every time (per-pair and grouped plans,
merged batches), and a different operand pair records a graph of its own.

Each test prints the case it runs (flushed) before touching the GPU.
"""
import sys

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu
PRM = (12, 5, 2, 2, 2)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    from paper_2604_11659_amd import fhe
    _say(f"[graph setup] {PRM}")
    ctx = fhe.Context(*PRM)
    sk = ctx.keygen(42)
    mats = []
    for t, (m, k, n, sa, sb) in enumerate([(6, 7, 5, 0.4, 0.4), (5, 4, 6, 0.3, 0.5), (4, 6, 3, 0.5, 0.2)]):
        a = synth.sparse_dense(m, k, sa, "uniform", 500 + t, 510 + t)
        b = synth.sparse_dense(k, n, sb, "uniform", 520 + t, 530 + t)
        A = ctx.encrypt_csr(sk, m, k, *synth.to_csr(a), seed=43 + t)
        B = ctx.encrypt_csc(sk, k, n, *synth.to_csc(b), seed=44 + t)
        mats.append((a, b, A, B))
    return fhe, ctx, sk, mats


def _limbs(ctx, C):
    return [ctx.export(C, c) for c in range(C.info()["chunks"])]


def _same(x, y):
    return len(x) == len(y) and all((u == v).all() for u, v in zip(x, y))


@pytest.mark.parametrize("grouped", [False, True])
def test_graph_replays_match_eager(env, grouped):
    fhe, ctx, sk, mats = env
    a, b, A, B = mats[0]
    _say(f"[graph] grouped={grouped} eager")
    ref = _limbs(ctx, ctx.spmspm(A, B, grouped=grouped))
    a2, b2, A2, B2 = mats[1]
    other = _limbs(ctx, ctx.spmspm(A2, B2, grouped=grouped))
    for rep in range(4):
        _say(f"[graph] grouped={grouped} graph call {rep}")
        C = ctx.spmspm(A, B, grouped=grouped, graph=True)
        assert _same(_limbs(ctx, C), ref), rep
        assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
        C.close()
        # eager work on the same context between replays
        assert _same(_limbs(ctx, ctx.spmspm(A2, B2, grouped=grouped)), other), rep


def test_graph_cache_switches_operands_and_batches(env):
    fhe, ctx, sk, mats = env
    As, Bs = [m[2] for m in mats], [m[3] for m in mats]
    _say("[graph] eager batch")
    ref = [_limbs(ctx, C) for C in ctx.spmspm_batch(As, Bs)]
    for rep in range(3):
        _say(f"[graph] batch graph call {rep}")
        got = [_limbs(ctx, C) for C in ctx.spmspm_batch(As, Bs, graph=True)]
        assert all(_same(x, y) for x, y in zip(got, ref)), rep
        # a single matmul in between records (or replays) a graph of its own
        _say(f"[graph] single graph call {rep}")
        assert _same(_limbs(ctx, ctx.spmspm(As[2], Bs[2], graph=True)), ref[2]), rep
    # against the oracle once
    op = ckks.Params(log_n=PRM[0], n_q=PRM[1], n_p=PRM[2], alpha=PRM[3], rot_digits=PRM[4])
    keys = ckks.Keys(op, 42)
    a, b = mats[2][0], mats[2][1]
    (m, k), n = a.shape, b.shape[1]
    _say("[graph] oracle")
    oref = spmspm.spmspm(op, keys, spmspm.encrypt_csr(op, keys, m, k, *synth.to_csr(a), seed=45),
                         spmspm.encrypt_csc(op, keys, k, n, *synth.to_csc(b), seed=46), workers=4)
    assert all((r == o.data).all() for r, o in zip(ref[2], oref))
