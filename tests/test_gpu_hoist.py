"""GPU parity of hoisted alignment rotations (FHE_PLAN_HOIST): bit-exact against the oracle's hoisted
plan (per-pair and digit-tree modes), at one and two rotation digits, and in a recorded graph.

Each test prints the case it runs (flushed) before touching the GPU.
"""
import sys

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu

PRM = [(12, 5, 2, 2, 2), (13, 4, 1, 1, 1)]
_CACHE = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(prm):
    if prm not in _CACHE:
        from paper_2604_11659_amd import fhe
        log_n, n_q, n_p, alpha, D = prm
        _say(f"[hoist setup] {prm}")
        op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
        ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
        _CACHE[prm] = (op, ckks.Keys(op, 42), ctx, ctx.keygen(42))
    return _CACHE[prm]


def _case(prm, m, k, n, sa, sb, seeds):
    op, okeys, ctx, sk = _setup(prm)
    a = synth.sparse_dense(m, k, sa, "uniform", seeds[0], seeds[2])
    b = synth.sparse_dense(k, n, sb, "uniform", seeds[1], seeds[3])
    A = ctx.encrypt_csr(sk, m, k, *synth.to_csr(a), seed=43)
    B = ctx.encrypt_csc(sk, k, n, *synth.to_csc(b), seed=44)
    if op.rot_digits == 1:
        ctx.keygen_rotations(sk, ctx.plan_rotations(A, B))
    OA = spmspm.encrypt_csr(op, okeys, m, k, *synth.to_csr(a), seed=43)
    OB = spmspm.encrypt_csc(op, okeys, k, n, *synth.to_csc(b), seed=44)
    return op, okeys, ctx, sk, a, b, A, B, OA, OB


def _same(ctx, C, ref):
    return all((ctx.export(C, c) == r.data).all() for c, r in enumerate(ref))


@pytest.mark.parametrize("prm", PRM)
def test_hoisted_alignment_parity(prm):
    op, okeys, ctx, sk, a, b, A, B, OA, OB = _case(prm, 6, 7, 5, 0.3, 0.4, (0, 1, 2, 3))
    assert ctx.plan_stats(A, B).align_keyswitches > 0
    _say(f"[hoist] {prm} per-pair gpu")
    C = ctx.spmspm(A, B, hoist=True)
    _say(f"[hoist] {prm} per-pair oracle")
    ref = spmspm.spmspm(op, okeys, OA, OB, hoist=True, workers=4)
    assert _same(ctx, C, ref)
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    # the hoisted limbs differ from the plain plan's (the mode does change the key-switch inputs)
    plain = ctx.spmspm(A, B)
    assert not all((ctx.export(C, c) == ctx.export(plain, c)).all() for c in range(len(ref)))
    _say(f"[hoist] {prm} tree gpu")
    Ct = ctx.spmspm(A, B, tree=True, hoist=True)
    _say(f"[hoist] {prm} tree oracle")
    assert _same(ctx, Ct, spmspm.spmspm(op, okeys, OA, OB, tree=True, hoist=True, workers=4))


def test_hoisted_graph_and_batch():
    prm = PRM[0]
    op, okeys, ctx, sk, a, b, A, B, OA, OB = _case(prm, 5, 6, 4, 0.3, 0.3, (20, 21, 22, 23))
    _say("[hoist] eager")
    ref = [ctx.export(C, 0) for C in [ctx.spmspm(A, B, hoist=True)]][0]
    for rep in range(3):
        _say(f"[hoist] graph call {rep}")
        C = ctx.spmspm(A, B, hoist=True, graph=True)
        assert (ctx.export(C, 0) == ref).all(), rep
    _say("[hoist] oracle")
    oref = spmspm.spmspm(op, okeys, OA, OB, hoist=True, workers=4)
    assert (ref == oref[0].data).all()
