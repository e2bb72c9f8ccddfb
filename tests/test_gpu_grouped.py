"""GPU parity of the grouped plan (FHE_PLAN_GROUPED): bit-exact against the oracle's grouped form.

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


@pytest.fixture(scope="module")
def fhe():
    from paper_2604_11659_amd import fhe as f
    return f


def _setup(fhe, prm):
    if prm not in _CACHE:
        log_n, n_q, n_p, alpha, D = prm
        _say(f"[grouped setup] {prm}")
        op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
        ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
        _CACHE[prm] = (op, ckks.Keys(op, 42), ctx, ctx.keygen(42))
    return _CACHE[prm]


def _operands(fhe, prm, a, b, seeds=(43, 44)):
    op, okeys, ctx, sk = _setup(fhe, prm)
    (m, k), n = a.shape, b.shape[1]
    ipa, ixa, va = synth.to_csr(a)
    ipb, ixb, vb = synth.to_csc(b)
    A = ctx.encrypt_csr(sk, m, k, ipa, ixa, va, seed=seeds[0])
    B = ctx.encrypt_csc(sk, k, n, ipb, ixb, vb, seed=seeds[1])
    if op.rot_digits == 1:
        ctx.keygen_rotations(sk, ctx.plan_rotations(A, B))
    OA = spmspm.encrypt_csr(op, okeys, m, k, ipa, ixa, va, seed=seeds[0])
    OB = spmspm.encrypt_csc(op, okeys, k, n, ipb, ixb, vb, seed=seeds[1])
    return op, okeys, ctx, sk, A, B, OA, OB


def _same(ctx, C, ref):
    return all((ctx.export(C, c) == r.data).all() for c, r in enumerate(ref))


@pytest.mark.parametrize("prm", PRM)
def test_grouped_parity_small(fhe, prm):
    a = synth.sparse_dense(6, 7, 0.4, "uniform", 0, 2)
    b = synth.sparse_dense(7, 5, 0.4, "uniform", 1, 3)
    op, okeys, ctx, sk, A, B, OA, OB = _operands(fhe, prm, a, b)
    groups, gks, _ = ctx.plan_groups(A, B)
    st = ctx.plan_stats(A, B)
    _say(f"[grouped] {prm} 6x7x5: {st.matched_pairs} pairs, {groups} groups, gpu")
    C = ctx.spmspm(A, B, grouped=True)
    _say(f"[grouped] {prm} oracle")
    pairs = spmspm.matched_pairs(6, 5, OA.indptr, OA.indices, OB.indptr, OB.indices)
    assert groups == len(spmspm.target_groups(op, pairs, 5)) < st.matched_pairs
    assert gks == sum(len(ckks.rotation_steps(op, r)) for (_, r), _ in spmspm.target_groups(op, pairs, 5))
    ref = spmspm.spmspm(op, okeys, OA, OB, grouped=True, workers=4)
    assert _same(ctx, C, ref)
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    # the per-pair form on the same handles is still the per-pair oracle's
    C1 = ctx.spmspm(A, B)
    assert _same(ctx, C1, spmspm.spmspm(op, okeys, OA, OB, workers=4))


def test_grouped_two_result_chunks_and_passes(fhe, monkeypatch):
    """64 x 40 result over two S-slot chunks; then the same with a group budget of 1 MiB (four
    resident products per pass, so the groups run in many passes, each recomputing the products it
    uses): identical limbs."""
    prm = PRM[0]
    a = synth.sparse_dense(64, 2, 0.85, "uniform", 10, 12)
    b = synth.sparse_dense(2, 40, 0.5, "uniform", 11, 13)
    op, okeys, ctx, sk, A, B, OA, OB = _operands(fhe, prm, a, b, seeds=(53, 54))
    st = ctx.plan_stats(A, B)
    assert st.result_chunks == 2
    _say(f"[grouped] two chunks: {st.matched_pairs} pairs, {ctx.plan_groups(A, B)[0]} groups, gpu")
    C = ctx.spmspm(A, B, grouped=True)
    _say("[grouped] two chunks oracle")
    ref = spmspm.spmspm(op, okeys, OA, OB, grouped=True, workers=8)
    assert _same(ctx, C, ref)
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    monkeypatch.setenv("FHE_GROUP_MB", "1")
    _say("[grouped] two chunks, 1 MiB group budget")
    C2 = ctx.spmspm(A, B, grouped=True)
    monkeypatch.delenv("FHE_GROUP_MB")
    assert _same(ctx, C2, ref)


def test_grouped_pair_ranges_and_batch(fhe):
    """Groups formed over a traversal range (fhe_spmspm_pairs form) and inside a merged batch."""
    prm = PRM[0]
    op, okeys, ctx, sk = _setup(fhe, prm)
    shapes = [(5, 6, 4, 0.3, 0.4), (4, 7, 5, 0.5, 0.2)]
    ops_ = []
    for t, (m, k, n, sa, sb) in enumerate(shapes):
        a = synth.sparse_dense(m, k, sa, "uniform", 150 + t, 250 + t)
        b = synth.sparse_dense(k, n, sb, "uniform", 350 + t, 450 + t)
        ops_.append((a, b) + _operands(fhe, prm, a, b, seeds=(73 + 10 * t, 74 + 10 * t)))
    F = [ctx.plan_stats(o[6], o[7]).matched_pairs for o in ops_]
    ranges = [(F[0] // 3, F[0]), (0, 0)]
    _say(f"[grouped] batch with ranges {ranges}")
    Cb = ctx.spmspm_batch([o[6] for o in ops_], [o[7] for o in ops_], pair_ranges=ranges, grouped=True)
    a, b, op, okeys, _, _, A, B, OA, OB = ops_[0]
    pairs = spmspm.matched_pairs(a.shape[0], b.shape[1], OA.indptr, OA.indices, OB.indptr, OB.indices)
    ref = spmspm.spmspm(op, okeys, OA, OB, grouped=True, pairs=pairs[ranges[0][0]:ranges[0][1]], workers=4)
    assert _same(ctx, Cb[0], ref)
    Cs = ctx.spmspm_pairs(A, B, *ranges[0], grouped=True)
    assert _same(ctx, Cs, ref)
    assert (ctx.export(Cb[1], 0) == 0).all()
    Cfull = ctx.spmspm_batch([o[6] for o in ops_], [o[7] for o in ops_], grouped=True)
    for t, o in enumerate(ops_):
        Ci = ctx.spmspm(o[6], o[7], grouped=True)
        assert all((ctx.export(Cfull[t], c) == ctx.export(Ci, c)).all() for c in range(Ci.info()["chunks"]))
        assert np.abs(ctx.decrypt_decode(o[5], Ci) - o[0] @ o[1]).max() < 1e-5
    with pytest.raises(fhe.FheError):
        ctx.spmspm_batch([A], [B], pair_ranges=[(3, 1)], grouped=True)


def test_grouped_full_sparsity_is_zero(fhe):
    op, _, ctx, sk = _setup(fhe, PRM[0])
    z = np.zeros((4, 4))
    ip, ix, v = synth.to_csr(z)
    C = ctx.spmspm(ctx.encrypt_csr(sk, 4, 4, ip, ix, v, seed=43), ctx.encrypt_csc(sk, 4, 4, ip, ix, v, seed=44),
                   grouped=True)
    assert (ctx.export(C, 0) == 0).all()


@pytest.mark.parametrize("prm", PRM)
def test_tree_parity_small(fhe, prm):
    """Grouped plan with its target rotations shared digit by digit (FHE_PLAN_TREE) against the
    oracle's tree mode; with one rotation digit it equals the grouped plan."""
    a = synth.sparse_dense(6, 7, 0.4, "uniform", 0, 2)
    b = synth.sparse_dense(7, 5, 0.4, "uniform", 1, 3)
    op, okeys, ctx, sk, A, B, OA, OB = _operands(fhe, prm, a, b)
    groups, gks, tks = ctx.plan_groups(A, B)
    _say(f"[tree] {prm}: {groups} groups, {gks} -> {tks} target key switches, gpu")
    C = ctx.spmspm(A, B, tree=True)
    _say(f"[tree] {prm} oracle")
    ref = spmspm.spmspm(op, okeys, OA, OB, tree=True, workers=4)
    assert _same(ctx, C, ref)
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    if op.rot_digits == 1:
        assert tks == gks
        assert _same(ctx, C, spmspm.spmspm(op, okeys, OA, OB, grouped=True, workers=4))
    else:
        assert tks < gks


def test_tree_two_result_chunks_passes_and_graph(fhe, monkeypatch):
    prm = PRM[0]
    a = synth.sparse_dense(64, 2, 0.85, "uniform", 10, 12)
    b = synth.sparse_dense(2, 40, 0.5, "uniform", 11, 13)
    op, okeys, ctx, sk, A, B, OA, OB = _operands(fhe, prm, a, b, seeds=(53, 54))
    _say(f"[tree] two chunks: {ctx.plan_groups(A, B)}, gpu")
    C = ctx.spmspm(A, B, tree=True)
    _say("[tree] two chunks oracle")
    ref = spmspm.spmspm(op, okeys, OA, OB, tree=True, workers=8)
    assert _same(ctx, C, ref)
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    monkeypatch.setenv("FHE_GROUP_MB", "1")
    _say("[tree] two chunks, 1 MiB group budget")
    assert _same(ctx, ctx.spmspm(A, B, tree=True), ref)
    monkeypatch.delenv("FHE_GROUP_MB")
    for rep in range(3):
        _say(f"[tree] graph call {rep}")
        assert _same(ctx, ctx.spmspm(A, B, tree=True, graph=True), ref)


def test_tree_store_kept_between_calls(fhe):
    """Direct grouped calls keep their resident product store on the context: a smaller digit-tree
    call after a larger one reuses it (not shrunk, contents left over), and the larger call again
    grows nothing; every result bit-exact against the oracle's tree mode on the same pair range."""
    prm = PRM[0]
    a = synth.sparse_dense(12, 9, 0.5, "uniform", 20, 22)
    b = synth.sparse_dense(9, 10, 0.5, "uniform", 21, 23)
    op, okeys, ctx, sk, A, B, OA, OB = _operands(fhe, prm, a, b, seeds=(63, 64))
    pairs = spmspm.matched_pairs(a.shape[0], b.shape[1], OA.indptr, OA.indices, OB.indptr, OB.indices)
    F = len(pairs)
    assert F >= 8
    _say(f"[tree store] {F} pairs, oracle")
    refs = {F: spmspm.spmspm(op, okeys, OA, OB, tree=True, workers=8),
            F // 4: spmspm.spmspm(op, okeys, OA, OB, tree=True, pairs=pairs[:F // 4], workers=4)}
    for hi in (F, F // 4, F):
        _say(f"[tree store] pairs [0, {hi}) gpu")
        assert _same(ctx, ctx.spmspm_pairs(A, B, 0, hi, tree=True), refs[hi])
