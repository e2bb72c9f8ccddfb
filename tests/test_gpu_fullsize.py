"""GPU parity at the benchmark workloads' full sizes.

* 16x16 x 16x16 (75% zeros each), N = 2^13: every result limb bit-exact against the oracle.
* DNN layer 128x128 (90% zeros) x 128x64 (50% zeros), N = 2^15: the full product decrypts to the FP64
  matmul within 1e-5 (max-abs); sampled pair ranges (start, middle, end of Algorithm 1's traversal)
  run through the same executor and are bit-exact against the oracle on the same pairs.
The oracle runs in 8 forked CPU workers (they never touch the GPU).
"""
import sys

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu
WORKERS = 8


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _prepare(w):
    from paper_2604_11659_amd import fhe
    a, b = w.operands()
    ipa, ixa, va = synth.to_csr(a)
    ipb, ixb, vb = synth.to_csc(b)
    ctx = fhe.Context(w.log_n, w.n_q, w.n_p, w.alpha, w.rot_digits)
    sk = ctx.keygen(42)
    A = ctx.encrypt_csr(sk, w.m, w.k, ipa, ixa, va, seed=43)
    B = ctx.encrypt_csc(sk, w.k, w.n, ipb, ixb, vb, seed=44)
    if w.rot_digits == 1:
        ctx.keygen_rotations(sk, ctx.plan_rotations(A, B))
    op = ckks.Params(log_n=w.log_n, n_q=w.n_q, n_p=w.n_p, alpha=w.alpha, rot_digits=w.rot_digits)
    keys = ckks.Keys(op, 42)
    OA = spmspm.encrypt_csr(op, keys, w.m, w.k, ipa, ixa, va, seed=43)
    OB = spmspm.encrypt_csc(op, keys, w.k, w.n, ipb, ixb, vb, seed=44)
    return a, b, ctx, sk, A, B, op, keys, OA, OB


@pytest.mark.timeout(900)
def test_plain_16x16_full_bit_exact():
    w = synth.WORKLOADS["plain"]
    _say("[full] plain 16x16 N=2^13 setup")
    a, b, ctx, sk, A, B, op, keys, OA, OB = _prepare(w)
    st = ctx.plan_stats(A, B)
    _say(f"[full] plain gpu spmspm, {st}")
    C = ctx.spmspm(A, B)
    _say("[full] plain oracle")
    ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS)
    assert len(ref) == st.result_chunks == 1
    assert (ctx.export(C, 0) == ref[0].data).all()
    err = np.abs(ctx.decrypt_decode(sk, C) - a @ b).max()
    assert err < 1e-5
    _say(f"[full] plain ok, max-abs error {err:.3e}")
    ctx.close()


@pytest.mark.timeout(1200)
def test_dnn_layer_full_fp64_and_sampled_bit_exact():
    w = synth.WORKLOADS["dnn"]
    _say("[full] dnn setup")
    a, b, ctx, sk, A, B, op, keys, OA, OB = _prepare(w)
    st = ctx.plan_stats(A, B)
    _say(f"[full] dnn gpu spmspm, {st}")
    C = ctx.spmspm(A, B)
    err = np.abs(ctx.decrypt_decode(sk, C) - a @ b).max()
    _say(f"[full] dnn max-abs error {err:.3e}")
    assert err < 1e-5
    F = st.matched_pairs
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    assert len(pairs) == F
    for lo, hi in [(0, 3), (F // 2, F // 2 + 3), (F - 3, F)]:
        _say(f"[full] dnn pairs [{lo}, {hi}) gpu")
        Cs = ctx.spmspm_pairs(A, B, lo, hi)
        _say(f"[full] dnn pairs [{lo}, {hi}) oracle")
        ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS, pairs=pairs[lo:hi])
        assert (ctx.export(Cs, 0) == ref[0].data).all(), (lo, hi)
    ctx.close()


def _merged_window(op, pairs, n, width):
    """The traversal window of `width` pairs whose grouped plan merges the most pairs (host only)."""
    best = (0, 0)
    for lo in range(0, max(1, len(pairs) - width), 997):
        merged = width - len(spmspm.target_groups(op, pairs[lo:lo + width], n))
        best = max(best, (merged, lo))
    return best[1], best[1] + width


@pytest.mark.timeout(1200)
def test_dnn_layer_grouped_full_fp64_and_sampled_bit_exact():
    """Grouped plan at the DNN layer's full size: decrypts within 1e-5 of FP64; a traversal window
    in which several pairs share groups is bit-exact against the oracle's grouped form."""
    w = synth.WORKLOADS["dnn"]
    _say("[full] dnn grouped setup")
    a, b, ctx, sk, A, B, op, keys, OA, OB = _prepare(w)
    groups, gks, _ = ctx.plan_groups(A, B)
    _say(f"[full] dnn grouped gpu spmspm: {groups} groups, {gks} target key switches")
    C = ctx.spmspm(A, B, grouped=True)
    err = np.abs(ctx.decrypt_decode(sk, C) - a @ b).max()
    _say(f"[full] dnn grouped max-abs error {err:.3e}")
    assert err < 1e-5
    C.close()
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    assert groups == len(spmspm.target_groups(op, pairs, w.n))
    lo, hi = _merged_window(op, pairs, w.n, 24)
    ng = len(spmspm.target_groups(op, pairs[lo:hi], w.n))
    assert ng < hi - lo
    _say(f"[full] dnn grouped pairs [{lo}, {hi}) ({ng} groups) gpu")
    Cs = ctx.spmspm_pairs(A, B, lo, hi, grouped=True)
    _say(f"[full] dnn grouped pairs [{lo}, {hi}) oracle")
    ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS, pairs=pairs[lo:hi], grouped=True)
    assert (ctx.export(Cs, 0) == ref[0].data).all(), (lo, hi)
    ctx.close()


@pytest.mark.timeout(1200)
def test_dnn_layer_tree_full_fp64_and_sampled_bit_exact():
    """Digit-tree plan at the DNN layer's full size: decrypts within 1e-5 of FP64; a traversal window
    whose groups merge is bit-exact against the oracle's tree mode."""
    w = synth.WORKLOADS["dnn"]
    _say("[full] dnn tree setup")
    a, b, ctx, sk, A, B, op, keys, OA, OB = _prepare(w)
    groups, gks, tks = ctx.plan_groups(A, B)
    _say(f"[full] dnn tree gpu spmspm: {groups} groups, {gks} -> {tks} target key switches")
    C = ctx.spmspm(A, B, tree=True)
    err = np.abs(ctx.decrypt_decode(sk, C) - a @ b).max()
    _say(f"[full] dnn tree max-abs error {err:.3e}")
    assert err < 1e-5
    C.close()
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    lo, hi = _merged_window(op, pairs, w.n, 24)
    _say(f"[full] dnn tree pairs [{lo}, {hi}) gpu")
    Cs = ctx.spmspm_pairs(A, B, lo, hi, tree=True)
    _say(f"[full] dnn tree pairs [{lo}, {hi}) oracle")
    ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS, pairs=pairs[lo:hi], tree=True)
    assert (ctx.export(Cs, 0) == ref[0].data).all(), (lo, hi)


# ---- the larger parameter sets (N = 2^16 with 24 Q + 3 P primes, N = 2^17 with 35 Q + 3 P) ----
    ctx.close()


def _ctx_pair(prm):
    from paper_2604_11659_amd import fhe
    log_n, n_q, n_p, alpha, D = prm
    ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
    sk = ctx.keygen(42)
    op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
    return ctx, sk, op, ckks.Keys(op, 42)


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prm,a,b", [
    # alignment rotations of A and B, a target rotation by S - 1 (three digit steps), shared products
    ((16, 24, 3, 3, 3), np.array([[0.5, -0.25, 0.75]]), np.array([[0.0, 0.3], [0.0, -0.6], [0.9, 0.0]])),
    # one product, one target rotation by 1: every key-switch kernel at alpha = K = 3, N = 2^17
    ((17, 35, 3, 3, 4), np.array([[0.5, -0.25]]), np.array([[0.75], [0.3]])),
])
def test_large_parameter_sets_bit_exact(prm, a, b):
    """The parameter sets of the large, batching and serving workloads (three primes per digit,
    three special primes, NTT splits 2^7 x 2^9 and 2^8 x 2^9): a small matmul bit-exact against the
    oracle in every limb."""
    _say(f"[large] {prm} setup")
    ctx, sk, op, keys = _ctx_pair(prm)
    (m, k), n = a.shape, b.shape[1]
    A = ctx.encrypt_csr(sk, m, k, *synth.to_csr(a), seed=43)
    B = ctx.encrypt_csc(sk, k, n, *synth.to_csc(b), seed=44)
    _say(f"[large] {prm} gpu {ctx.plan_stats(A, B)}")
    C = ctx.spmspm(A, B)
    _say(f"[large] {prm} oracle")
    ref = spmspm.spmspm(op, keys, spmspm.encrypt_csr(op, keys, m, k, *synth.to_csr(a), seed=43),
                        spmspm.encrypt_csc(op, keys, k, n, *synth.to_csc(b), seed=44), workers=WORKERS)
    assert (ctx.export(C, 0) == ref[0].data).all()
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    C.close()
    ctx.close()


@pytest.mark.timeout(1200)
def test_large_workload_sampled_pairs_bit_exact():
    """The 512 x 512 workload at N = 2^16 (B over four operand chunks, C over eight result chunks):
    pair ranges at the start, middle and end of Algorithm 1's traversal are bit-exact against the
    oracle on the same pairs."""
    w = synth.WORKLOADS["large"]
    _say("[full] large setup")
    a, b, ctx, sk, A, B, op, keys, OA, OB = _prepare(w)
    st = ctx.plan_stats(A, B)
    assert st.result_chunks == 8 and B.info()["chunks"] == 4
    F = st.matched_pairs
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    assert len(pairs) == F
    for lo, hi in [(0, 2), (F // 2, F // 2 + 2), (F - 2, F)]:
        _say(f"[full] large pairs [{lo}, {hi}) gpu")
        Cs = ctx.spmspm_pairs(A, B, lo, hi)
        _say(f"[full] large pairs [{lo}, {hi}) oracle")
        ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS, pairs=pairs[lo:hi])
        for c, r in enumerate(ref):
            assert (ctx.export(Cs, c) == r.data).all(), (lo, hi, c)
        Cs.close()
    ctx.close()


@pytest.mark.timeout(1200)
def test_dnn_layer_hoisted_window_bit_exact():
    """Hoisted alignment rotations at the DNN layer's size: a traversal window (its products rotate
    operand chunks by several amounts) bit-exact against the oracle's hoisted plan, per pair and with
    the digit tree; the full layer decrypts within 1e-5 with both."""
    w = synth.WORKLOADS["dnn"]
    _say("[full] dnn hoisted setup")
    a, b, ctx, sk, A, B, op, keys, OA, OB = _prepare(w)
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    lo, hi = _merged_window(op, pairs, w.n, 24)
    for tree in (False, True):
        _say(f"[full] dnn hoisted tree={tree} pairs [{lo}, {hi}) gpu")
        Cs = ctx.spmspm_pairs(A, B, lo, hi, tree=tree, hoist=True)
        _say(f"[full] dnn hoisted tree={tree} oracle")
        ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS, pairs=pairs[lo:hi], tree=tree, hoist=True)
        assert (ctx.export(Cs, 0) == ref[0].data).all(), (tree, lo, hi)
        Cs.close()
        _say(f"[full] dnn hoisted tree={tree} full layer")
        C = ctx.spmspm(A, B, tree=tree, hoist=True)
        err = np.abs(ctx.decrypt_decode(sk, C) - a @ b).max()
        _say(f"[full] dnn hoisted tree={tree} max-abs error {err:.3e}")
        assert err < 1e-5
        C.close()
    ctx.close()
