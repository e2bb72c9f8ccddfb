"""GPU parity at the benchmark workloads' full sizes and parameter sets.

* 16x16 x 16x16 (75% zeros each), N = 2^13: every result limb bit-exact against the oracle.
* DNN layer 128x128 (90% zeros) x 128x64 (50% zeros), N = 2^15: the full product decrypts to the FP64
  matmul within 1e-5 (max-abs, every plan mode); sampled pair ranges (start, middle, end of Algorithm
  1's traversal) and one wide range whose launches carry over 64 items that share rotation keys run
  through the same executor and are bit-exact against the oracle on the same pairs.
* N = 2^16 (24 Q + 3 P primes, three digits) and N = 2^17 (35 Q + 3 P, four digits): small matmuls
  bit-exact; the 512 x 512 workload bit-exact on pair ranges; and a merged batch of three uneven
  matmuls of the batching workload (seeded prefixes and a tail range) bit-exact in every chunk.
The oracle runs in up to 16 forked CPU workers (they never touch the GPU). Contexts, keys and encrypted
operands of one parameter set are built once per module and shared by its tests.
"""
import os
import sys

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu
# oracle worker processes: the CPUs this process may use, at most 16 (a GPU machine's CPU share)
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class _Env:
    """A GPU context and the oracle's keys for one parameter set, plus encrypted operands by name."""

    def __init__(self, prm):
        from paper_2604_11659_amd import fhe
        log_n, n_q, n_p, alpha, D = prm
        _say(f"[full] context {prm}")
        self.ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
        self.sk = self.ctx.keygen(42)
        self.op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
        self.keys = ckks.Keys(self.op, 42)
        self.mats = {}

    def operands(self, name, a, b, seeds=(43, 44)):
        """(A, B, oracle A, oracle B) of a (CSR) times b (CSC), encrypted once."""
        if name not in self.mats:
            (m, k), n = a.shape, b.shape[1]
            ipa, ixa, va = synth.to_csr(a)
            ipb, ixb, vb = synth.to_csc(b)
            A = self.ctx.encrypt_csr(self.sk, m, k, ipa, ixa, va, seed=seeds[0])
            B = self.ctx.encrypt_csc(self.sk, k, n, ipb, ixb, vb, seed=seeds[1])
            if self.op.rot_digits == 1:
                self.ctx.keygen_rotations(self.sk, self.ctx.plan_rotations(A, B))
            OA = spmspm.encrypt_csr(self.op, self.keys, m, k, ipa, ixa, va, seed=seeds[0])
            OB = spmspm.encrypt_csc(self.op, self.keys, k, n, ipb, ixb, vb, seed=seeds[1])
            self.mats[name] = (A, B, OA, OB)
        return self.mats[name]

    def oracle(self, OA, OB, pairs=None, **kw):
        return spmspm.spmspm(self.op, self.keys, OA, OB, workers=WORKERS, pairs=pairs, **kw)

    def check(self, C, ref, what):
        assert C.info()["chunks"] == len(ref), what
        for c, r in enumerate(ref):
            assert (self.ctx.export(C, c) == r.data).all(), (what, c)


def _params(w):
    return (w.log_n, w.n_q, w.n_p, w.alpha, w.rot_digits)


@pytest.fixture(scope="module")
def dnn():
    w = synth.WORKLOADS["dnn"]
    env = _Env(_params(w))
    a, b = w.operands()
    A, B, OA, OB = env.operands("dnn", a, b)
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    yield env, w, a, b, A, B, OA, OB, pairs
    env.ctx.close()


@pytest.fixture(scope="module")
def large():
    env = _Env(_params(synth.WORKLOADS["large"]))
    yield env
    env.ctx.close()


@pytest.mark.timeout(900)
def test_plain_16x16_full_bit_exact():
    w = synth.WORKLOADS["plain"]
    _say("[full] plain 16x16 N=2^13 setup")
    env = _Env(_params(w))
    a, b = w.operands()
    A, B, OA, OB = env.operands("plain", a, b)
    st = env.ctx.plan_stats(A, B)
    _say(f"[full] plain gpu spmspm, {st}")
    C = env.ctx.spmspm(A, B)
    _say("[full] plain oracle")
    ref = env.oracle(OA, OB)
    assert len(ref) == st.result_chunks == 1
    env.check(C, ref, "plain")
    err = np.abs(env.ctx.decrypt_decode(env.sk, C) - a @ b).max()
    assert err < 1e-5
    _say(f"[full] plain ok, max-abs error {err:.3e}")
    env.ctx.close()


@pytest.mark.timeout(1200)
def test_dnn_layer_full_fp64_and_sampled_bit_exact(dnn):
    env, w, a, b, A, B, OA, OB, pairs = dnn
    st = env.ctx.plan_stats(A, B)
    _say(f"[full] dnn gpu spmspm, {st}")
    C = env.ctx.spmspm(A, B)
    err = np.abs(env.ctx.decrypt_decode(env.sk, C) - a @ b).max()
    _say(f"[full] dnn max-abs error {err:.3e}")
    assert err < 1e-5
    C.close()
    F = st.matched_pairs
    assert len(pairs) == F
    for lo, hi in [(0, 3), (F // 2, F // 2 + 3), (F - 3, F)]:
        _say(f"[full] dnn pairs [{lo}, {hi}) gpu")
        Cs = env.ctx.spmspm_pairs(A, B, lo, hi)
        _say(f"[full] dnn pairs [{lo}, {hi}) oracle")
        env.check(Cs, env.oracle(OA, OB, pairs[lo:hi]), (lo, hi))
        Cs.close()


def _shared_key_window(op, pairs, n, width):
    """A traversal window of `width` pairs whose target rotations use few distinct digit keys (host
    only): the window where the most target-rotation key uses repeat a key already used."""
    best = (-1, 0)
    for lo in range(0, len(pairs) - width, 499):
        steps = []
        for (i, j, a_pos, b_pos) in pairs[lo:lo + width]:
            mn = spmspm.alignment(op, a_pos, b_pos)[4]
            steps += ckks.rotation_steps(op, spmspm.target(op, i, j, n, mn)[1])
        shared = len(steps) - len(set(steps))
        best = max(best, (shared, lo))
    return best[1], best[1] + width, best[0]


@pytest.mark.timeout(1200)
def test_dnn_layer_wide_range_shared_keys_bit_exact(dnn):
    """A traversal range of 96 pairs at the DNN layer's size: its tail launches carry all 96 items at
    once, sorted so that items using the same rotation key are neighbours (the key-stationary order
    of the timed runs). Bit-exact against the oracle on the same pairs."""
    env, w, a, b, A, B, OA, OB, pairs = dnn
    lo, hi, shared = _shared_key_window(env.op, pairs, w.n, 96)
    assert hi - lo >= 64 and shared >= 32, (lo, hi, shared)
    _say(f"[full] dnn wide range [{lo}, {hi}) ({shared} key uses shared) gpu")
    Cs = env.ctx.spmspm_pairs(A, B, lo, hi)
    _say(f"[full] dnn wide range [{lo}, {hi}) oracle")
    env.check(Cs, env.oracle(OA, OB, pairs[lo:hi]), (lo, hi))
    Cs.close()


def _merged_window(op, pairs, n, width):
    """The traversal window of `width` pairs whose grouped plan merges the most pairs (host only)."""
    best = (0, 0)
    for lo in range(0, max(1, len(pairs) - width), 997):
        merged = width - len(spmspm.target_groups(op, pairs[lo:lo + width], n))
        best = max(best, (merged, lo))
    return best[1], best[1] + width


@pytest.mark.timeout(1200)
def test_dnn_layer_grouped_full_fp64_and_sampled_bit_exact(dnn):
    """Grouped plan at the DNN layer's full size: decrypts within 1e-5 of FP64; a traversal window
    in which several pairs share groups is bit-exact against the oracle's grouped form."""
    env, w, a, b, A, B, OA, OB, pairs = dnn
    groups, gks, _ = env.ctx.plan_groups(A, B)
    _say(f"[full] dnn grouped gpu spmspm: {groups} groups, {gks} target key switches")
    C = env.ctx.spmspm(A, B, grouped=True)
    err = np.abs(env.ctx.decrypt_decode(env.sk, C) - a @ b).max()
    _say(f"[full] dnn grouped max-abs error {err:.3e}")
    assert err < 1e-5
    C.close()
    assert groups == len(spmspm.target_groups(env.op, pairs, w.n))
    lo, hi = _merged_window(env.op, pairs, w.n, 24)
    ng = len(spmspm.target_groups(env.op, pairs[lo:hi], w.n))
    assert ng < hi - lo
    _say(f"[full] dnn grouped pairs [{lo}, {hi}) ({ng} groups) gpu")
    Cs = env.ctx.spmspm_pairs(A, B, lo, hi, grouped=True)
    _say(f"[full] dnn grouped pairs [{lo}, {hi}) oracle")
    env.check(Cs, env.oracle(OA, OB, pairs[lo:hi], grouped=True), (lo, hi))
    Cs.close()


@pytest.mark.timeout(1200)
def test_dnn_layer_tree_full_fp64_and_sampled_bit_exact(dnn):
    """Digit-tree plan at the DNN layer's full size: decrypts within 1e-5 of FP64; a traversal window
    whose groups merge is bit-exact against the oracle's tree mode."""
    env, w, a, b, A, B, OA, OB, pairs = dnn
    groups, gks, tks = env.ctx.plan_groups(A, B)
    _say(f"[full] dnn tree gpu spmspm: {groups} groups, {gks} -> {tks} target key switches")
    C = env.ctx.spmspm(A, B, tree=True)
    err = np.abs(env.ctx.decrypt_decode(env.sk, C) - a @ b).max()
    _say(f"[full] dnn tree max-abs error {err:.3e}")
    assert err < 1e-5
    C.close()
    lo, hi = _merged_window(env.op, pairs, w.n, 24)
    _say(f"[full] dnn tree pairs [{lo}, {hi}) gpu")
    Cs = env.ctx.spmspm_pairs(A, B, lo, hi, tree=True)
    _say(f"[full] dnn tree pairs [{lo}, {hi}) oracle")
    env.check(Cs, env.oracle(OA, OB, pairs[lo:hi], tree=True), (lo, hi))
    Cs.close()


@pytest.mark.timeout(1200)
def test_dnn_layer_hoisted_window_bit_exact(dnn):
    """Hoisted alignment rotations at the DNN layer's size: a traversal window (its products rotate
    operand chunks by several amounts) bit-exact against the oracle's hoisted plan, per pair and with
    the digit tree; the full layer decrypts within 1e-5 with both."""
    env, w, a, b, A, B, OA, OB, pairs = dnn
    lo, hi = _merged_window(env.op, pairs, w.n, 24)
    for tree in (False, True):
        _say(f"[full] dnn hoisted tree={tree} pairs [{lo}, {hi}) gpu")
        Cs = env.ctx.spmspm_pairs(A, B, lo, hi, tree=tree, hoist=True)
        _say(f"[full] dnn hoisted tree={tree} oracle")
        env.check(Cs, env.oracle(OA, OB, pairs[lo:hi], tree=tree, hoist=True), (tree, lo, hi))
        Cs.close()
        _say(f"[full] dnn hoisted tree={tree} full layer")
        C = env.ctx.spmspm(A, B, tree=tree, hoist=True)
        err = np.abs(env.ctx.decrypt_decode(env.sk, C) - a @ b).max()
        _say(f"[full] dnn hoisted tree={tree} max-abs error {err:.3e}")
        assert err < 1e-5
        C.close()


# ---- the larger parameter sets (N = 2^16 with 24 Q + 3 P primes, N = 2^17 with 35 Q + 3 P) ----

@pytest.mark.timeout(1200)
def test_large_parameter_set_small_matmul_bit_exact(large):
    """N = 2^16, three primes per digit, three special primes, NTT split 2^7 x 2^9: alignment rotations
    of A and B, a target rotation by S - 1 (three digit steps), shared products; every limb bit-exact."""
    a = np.array([[0.5, -0.25, 0.75]])
    b = np.array([[0.0, 0.3], [0.0, -0.6], [0.9, 0.0]])
    A, B, OA, OB = large.operands("small", a, b)
    _say(f"[large] gpu {large.ctx.plan_stats(A, B)}")
    C = large.ctx.spmspm(A, B)
    _say("[large] oracle")
    large.check(C, large.oracle(OA, OB), "small")
    assert np.abs(large.ctx.decrypt_decode(large.sk, C) - a @ b).max() < 1e-5
    C.close()


@pytest.mark.timeout(1200)
def test_n17_parameter_set_small_matmul_bit_exact():
    """N = 2^17 (35 Q + 3 P primes, four digits, split 2^8 x 2^9): one product, one target rotation by
    1; every key-switch kernel at alpha = K = 3, bit-exact."""
    env = _Env((17, 35, 3, 3, 4))
    a, b = np.array([[0.5, -0.25]]), np.array([[0.75], [0.3]])
    A, B, OA, OB = env.operands("small", a, b)
    _say(f"[large] N=2^17 gpu {env.ctx.plan_stats(A, B)}")
    C = env.ctx.spmspm(A, B)
    _say("[large] N=2^17 oracle")
    env.check(C, env.oracle(OA, OB), "n17")
    assert np.abs(env.ctx.decrypt_decode(env.sk, C) - a @ b).max() < 1e-5
    C.close()
    env.ctx.close()


@pytest.mark.timeout(1200)
def test_large_workload_sampled_pairs_bit_exact(large):
    """The 512 x 512 workload at N = 2^16 (B over four operand chunks, C over eight result chunks):
    pair ranges at the start, middle and end of Algorithm 1's traversal are bit-exact against the
    oracle on the same pairs."""
    w = synth.WORKLOADS["large"]
    _say("[full] large setup")
    a, b = w.operands()
    A, B, OA, OB = large.operands("large", a, b)
    st = large.ctx.plan_stats(A, B)
    assert st.result_chunks == 8 and B.info()["chunks"] == 4
    F = st.matched_pairs
    pairs = spmspm.matched_pairs(w.m, w.n, OA.indptr, OA.indices, OB.indptr, OB.indices)
    assert len(pairs) == F
    for lo, hi in [(0, 2), (F // 2, F // 2 + 2), (F - 2, F)]:
        _say(f"[full] large pairs [{lo}, {hi}) gpu")
        Cs = large.ctx.spmspm_pairs(A, B, lo, hi)
        _say(f"[full] large pairs [{lo}, {hi}) oracle")
        large.check(Cs, large.oracle(OA, OB, pairs[lo:hi]), (lo, hi))
        Cs.close()


@pytest.mark.timeout(1200)
def test_batching_parameters_merged_batch_bit_exact(large):
    """The batching workload's parameters (N = 2^16, 24 Q + 3 P primes, alpha = 3, three digits): three
    of its matmuls of different sizes in ONE fhe_spmspm_batch_pairs call (merged plans, shared
    launches), on seeded prefixes and, for the largest, a range at the end of its traversal (its
    second result chunk). Every result chunk bit-exact against the oracle on the same pairs."""
    from paper_2604_11659_amd import fhe
    w = synth.BATCH_WORKLOADS["batch"]
    specs = w.specs()
    pick, seen = [], set()
    for i, sp in enumerate(specs):  # the first matmul of each of three sizes
        if sp[0] not in seen and len(pick) < 3:
            seen.add(sp[0])
            pick.append(i)
    pick.sort(key=lambda i: specs[i][0])
    As, Bs, ranges, refs = [], [], [], []
    for t, i in enumerate(pick):
        a, b = w.operands(i, specs[i])
        A, B, OA, OB = large.operands(f"batch{i}", a, b, seeds=(10_000 + i, 20_000 + i))
        pairs = spmspm.matched_pairs(a.shape[0], b.shape[1], OA.indptr, OA.indices, OB.indptr, OB.indices)
        lo, hi = (0, 3) if t < 2 else (len(pairs) - 3, len(pairs))
        As.append(A)
        Bs.append(B)
        ranges.append((lo, hi))
        refs.append((OA, OB, pairs[lo:hi]))
    assert len({specs[i][0] for i in pick}) == 3
    _say(f"[batch] matmuls {[(i, specs[i][0]) for i in pick]} ranges {ranges} gpu")
    Cs = large.ctx.spmspm_batch(As, Bs, pair_ranges=ranges)
    assert isinstance(Cs[0], fhe.Matrix)
    for t, (C, (OA, OB, prs)) in enumerate(zip(Cs, refs)):
        _say(f"[batch] oracle of matmul {pick[t]}")
        large.check(C, large.oracle(OA, OB, prs), pick[t])
        C.close()
