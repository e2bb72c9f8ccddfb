"""Pins of the oracle's naive sparse and naive dense plans (the paper's evaluation baselines, Section 4).

Naive dense multiplies every entry of A by every entry of B it meets (operands store every entry);
naive sparse skips a product only where both of its values are zero. The pins:
  * a slot-level FP64 simulation of the naive sparse plan equals the dense matmul, by brute force
    over small shapes and zero patterns (the skipped products are 0 x 0);
  * the number of products has a closed form, sum_k (n a_k + m b_k - a_k b_k) with a_k / b_k the
    nonzeros in column k of A / row k of B, which differs both from the naive dense count m k n and
    from the CSR x CSC count sum_k a_k b_k (a reading that skipped a product when EITHER value is zero
    would give the latter);
  * all-nonzero flags give the naive dense pairs; all-zero operands give no pairs;
  * an encrypted naive sparse matmul decrypts within 1e-5 of FP64, and equals the per-pair sequence
    on exactly the kept pairs.
"""
import itertools

import numpy as np

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth


class _SlotParams:
    def __init__(self, S):
        self.S = S


def _naive_pairs(a, b):
    ipa, ixa, _ = synth.full_csr(a)
    ipb, ixb, _ = synth.full_csc(b)
    return spmspm.naive_sparse_pairs(a.shape[0], b.shape[1], ipa, ixa, ipb, ixb, synth.stored_nonzero_csr(a),
                                     synth.stored_nonzero_csc(b))


def _simulate(S, a, b, pairs):
    """The oracle's alignment / mask / target decisions on plaintext slot vectors of the dense packing."""
    m, n = a.shape[0], b.shape[1]
    va, vb = synth.full_csr(a)[2], synth.full_csc(b)[2]
    pr = _SlotParams(S)

    def chunks(v):
        nch = max(1, -(-len(v) // S))
        out = np.zeros((nch, S))
        for c in range(nch):
            seg = v[c * S:(c + 1) * S]
            out[c, :len(seg)] = seg
        return out

    ca_vec, cb_vec = chunks(va), chunks(vb)
    res = np.zeros((spmspm.result_chunks(pr, m, n), S))
    for (i, j, a_pos, b_pos) in pairs:
        ca, cb, ra, rb, mn = spmspm.alignment(pr, a_pos, b_pos)
        d = np.roll(ca_vec[ca], -ra) * np.roll(cb_vec[cb], -rb)
        onehot = np.zeros(S)
        onehot[mn] = 1.0
        cr, rot = spmspm.target(pr, i, j, n, mn)
        res[cr] += np.roll(d * onehot, -rot)
    return res.reshape(-1)[: m * n].reshape(m, n)


def test_naive_sparse_simulator_equals_dense_bruteforce():
    rng = np.random.default_rng(11)
    for S in (4, 16, 64):
        for m, k, n in itertools.product([1, 2, 4], [1, 3, 5], [1, 2, 3]):
            for sa, sb in [(0.0, 0.0), (0.5, 0.3), (0.8, 0.8), (1.0, 0.5), (1.0, 1.0)]:
                a = synth.sparse_dense(m, k, sa, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
                b = synth.sparse_dense(k, n, sb, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
                got = _simulate(S, a, b, _naive_pairs(a, b))
                assert np.abs(got - a @ b).max() < 1e-12, (S, m, k, n, sa, sb)


def test_naive_sparse_pair_count_closed_form():
    for seed, (m, k, n, sa, sb) in enumerate([(4, 5, 3, 0.5, 0.5), (6, 6, 6, 0.8, 0.2), (3, 7, 2, 0.0, 0.9),
                                              (5, 4, 5, 0.6, 0.6)]):
        a = synth.sparse_dense(m, k, sa, "uniform", seed, seed + 10)
        b = synth.sparse_dense(k, n, sb, "halfnormal", seed + 20, seed + 30)
        ak = (a != 0).sum(axis=0)
        bk = (b != 0).sum(axis=1)
        pairs = _naive_pairs(a, b)
        assert len(pairs) == int(np.sum(n * ak + m * bk - ak * bk))
        # every kept pair has at least one nonzero value; every dropped triple has two zeros
        kept = {(i, j, pa % k) for (i, j, pa, _) in pairs}
        for i, kk, j in itertools.product(range(m), range(k), range(n)):
            assert ((i, j, kk) in kept) == (a[i, kk] != 0 or b[kk, j] != 0)
        if 0 < sa < 1 and 0 < sb < 1:
            assert len(pairs) not in (m * k * n, int(ak @ bk))


def test_naive_sparse_extremes():
    a = synth.sparse_dense(3, 4, 0.0, "uniform", 1, 2)
    b = synth.sparse_dense(4, 2, 0.0, "uniform", 3, 4)
    ipa, ixa, _ = synth.full_csr(a)
    ipb, ixb, _ = synth.full_csc(b)
    dense = spmspm.matched_pairs(3, 2, ipa, ixa, ipb, ixb)
    assert len(dense) == 3 * 4 * 2
    assert _naive_pairs(a, b) == dense  # nothing is zero: the naive dense pairs, in the same order
    z = np.zeros((3, 4)), np.zeros((4, 2))
    assert _naive_pairs(*z) == []


def test_encrypted_naive_sparse_matches_fp64_and_per_pair_sequence():
    pr = ckks.Params(log_n=12, n_q=4, n_p=1, alpha=1, rot_digits=2)
    keys = ckks.Keys(pr, 42)
    a = synth.sparse_dense(3, 4, 0.5, "uniform", 5, 6)
    b = synth.sparse_dense(4, 3, 0.5, "uniform", 7, 8)
    A = spmspm.encrypt_csr(pr, keys, 3, 4, *synth.full_csr(a), seed=43)
    B = spmspm.encrypt_csc(pr, keys, 4, 3, *synth.full_csc(b), seed=44)
    pairs = _naive_pairs(a, b)
    res = spmspm.spmspm(pr, keys, A, B, pairs=pairs)
    got = spmspm.decrypt_result(pr, keys, res, 3, 3)
    assert np.abs(got - a @ b).max() < 1e-5
    # the naive dense plan runs more products and reaches the same values
    dense = spmspm.spmspm(pr, keys, A, B)
    assert np.abs(spmspm.decrypt_result(pr, keys, dense, 3, 3) - a @ b).max() < 1e-5
    assert not (dense[0].data == res[0].data).all()
