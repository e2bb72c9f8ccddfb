"""Pins of the oracle's grouped target rotations (pairs sharing result chunk and rotation summed
before one rescale and one rotation).

* slot level: the grouped plan on plaintext slot vectors equals the dense product (brute force,
  several result chunks, so a grouping key that forgot the chunk or the rotation fails);
* singleton groups: when every group holds one pair the grouped form is Algorithm 2's per-pair
  sequence bit for bit;
* operation counts: one second rescale and one target rotation per group, not per pair;
* encrypted: the decrypted grouped matmul is within the 1e-5 gate of FP64, also over several
  operand and result chunks with two rotation digits.

Digit tree (the grouped plan with its target rotations shared digit by digit):
* the tree's sum on plaintext slot vectors equals rotating every item by its full amount (random
  items, one to four digits), and the tree plan equals the dense product;
* with one rotation digit it is the grouped plan bit for bit;
* key switches: alignment + one per group with a nonzero low digit + one per distinct nonzero
  (chunk, high digit); decrypted within 1e-5; worker splits give the same limbs.
"""
import itertools

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth


class _SlotParams:
    def __init__(self, S):
        self.S = S


def _simulate_grouped(S, a, b):
    m, k = a.shape
    n = b.shape[1]
    ip_a, ix_a, va = synth.to_csr(a)
    ip_b, ix_b, vb = synth.to_csc(b)
    pr = _SlotParams(S)

    def chunks(v):
        out = np.zeros((max(1, -(-len(v) // S)), S))
        for c in range(out.shape[0]):
            seg = v[c * S:(c + 1) * S]
            out[c, :len(seg)] = seg
        return out

    ca_vec, cb_vec = chunks(va), chunks(vb)
    res = np.zeros((spmspm.result_chunks(pr, m, n), S))
    pairs = spmspm.matched_pairs(m, n, ip_a, ix_a, ip_b, ix_b)
    groups = spmspm.target_groups(pr, pairs, n)
    assert sum(len(mem) for _, mem in groups) == len(pairs)
    for (cr, rot), members in groups:
        acc = np.zeros(S)
        for (i, j, a_pos, b_pos) in members:
            ca, cb, ra, rb, mn = spmspm.alignment(pr, a_pos, b_pos)
            onehot = np.zeros(S)
            onehot[mn] = 1.0
            acc += np.roll(ca_vec[ca], -ra) * np.roll(cb_vec[cb], -rb) * onehot
        res[cr] += np.roll(acc, -rot)
    return res.reshape(-1)[: m * n].reshape(m, n), len(groups), len(pairs)


@pytest.mark.parametrize("S", [4, 8, 64])
def test_grouped_simulator_equals_dense_bruteforce(S):
    rng = np.random.default_rng(100 + S)
    merged = 0
    for m, k, n in itertools.product([1, 3, 5], [2, 4], [2, 3, 6]):
        for sp in [0.0, 0.5, 1.0]:
            a = synth.sparse_dense(m, k, sp, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
            b = synth.sparse_dense(k, n, sp, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
            c, ng, F = _simulate_grouped(S, a, b)
            assert np.abs(c - a @ b).max() < 1e-12
            merged += F - ng
    assert merged > 0  # the cases do exercise groups of several pairs


def _enc(params, keys, a, b):
    m, k = a.shape
    n = b.shape[1]
    A = spmspm.encrypt_csr(params, keys, m, k, *synth.to_csr(a), seed=43)
    B = spmspm.encrypt_csc(params, keys, k, n, *synth.to_csc(b), seed=44)
    return A, B


def test_singleton_groups_equal_per_pair_sequence():
    """A dense row times a dense column: pair p isolates slot p with rotation p, so every group
    is a single pair and the grouped form must reproduce Algorithm 2 exactly."""
    params = ckks.Params(log_n=8, n_q=4, n_p=1, alpha=1, rot_digits=1)
    keys = ckks.Keys(params, 42)
    rng = np.random.default_rng(5)
    a = rng.uniform(-1, 1, (1, 6))
    b = rng.uniform(-1, 1, (6, 1))
    A, B = _enc(params, keys, a, b)
    pairs = spmspm.matched_pairs(1, 1, A.indptr, A.indices, B.indptr, B.indices)
    groups = spmspm.target_groups(params, pairs, 1)
    assert len(groups) == len(pairs) == 6
    lit = spmspm.spmspm(params, keys, A, B)
    grp = spmspm.spmspm(params, keys, A, B, grouped=True)
    assert all((x.data == y.data).all() for x, y in zip(lit, grp))


def test_grouped_issues_one_rescale_and_rotation_per_group(monkeypatch):
    params = ckks.Params(log_n=8, n_q=4, n_p=1, alpha=1, rot_digits=1)
    keys = ckks.Keys(params, 42)
    a = synth.sparse_dense(4, 5, 0.3, "uniform", 7, 9)
    b = synth.sparse_dense(5, 4, 0.3, "uniform", 8, 10)
    A, B = _enc(params, keys, a, b)
    pairs = spmspm.matched_pairs(4, 4, A.indptr, A.indices, B.indptr, B.indices)
    groups = spmspm.target_groups(params, pairs, 4)
    assert len(groups) < len(pairs)
    calls = {"rescale": 0, "rot": 0}
    real_rescale, real_rot = ckks.rescale, ckks.rotate_single

    def rescale(p, ct):
        calls["rescale"] += 1
        return real_rescale(p, ct)

    def rot(p, k, ct, r):
        calls["rot"] += 1
        return real_rot(p, k, ct, r)

    monkeypatch.setattr(ckks, "rescale", rescale)
    monkeypatch.setattr(ckks, "rotate_single", rot)
    spmspm.spmspm(params, keys, A, B, grouped=True)
    align = sum(len(ckks.rotation_steps(params, max(r[2], r[3])))
                for r in (spmspm.alignment(params, ap, bp) for (_, _, ap, bp) in pairs))
    target = sum(len(ckks.rotation_steps(params, rot_)) for (_, rot_), _ in groups)
    # rescale #1 per pair (the oracle recomputes every product), rescale #2 per group
    assert calls["rescale"] == len(pairs) + len(groups)
    assert calls["rot"] == align + target


def test_grouped_encrypted_matmul_matches_fp64():
    params = ckks.Params(log_n=10, n_q=4, n_p=1, alpha=1, rot_digits=1)
    keys = ckks.Keys(params, 42)
    a = synth.sparse_dense(6, 5, 0.4, "uniform", 0, 2)
    b = synth.sparse_dense(5, 7, 0.4, "uniform", 1, 3)
    A, B = _enc(params, keys, a, b)
    res = spmspm.spmspm(params, keys, A, B, grouped=True)
    c = spmspm.decrypt_result(params, keys, res, 6, 7)
    assert np.abs(c - a @ b).max() < 1e-5
    # fewer roundings and key switches than the per-pair form: the error is no larger
    lit = spmspm.decrypt_result(params, keys, spmspm.spmspm(params, keys, A, B), 6, 7)
    assert np.abs(c - a @ b).max() <= 1.5 * np.abs(lit - a @ b).max() + 1e-12


def test_grouped_chunked_digits_workers():
    """Operands and result over several S-slot chunks, alpha = 2, two rotation digits, groups split
    across worker processes (exact modular sums: the split does not change the bits)."""
    params = ckks.Params(log_n=6, n_q=6, n_p=2, alpha=2, rot_digits=2)
    keys = ckks.Keys(params, 42)
    a = synth.sparse_dense(8, 8, 0.3, "uniform", 10, 12)
    b = synth.sparse_dense(8, 8, 0.3, "halfnormal", 11, 13)
    A, B = _enc(params, keys, a, b)
    r1 = spmspm.spmspm(params, keys, A, B, grouped=True)
    r4 = spmspm.spmspm(params, keys, A, B, grouped=True, workers=4)
    assert len(r1) == 2
    assert all((x.data == y.data).all() for x, y in zip(r1, r4))
    c = spmspm.decrypt_result(params, keys, r1, 8, 8)
    assert np.abs(c - a @ b).max() < 1e-5


# ---- digit tree (grouped plan whose target rotations are shared digit by digit) ----

class _TreeParams:
    def __init__(self, S, D):
        self.S, self.rot_digits = S, D

    def rot_step_bits(self):
        return -(-(self.S.bit_length() - 1) // self.rot_digits)


@pytest.mark.parametrize("S,D", [(16, 2), (64, 2), (64, 3), (256, 4), (32, 1)])
def test_digit_tree_sum_equals_direct_rotations(S, D):
    """On plaintext slot vectors (exact cyclic rotations): the tree's sum equals rotating every item
    by its full amount and adding per chunk."""
    pr = _TreeParams(S, D)
    rng = np.random.default_rng(S * 10 + D)
    for trial in range(20):
        n, nres = int(rng.integers(1, 40)), int(rng.integers(1, 4))
        items = [(int(rng.integers(nres)), int(rng.integers(S)), rng.normal(size=S)) for _ in range(n)]
        got = spmspm.digit_tree_sum(pr, items, nres, lambda x, r: np.roll(x, -r), lambda x, y: x + y)
        want = [None] * nres
        for (cr, rot, x) in items:
            v = np.roll(x, -rot)
            want[cr] = v if want[cr] is None else want[cr] + v
        for g, w in zip(got, want):
            assert (g is None) == (w is None)
            if w is not None:
                assert np.abs(g - w).max() < 1e-12


@pytest.mark.parametrize("S,D", [(8, 2), (16, 2), (64, 3)])
def test_digit_tree_plan_simulator_equals_dense(S, D):
    pr = _TreeParams(S, D)
    rng = np.random.default_rng(7 * S + D)
    for m, k, n in itertools.product([2, 5], [2, 4], [3, 6]):
        a = synth.sparse_dense(m, k, 0.3, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
        b = synth.sparse_dense(k, n, 0.3, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
        ip_a, ix_a, va = synth.to_csr(a)
        ip_b, ix_b, vb = synth.to_csc(b)

        def chunks(v):
            out = np.zeros((max(1, -(-len(v) // S)), S))
            for c in range(out.shape[0]):
                seg = v[c * S:(c + 1) * S]
                out[c, :len(seg)] = seg
            return out

        ca_vec, cb_vec = chunks(va), chunks(vb)
        pairs = spmspm.matched_pairs(m, n, ip_a, ix_a, ip_b, ix_b)
        items = []
        for (cr, rot), members in spmspm.target_groups(pr, pairs, n):
            acc = np.zeros(S)
            for (i, j, a_pos, b_pos) in members:
                ca, cb, ra, rb, mn = spmspm.alignment(pr, a_pos, b_pos)
                onehot = np.zeros(S)
                onehot[mn] = 1.0
                acc += np.roll(ca_vec[ca], -ra) * np.roll(cb_vec[cb], -rb) * onehot
            items.append((cr, rot, acc))
        nres = spmspm.result_chunks(pr, m, n)
        res = spmspm.digit_tree_sum(pr, items, nres, lambda x, r: np.roll(x, -r), lambda x, y: x + y)
        flat = np.concatenate([np.zeros(S) if r is None else r for r in res])[: m * n]
        assert np.abs(flat.reshape(m, n) - a @ b).max() < 1e-12


def test_digit_tree_with_one_digit_is_the_grouped_plan():
    params = ckks.Params(log_n=8, n_q=4, n_p=1, alpha=1, rot_digits=1)
    keys = ckks.Keys(params, 42)
    a = synth.sparse_dense(4, 5, 0.3, "uniform", 7, 9)
    b = synth.sparse_dense(5, 4, 0.3, "uniform", 8, 10)
    A, B = _enc(params, keys, a, b)
    g = spmspm.spmspm(params, keys, A, B, grouped=True)
    t = spmspm.spmspm(params, keys, A, B, tree=True)
    assert all((x.data == y.data).all() for x, y in zip(g, t))


def test_digit_tree_encrypted_counts_and_fp64(monkeypatch):
    """Two rotation digits over two result chunks: decrypts within 1e-5 of FP64; the key switches are
    the alignment ones plus one per group with a nonzero low digit plus one per distinct (chunk,
    high digit) that is nonzero; the worker split does not change the limbs."""
    params = ckks.Params(log_n=6, n_q=6, n_p=2, alpha=2, rot_digits=2)
    keys = ckks.Keys(params, 42)
    a = synth.sparse_dense(8, 8, 0.3, "uniform", 10, 12)
    b = synth.sparse_dense(8, 8, 0.3, "halfnormal", 11, 13)
    A, B = _enc(params, keys, a, b)
    r4 = spmspm.spmspm(params, keys, A, B, tree=True, workers=4)
    pairs = spmspm.matched_pairs(8, 8, A.indptr, A.indices, B.indptr, B.indices)
    groups = spmspm.target_groups(params, pairs, 8)
    bits = params.rot_step_bits()
    low = (1 << bits) - 1
    align = sum(len(ckks.rotation_steps(params, max(r[2], r[3])))
                for r in (spmspm.alignment(params, ap, bp) for (_, _, ap, bp) in pairs))
    lvl0 = sum(1 for (_, rot), _ in groups if rot & low)
    lvl1 = len({(cr, rot >> bits) for (cr, rot), _ in groups if rot >> bits})
    assert lvl0 + lvl1 < sum(len(ckks.rotation_steps(params, rot)) for (_, rot), _ in groups)
    calls = {"rot": 0}
    real_rot = ckks.rotate_single

    def rot(p, k, ct, r):
        calls["rot"] += 1
        return real_rot(p, k, ct, r)

    monkeypatch.setattr(ckks, "rotate_single", rot)
    r1 = spmspm.spmspm(params, keys, A, B, tree=True)
    monkeypatch.setattr(ckks, "rotate_single", real_rot)
    assert calls["rot"] == align + lvl0 + lvl1
    assert len(r1) == 2
    assert all((x.data == y.data).all() for x, y in zip(r1, r4))
    c = spmspm.decrypt_result(params, keys, r1, 8, 8)
    assert np.abs(c - a @ b).max() < 1e-5
