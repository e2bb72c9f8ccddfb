"""Pins of the oracle's Algorithm 1/2 plan and of the end-to-end encrypted matmul.

The plan is checked with a slot-level FP64 simulator (plaintext vectors of S
slots, exact cyclic rotations, element-wise products, one-hot masks) against
the dense product; the encrypted path against the FP64 matmul within the
1e-5 max-abs gate.
"""
import itertools

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth


class _SlotParams:
    def __init__(self, S):
        self.S = S


def _simulate(S, a, b):
    """Run the oracle's plan decisions on plaintext slot vectors."""
    m, k = a.shape
    n = b.shape[1]
    ip_a, ix_a, va = synth.to_csr(a)
    ip_b, ix_b, vb = synth.to_csc(b)
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
    rotations = 0
    for (i, j, a_pos, b_pos) in spmspm.matched_pairs(m, n, ip_a, ix_a, ip_b, ix_b):
        ca, cb, ra, rb, mn = spmspm.alignment(pr, a_pos, b_pos)
        vA, vB = np.roll(ca_vec[ca], -ra), np.roll(cb_vec[cb], -rb)
        rotations += (ra != 0) + (rb != 0)
        assert (ra != 0) + (rb != 0) <= 1
        d = vA * vB
        onehot = np.zeros(S)
        onehot[mn] = 1.0
        d = d * onehot
        cr, rot = spmspm.target(pr, i, j, n, mn)
        res[cr] += np.roll(d, -rot)
    flat = res.reshape(-1)[: m * n]
    return flat.reshape(m, n), rotations


@pytest.mark.parametrize("S", [4, 8, 64])
def test_plan_simulator_equals_dense_bruteforce(S):
    rng = np.random.default_rng(S)
    for m, k, n in itertools.product([1, 2, 3, 5], [1, 3, 4], [1, 2, 5]):
        for sp in [0.0, 0.4, 0.8, 1.0]:
            a = synth.sparse_dense(m, k, sp, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
            b = synth.sparse_dense(k, n, sp, "uniform", int(rng.integers(1 << 30)), int(rng.integers(1 << 30)))
            c, _ = _simulate(S, a, b)
            assert np.abs(c - a @ b).max() < 1e-12


def test_matched_pairs_is_the_nonzero_product_set():
    rng = np.random.default_rng(7)
    for trial in range(20):
        m, k, n = (int(x) for x in rng.integers(1, 9, 3))
        a = synth.sparse_dense(m, k, float(rng.uniform()), "uniform", trial, trial + 100)
        b = synth.sparse_dense(k, n, float(rng.uniform()), "uniform", trial + 200, trial + 300)
        ip_a, ix_a, _ = synth.to_csr(a)
        ip_b, ix_b, _ = synth.to_csc(b)
        pairs = spmspm.matched_pairs(m, n, ip_a, ix_a, ip_b, ix_b)
        brute = []
        for i in range(m):
            for j in range(n):
                for kk in range(k):
                    if a[i, kk] != 0 and b[kk, j] != 0:
                        ap = int(ip_a[i]) + int(np.count_nonzero(a[i, :kk]))
                        bp = int(ip_b[j]) + int(np.count_nonzero(b[:kk, j]))
                        brute.append((i, j, ap, bp))
        assert pairs == brute
        # F = sum_k nnzcol_A(k) * nnzrow_B(k)
        F = sum(int(np.count_nonzero(a[:, kk])) * int(np.count_nonzero(b[kk, :])) for kk in range(k))
        assert len(pairs) == F


def test_full_sparsity_does_no_work():
    a = np.zeros((16, 16))
    ip_a, ix_a, _ = synth.to_csr(a)
    assert spmspm.matched_pairs(16, 16, ip_a, ix_a, ip_a, ix_a) == []


def test_workload_shapes_and_counts():
    """Exact zero counts (round(sparsity * size)) and the plan size of the small workload."""
    w = synth.WORKLOADS["plain"]
    a, b = w.operands()
    assert a.shape == (16, 16) and b.shape == (16, 16)
    assert int((a == 0).sum()) == 192 and int((b == 0).sum()) == 192
    ip_a, ix_a, _ = synth.to_csr(a)
    ip_b, ix_b, _ = synth.to_csc(b)
    F = len(spmspm.matched_pairs(16, 16, ip_a, ix_a, ip_b, ix_b))
    assert F == sum(int(np.count_nonzero(a[:, kk])) * int(np.count_nonzero(b[kk, :])) for kk in range(16))


def _e2e(params, a, b, workers=1):
    keys = ckks.Keys(params, 42)
    m, k = a.shape
    n = b.shape[1]
    A = spmspm.encrypt_csr(params, keys, m, k, *synth.to_csr(a), seed=43)
    B = spmspm.encrypt_csc(params, keys, k, n, *synth.to_csc(b), seed=44)
    res = spmspm.spmspm(params, keys, A, B, workers=workers)
    return res, spmspm.decrypt_result(params, keys, res, m, n)


def test_encrypted_matmul_matches_fp64():
    params = ckks.Params(log_n=10, n_q=4, n_p=1, alpha=1, rot_digits=1)
    a = synth.sparse_dense(6, 5, 0.5, "uniform", 0, 2)
    b = synth.sparse_dense(5, 7, 0.5, "uniform", 1, 3)
    res, c = _e2e(params, a, b)
    assert len(res) == 1 and res[0].nl == 2 and res[0].scale == 2.0 ** 50
    assert np.abs(c - a @ b).max() < 1e-5


def test_encrypted_matmul_chunked_digits():
    """Operands and result spill over several S-slot chunks; alpha = 2, two rotation digits."""
    params = ckks.Params(log_n=6, n_q=6, n_p=2, alpha=2, rot_digits=2)
    a = synth.sparse_dense(8, 8, 0.3, "uniform", 10, 12)
    b = synth.sparse_dense(8, 8, 0.3, "halfnormal", 11, 13)
    assert np.count_nonzero(a) > params.S and 64 > params.S
    res, c = _e2e(params, a, b, workers=4)
    assert len(res) == 2
    assert np.abs(c - a @ b).max() < 1e-5


def test_full_sparsity_result_is_exact_zero():
    params = ckks.Params(log_n=8, n_q=4, n_p=1, alpha=1, rot_digits=1)
    a = np.zeros((4, 4))
    res, c = _e2e(params, a, a)
    assert (res[0].data == 0).all()
    assert (c == 0).all()


def test_worker_split_is_bit_identical():
    params = ckks.Params(log_n=8, n_q=4, n_p=1, alpha=1, rot_digits=1)
    a = synth.sparse_dense(4, 4, 0.5, "uniform", 3, 5)
    b = synth.sparse_dense(4, 4, 0.5, "uniform", 4, 6)
    r1, _ = _e2e(params, a, b, workers=1)
    r3, _ = _e2e(params, a, b, workers=3)
    assert all((x.data == y.data).all() for x, y in zip(r1, r3))
