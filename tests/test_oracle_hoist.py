"""Pins of the oracle's hoisted rotation (the automorphism applied to the ModUp digits of the input,
so one ModUp serves every rotation of a ciphertext) and of the plan that hoists its alignment rotations.

* the digit-wise key switch with the identity automorphism is the key switch itself, bit for bit;
* tau_g(ModUp_j(x)) is congruent to tau_g(x) modulo the digit modulus D_j with a multiplier below alpha
  in magnitude (big-integer CRT): a valid key-switch input for tau_g(x);
* a hoisted key switch decrypts to tau_g(d) s' within the noise bound (and not to a wrong target);
* a hoisted rotation decrypts to the left rotation of the slots;
* the plan with hoisted alignment rotations decrypts within 1e-5 of FP64, equals the per-pair plan bit for
  bit when no alignment rotation is needed, and differs from it when some are.
"""
import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth
from tests.bigint import centered, crt
from tests.test_oracle_ops import _ks_error, _rand_limbs


@pytest.mark.parametrize("alpha,n_q,n_p,nl", [(1, 4, 1, 4), (2, 6, 2, 5), (3, 6, 3, 6)])
def test_digit_keyswitch_with_identity_is_keyswitch(alpha, n_q, n_p, nl):
    params = ckks.Params(log_n=6, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=1)
    keys = ckks.Keys(params, 42)
    d = _rand_limbs(np.random.default_rng(nl), params.q[:nl], params.N)
    g = pow(5, 3, 2 * params.N)
    ref = ckks.keyswitch(params, d, keys.rot_key(g))
    got = ckks.keyswitch_digits(params, ckks.modup_digits(params, d), keys.rot_key(g), nl, 1)
    assert (ref == got).all()


@pytest.mark.parametrize("alpha,nl,j", [(2, 5, 0), (2, 5, 2), (3, 6, 1)])
def test_automorphism_of_modup_is_a_lift_of_the_automorphism(alpha, nl, j):
    params = ckks.Params(log_n=5, n_q=6, n_p=3, alpha=alpha, rot_digits=1)
    N = params.N
    d = _rand_limbs(np.random.default_rng(10 * alpha + j), params.q[:nl], N)
    g = pow(5, 7, 2 * N)
    em = ckks.ext_moduli(params, nl)
    ext = ckks.modup_digits(params, d)[j]
    tau_ext = np.zeros_like(ext)
    from oracle._lib import P, lib
    lib().or_automorph(P(np.ascontiguousarray(ext)), P(tau_ext), N, g, P(em), nl + params.n_p)
    tau_d = ckks.automorph(params, ckks.Ct(d[None], 1.0), g).data[0]
    lo, hi = j * alpha, min((j + 1) * alpha, nl)
    digit = [int(q) for q in em[lo:hi]]
    Dj = 1
    for q in digit:
        Dj *= q
    outside = [e for e in range(nl + params.n_p) if not (lo <= e < hi)]
    for k in range(N):
        x, _ = crt([tau_d[i, k] for i in range(lo, hi)], digit)
        for i in range(lo, hi):  # inside the digit: exactly tau_g(x)
            assert int(tau_ext[i, k]) == int(tau_d[i, k])
        Y, M = crt([tau_ext[e, k] for e in outside], [int(em[e]) for e in outside])
        y = centered(Y, M)
        assert (y - x) % Dj == 0 and abs((y - x) // Dj) < alpha + 1


@pytest.mark.parametrize("alpha,n_q,n_p,nl", [(1, 4, 1, 4), (2, 6, 2, 6), (3, 6, 3, 4)])
def test_hoisted_keyswitch_decrypts_to_target(alpha, n_q, n_p, nl):
    params = ckks.Params(log_n=7, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=1)
    keys = ckks.Keys(params, 42)
    d = _rand_limbs(np.random.default_rng(3 + nl), params.q[:nl], params.N)
    g = pow(5, 5, 2 * params.N)
    u = ckks.keyswitch_digits(params, ckks.modup_digits(params, d), keys.rot_key(g), nl, g)
    tau_d = ckks.automorph(params, ckks.Ct(d[None], 1.0), g).data[0]
    bound = n_p * (params.N + 1) + alpha * 4096
    assert _ks_error(params, keys, tau_d, u, ckks.automorph_signed(keys.s, g)) <= bound
    assert _ks_error(params, keys, d, u, ckks.automorph_signed(keys.s, g)) > 2 ** 60


@pytest.mark.parametrize("r", [1, 3, 127, 128, 300, 511])
def test_hoisted_rotation_decrypts_to_left_rotation(r):
    params = ckks.Params(log_n=10, n_q=5, n_p=2, alpha=2, rot_digits=2)
    keys = ckks.Keys(params, 42)
    z = np.random.default_rng(2).uniform(-1, 1, params.S)
    ct = ckks.encrypt(params, keys, ckks.encode(z, params.delta_a, params.N), 43, 0, params.delta_a)
    out = ckks.decrypt_decode(params, keys, ckks.rotate_hoisted(params, keys, ct, r), np.arange(params.S))
    assert np.abs(out - np.roll(z, -r)).max() < 1e-6


def _enc(params, keys, a, b):
    (m, k), n = a.shape, b.shape[1]
    return (spmspm.encrypt_csr(params, keys, m, k, *synth.to_csr(a), seed=43),
            spmspm.encrypt_csc(params, keys, k, n, *synth.to_csc(b), seed=44))


def test_hoisted_plan_fp64_and_bits():
    params = ckks.Params(log_n=6, n_q=6, n_p=2, alpha=2, rot_digits=2)
    keys = ckks.Keys(params, 42)
    a = synth.sparse_dense(8, 8, 0.3, "uniform", 10, 12)
    b = synth.sparse_dense(8, 8, 0.3, "halfnormal", 11, 13)
    A, B = _enc(params, keys, a, b)
    h = spmspm.spmspm(params, keys, A, B, hoist=True, workers=4)
    c = spmspm.decrypt_result(params, keys, h, 8, 8)
    assert np.abs(c - a @ b).max() < 1e-5
    lit = spmspm.spmspm(params, keys, A, B, workers=4)
    assert any((x.data != y.data).any() for x, y in zip(h, lit))  # alignment rotations present
    t = spmspm.spmspm(params, keys, A, B, tree=True, hoist=True, workers=4)
    assert np.abs(spmspm.decrypt_result(params, keys, t, 8, 8) - a @ b).max() < 1e-5


def test_hoisted_plan_without_alignment_is_per_pair():
    """A dense row times a dense column: every pair has equal local slots, so no alignment rotation."""
    params = ckks.Params(log_n=8, n_q=4, n_p=1, alpha=1, rot_digits=1)
    keys = ckks.Keys(params, 42)
    rng = np.random.default_rng(9)
    a, b = rng.uniform(-1, 1, (1, 5)), rng.uniform(-1, 1, (5, 1))
    A, B = _enc(params, keys, a, b)
    h = spmspm.spmspm(params, keys, A, B, hoist=True)
    lit = spmspm.spmspm(params, keys, A, B)
    assert all((x.data == y.data).all() for x, y in zip(h, lit))
