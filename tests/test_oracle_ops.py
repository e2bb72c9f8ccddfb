"""Pins of the oracle's CKKS operations.

ModUp / ModDown / rescale are checked against exact big-integer identities;
the tensor product against the ring identity on decryption; key switching,
rotation, multiplication and masking against decrypt-after-operation
invariants within the noise bound.
"""
import numpy as np
import pytest

from oracle import ckks
from oracle._lib import P, lib
from tests.bigint import centered, crt, negacyclic_mul


def _rand_limbs(rng, moduli, N):
    return np.stack([rng.integers(0, int(q), N, dtype=np.uint64) for q in moduli])


@pytest.mark.parametrize("alpha,nl,j", [(3, 6, 0), (3, 6, 1), (3, 5, 1), (2, 5, 2), (1, 4, 2)])
def test_modup_is_crt_lift_plus_small_multiple(alpha, nl, j):
    """ext = x + u D_j on every modulus, with 0 <= u < alpha (no correction term)."""
    params = ckks.Params(log_n=5, n_q=6, n_p=3, alpha=alpha, rot_digits=1)
    N = params.N
    rng = np.random.default_rng(alpha * 10 + nl + j)
    d = _rand_limbs(rng, params.q[:nl], N)
    lo, hi = j * alpha, min((j + 1) * alpha, nl)
    ext_mod = np.array(list(params.q[:nl]) + list(params.p), np.uint64)
    ext = np.zeros((nl + params.n_p, N), np.uint64)
    lib().or_modup(P(d), nl, lo, hi, P(ext_mod), params.n_p, N, P(ext))
    digit = [int(x) for x in ext_mod[lo:hi]]
    Dj = 1
    for q in digit:
        Dj *= q
    outside = [e for e in range(nl + params.n_p) if not (lo <= e < hi)]
    for k in range(N):
        x, _ = crt([d[i, k] for i in range(lo, hi)], digit)
        Y, M = crt([ext[e, k] for e in outside], [int(ext_mod[e]) for e in outside])
        assert M > alpha * Dj
        assert Y < alpha * Dj and (Y - x) % Dj == 0
        for i in range(lo, hi):
            assert int(ext[i, k]) == int(d[i, k])


@pytest.mark.parametrize("nl,nk", [(4, 1), (6, 2), (5, 3)])
def test_moddown_is_division_by_p_up_to_k(nl, nk):
    """out * P = U - Z (mod Q P) with Z = U (mod P) and |Z| < K P / 2 (centred conversion): out is U / P
    rounded with an error below K / 2 + 1 / 2; with one special prime it is the nearest integer."""
    params = ckks.Params(log_n=5, n_q=6, n_p=nk, alpha=1, rot_digits=1)
    N = params.N
    rng = np.random.default_rng(nl * 7 + nk)
    ext_mod = np.array(list(params.q[:nl]) + list(params.p), np.uint64)
    u = _rand_limbs(rng, ext_mod, N)
    out = np.zeros((nl, N), np.uint64)
    lib().or_moddown(P(u), nl, P(ext_mod), nk, N, P(out))
    Pp = 1
    for p in params.p:
        Pp *= p
    Ql = 1
    for q in params.q[:nl]:
        Ql *= q
    for k in range(N):
        U, _ = crt([u[e, k] for e in range(nl + nk)], [int(m) for m in ext_mod])
        W, _ = crt([out[i, k] for i in range(nl)], list(params.q[:nl]))
        Z = centered((U - W * Pp) % (Ql * Pp), Ql * Pp)
        assert 2 * abs(Z) < nk * Pp
        assert (Z - U) % Pp == 0


@pytest.mark.parametrize("nl", [2, 3, 5])
def test_rescale_is_exact_rounded_division(nl):
    params = ckks.Params(log_n=5, n_q=5, n_p=1, alpha=1, rot_digits=1)
    N = params.N
    rng = np.random.default_rng(nl)
    c = _rand_limbs(rng, params.q[:nl], N)[None].copy()
    out = ckks.rescale(params, ckks.Ct(c, 1.0)).data[0]
    ql = params.q[nl - 1]
    for k in range(N):
        X, _ = crt([c[0, i, k] for i in range(nl)], list(params.q[:nl]))
        v = centered(X % ql, ql)
        assert (X - v) % ql == 0
        Y = (X - v) // ql
        for i in range(nl - 1):
            assert int(out[i, k]) == Y % params.q[i]


def test_tensor_ring_identity():
    """d0 + d1 s + d2 s^2 = (a0 + a1 s)(b0 + b1 s) in Z_q[X]/(X^N+1), Python schoolbook."""
    params = ckks.Params(log_n=4, n_q=3, n_p=1, alpha=1, rot_digits=1)
    N = params.N
    rng = np.random.default_rng(5)
    a = np.stack([_rand_limbs(rng, params.q, N) for _ in range(2)])
    b = np.stack([_rand_limbs(rng, params.q, N) for _ in range(2)])
    s = rng.integers(-1, 2, N)
    d = np.zeros((3, 3, N), np.uint64)
    lib().or_tensor(P(a), P(b), 3, N, P(params.qp(3)), P(d))
    for i, q in enumerate(params.q):
        sl = [int(x) % q for x in s]
        s2 = negacyclic_mul(sl, sl, q)
        lhs = [(int(d[0, i, k]) + x + y) % q for k, (x, y) in
               enumerate(zip(negacyclic_mul(d[1, i], sl, q), negacyclic_mul(d[2, i], s2, q)))]
        ma = [(int(a[0, i, k]) + x) % q for k, x in enumerate(negacyclic_mul(a[1, i], sl, q))]
        mb = [(int(b[0, i, k]) + x) % q for k, x in enumerate(negacyclic_mul(b[1, i], sl, q))]
        assert lhs == negacyclic_mul(ma, mb, q)


def _ks_error(params, keys, d, u, sprime_signed):
    return max(abs(e) for e in _ks_errors(params, keys, d, u, sprime_signed))


def _ks_errors(params, keys, d, u, sprime_signed):
    """Centred CRT of u0 + u1 s - d s' over the active Q limbs (Python schoolbook)."""
    nl = d.shape[0]
    N = params.N
    rows = []
    for i in range(nl):
        q = params.q[i]
        sl = [int(x) % q for x in keys.s]
        spl = [int(x) % q for x in sprime_signed]
        t1 = negacyclic_mul(u[1, i], sl, q)
        t2 = negacyclic_mul(d[i], spl, q)
        rows.append([(int(u[0, i, k]) + t1[k] - t2[k]) % q for k in range(N)])
    errs = []
    for k in range(N):
        x, M = crt([rows[i][k] for i in range(nl)], list(params.q[:nl]))
        errs.append(centered(x, M))
    return errs


@pytest.mark.parametrize("alpha,n_q,n_p,nl", [(1, 4, 1, 4), (1, 4, 1, 2), (2, 6, 2, 6), (2, 6, 2, 5), (3, 6, 3, 4)])
def test_keyswitch_decrypts_to_target_secret(alpha, n_q, n_p, nl):
    params = ckks.Params(log_n=7, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=1)
    keys = ckks.Keys(params, 42)
    rng = np.random.default_rng(alpha + nl)
    d = _rand_limbs(rng, params.q[:nl], params.N)
    # relinearisation key: s' = s^2 (as an integer polynomial)
    s2 = negacyclic_mul(list(keys.s), list(keys.s))
    u = ckks.keyswitch(params, d, keys.relin)
    bound = n_p * (params.N + 1) + 4096
    assert _ks_error(params, keys, d, u, s2) <= bound
    # rotation key: s' = tau_g(s)
    g = pow(5, 3, 2 * params.N)
    u = ckks.keyswitch(params, d, keys.rot_key(g))
    assert _ks_error(params, keys, d, u, ckks.automorph_signed(keys.s, g)) <= bound
    # and a wrong target is far off (the pin has teeth)
    assert _ks_error(params, keys, d, u, s2) > 2 ** 60


@pytest.mark.parametrize("alpha,n_q,n_p", [(1, 4, 1), (2, 6, 2), (3, 6, 3)])
def test_keyswitch_error_is_zero_mean(alpha, n_q, n_p):
    """The key-switch error e = u0 + u1 s - d s' has no systematic part. A ModDown rounding error v with
    mean mu per coefficient would add -mu (1 + 1 * s) (1 = the all-ones polynomial, * the negacyclic
    product); the projection of e on that direction must stay within a few standard deviations."""
    params = ckks.Params(log_n=8, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=1)
    keys = ckks.Keys(params, 42)
    N = params.N
    g = pow(5, 7, 2 * N)
    target = ckks.automorph_signed(keys.s, g)
    bias = [1 + x for x in negacyclic_mul([1] * N, list(keys.s))]
    norm = sum(x * x for x in bias) ** 0.5
    proj, sq, cnt, trials = 0.0, 0, 0, 6
    for trial in range(trials):
        d = _rand_limbs(np.random.default_rng(100 + trial), params.q, N)
        u = ckks.keyswitch(params, d, keys.rot_key(g))
        errs = _ks_errors(params, keys, d, u, target)
        proj += sum(e * b for e, b in zip(errs, bias)) / norm
        sq += sum(e * e for e in errs)
        cnt += len(errs)
    std = (sq / cnt) ** 0.5
    assert abs(proj) < 6 * std * trials ** 0.5, (proj, std)


@pytest.fixture(scope="module")
def small():
    params = ckks.Params(log_n=10, n_q=5, n_p=2, alpha=2, rot_digits=2)
    keys = ckks.Keys(params, 42)
    return params, keys


def _enc(params, keys, z, scale, seed=43):
    return ckks.encrypt(params, keys, ckks.encode(z, scale, params.N), seed, 0, scale)


def test_encrypt_decrypt(small):
    params, keys = small
    z = np.random.default_rng(1).uniform(-1, 1, params.S)
    ct = _enc(params, keys, z, params.delta_a)
    out = ckks.decrypt_decode(params, keys, ct, np.arange(params.S))
    assert np.abs(out - z).max() < 1e-7


@pytest.mark.parametrize("r", [0, 1, 3, 127, 128, 129, 300, 511])
def test_rotate_decrypts_to_left_rotation(small, r):
    params, keys = small
    z = np.random.default_rng(2).uniform(-1, 1, params.S)
    ct = _enc(params, keys, z, params.delta_a)
    out = ckks.decrypt_decode(params, keys, ckks.rotate(params, keys, ct, r), np.arange(params.S))
    assert np.abs(out - np.roll(z, -r)).max() < 1e-6


def test_rotation_steps_decomposition(small):
    params, _ = small
    b = params.rot_step_bits()
    assert b == 5  # S = 2^9, two digits
    for r in range(0, 3 * params.S):
        steps = ckks.rotation_steps(params, r)
        assert sum(steps) % params.S == r % params.S
        assert len(steps) <= params.rot_digits
        for st in steps:
            t = 0
            while st % (1 << (b * (t + 1))) == 0:
                t += 1
            assert 0 < st >> (b * t) < (1 << b)


def test_mult_relin_rescale(small):
    params, keys = small
    rng = np.random.default_rng(3)
    za, zb = rng.uniform(-1, 1, params.S), rng.uniform(-1, 1, params.S)
    a = _enc(params, keys, za, params.delta_a, 43)
    b = _enc(params, keys, zb, params.delta_b, 44)
    d = ckks.rescale(params, ckks.mult_relin(params, keys, a, b))
    assert d.nl == params.n_q - 1
    assert d.scale == params.delta_a  # B at exactly q_top
    out = ckks.decrypt_decode(params, keys, d, np.arange(params.S))
    assert np.abs(out - za * zb).max() < 1e-7


def test_mask_isolates_one_slot(small):
    params, keys = small
    rng = np.random.default_rng(4)
    za, zb = rng.uniform(-1, 1, params.S), rng.uniform(-1, 1, params.S)
    d = ckks.rescale(params, ckks.mult_relin(params, keys, _enc(params, keys, za, params.delta_a, 43),
                                             _enc(params, keys, zb, params.delta_b, 44)))
    p = 37
    m = ckks.mul_plain(params, d, ckks.mask(params, p), params.delta_mask)
    m = ckks.rescale(params, m)
    assert m.scale == params.delta_out
    out = ckks.decrypt_decode(params, keys, m, np.arange(params.S))
    ref = np.zeros(params.S)
    ref[p] = za[p] * zb[p]
    assert np.abs(out - ref).max() < 1e-7


def test_automorph_coefficient_definition():
    params = ckks.Params(log_n=4, n_q=2, n_p=1, alpha=1, rot_digits=1)
    N = params.N
    rng = np.random.default_rng(6)
    a = _rand_limbs(rng, params.q, N)[None].copy()
    for g in [3, 5, 25, 2 * N - 1]:
        out = ckks.automorph(params, ckks.Ct(a, 1.0), g).data[0]
        for i, q in enumerate(params.q):
            ref = [0] * N
            for k in range(N):
                e = k * g
                sign = -1 if (e // N) % 2 else 1
                ref[e % N] = (sign * int(a[0, i, k])) % q
            assert [int(x) for x in out[i]] == ref
