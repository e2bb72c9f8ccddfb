"""The no-allocation rotation (fhe_ct_rotate_into, scratch in a static device array) against the
allocating rotation (fhe_ct_rotate) on the same inputs: bit-identical on two calls in a row, the
second with a smaller input (fewer limbs, another amount) and in place, plus its error paths. The
first call is also checked against the oracle's rotation."""
import sys

import numpy as np
import pytest

from oracle import ckks

pytestmark = pytest.mark.gpu

# (log_n, n_q, n_p, alpha, rotation digits): two-prime digits, two special primes, two-step rotations
PRM = (13, 6, 2, 2, 2)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rand(primes, N, nl, seed):
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([rng.integers(0, primes[i], N, dtype=np.uint64) for i in range(nl)])
                     for _ in range(2)])


def test_rotate_into_matches_rotate_on_two_calls():
    from paper_2604_11659_amd import fhe
    log_n, n_q, n_p, alpha, D = PRM
    _say(f"[no-alloc] context {PRM}")
    ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
    sk = ctx.keygen(42)
    primes, N, S = ctx.primes, 1 << log_n, 1 << (log_n - 1)
    # call 1: top level, a rotation of two digit steps, into an output holding other values
    r1 = S - 1
    a = _rand(primes, N, n_q, 1)
    ca = ctx.ct_import(a, 1.0)
    _say(f"[no-alloc] call 1: {n_q} limbs, r={r1}")
    ref1 = ctx.ct_export(ctx.ct_rotate(ca, r1))
    out1 = ctx.ct_import(_rand(primes, N, n_q, 2), 3.0)
    ctx.ct_rotate_into(ca, r1, out1)
    got1 = ctx.ct_export(out1)
    assert (got1 == ref1).all()
    assert out1.info()["scale"] == 1.0
    op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
    okeys = ckks.Keys(op, 42)
    assert (got1 == ckks.rotate(op, okeys, ckks.Ct(a, 1.0), r1).data).all()
    # call 2: a smaller input (three limbs), one digit step; then the same in place
    r2 = 5
    b = _rand(primes, N, 3, 3)
    cb = ctx.ct_import(b, 1.0)
    _say(f"[no-alloc] call 2: 3 limbs, r={r2}")
    ref2 = ctx.ct_export(ctx.ct_rotate(cb, r2))
    out2 = ctx.ct_import(_rand(primes, N, 3, 4), 1.0)
    ctx.ct_rotate_into(cb, r2, out2)
    assert (ctx.ct_export(out2) == ref2).all()
    _say("[no-alloc] call 3: in place, 3 limbs, two steps")
    ref3 = ctx.ct_export(ctx.ct_rotate(cb, r1))
    ctx.ct_rotate_into(cb, r1, cb)
    assert (ctx.ct_export(cb) == ref3).all()
    _say("[no-alloc] call 4: rotation by 0 (copy)")
    ctx.ct_rotate_into(ca, 0, out1)
    assert (ctx.ct_export(out1) == a).all()
    ctx.close()


def test_rotate_into_error_paths():
    from paper_2604_11659_amd import fhe
    log_n, n_q, n_p, alpha, D = PRM
    _say(f"[no-alloc] errors, context {PRM}")
    ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
    primes, N = ctx.primes, 1 << log_n
    ca = ctx.ct_import(_rand(primes, N, n_q, 5), 1.0)
    small = ctx.ct_import(_rand(primes, N, 3, 6), 1.0)
    with pytest.raises(fhe.FheError) as ei:
        ctx.ct_rotate_into(ca, 1, small)
    assert ei.value.code == -2  # FHE_ESHAPE: limb counts differ
    with pytest.raises(fhe.FheError) as ei:
        ctx.ct_rotate_into(ca, 1, ca)
    assert ei.value.code == -4  # FHE_EKEY: no keys generated in this context
    ctx.close()
    # N = 2^16 with 30 Q primes: a top-level rotation needs more scratch than the array holds; the
    # check comes before the key lookup, so no keys are needed to see it
    _say("[no-alloc] errors, N=2^16 with 30 Q primes")
    big = fhe.Context(16, 30, 3, 3, 3)
    cbig = big.ct_import(np.zeros((2, 30, 1 << 16), np.uint64), 1.0)
    with pytest.raises(fhe.FheError) as ei:
        big.ct_rotate_into(cbig, 1, cbig)
    assert ei.value.code == -5 and "scratch" in str(ei.value)
    big.close()
