"""GPU parity of the paper's evaluation baselines (Section 4) on the same executor, 8 x 8 x 8:
naive dense (operands store every entry, every product runs) and naive sparse (a product is skipped
only where both values are zero), every result limb bit-exact against the oracle's plan on the same
seeded keys, noise and operands."""
import sys

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu
WORKERS = 8
PRM = (12, 4, 1, 1, 2)  # log_n, n_q, n_p, alpha, rotation digits


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    from paper_2604_11659_amd import fhe
    log_n, n_q, n_p, alpha, D = PRM
    ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
    sk = ctx.keygen(42)
    op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
    keys = ckks.Keys(op, 42)
    a = synth.sparse_dense(8, 8, 0.5, "uniform", 21, 22)
    b = synth.sparse_dense(8, 8, 0.5, "halfnormal", 23, 24)
    A = ctx.encrypt_csr(sk, 8, 8, *synth.full_csr(a), seed=43)
    B = ctx.encrypt_csc(sk, 8, 8, *synth.full_csc(b), seed=44)
    OA = spmspm.encrypt_csr(op, keys, 8, 8, *synth.full_csr(a), seed=43)
    OB = spmspm.encrypt_csc(op, keys, 8, 8, *synth.full_csc(b), seed=44)
    yield fhe, ctx, sk, a, b, A, B, op, keys, OA, OB
    ctx.close()


@pytest.mark.timeout(600)
def test_naive_dense_8x8_bit_exact(env):
    fhe, ctx, sk, a, b, A, B, op, keys, OA, OB = env
    st = ctx.plan_stats(A, B)
    assert st.matched_pairs == 8 * 8 * 8
    _say("[naive] dense gpu")
    C = ctx.spmspm(A, B)
    _say("[naive] dense oracle")
    ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS)
    assert (ctx.export(C, 0) == ref[0].data).all()
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    C.close()


@pytest.mark.timeout(600)
def test_naive_sparse_8x8_bit_exact(env):
    fhe, ctx, sk, a, b, A, B, op, keys, OA, OB = env
    za, zb = synth.stored_nonzero_csr(a), synth.stored_nonzero_csc(b)
    pairs = spmspm.naive_sparse_pairs(8, 8, OA.indptr, OA.indices, OB.indptr, OB.indices, za, zb)
    ak, bk = (a != 0).sum(axis=0), (b != 0).sum(axis=1)
    assert len(pairs) == int(np.sum(8 * ak + 8 * bk - ak * bk))
    assert ctx.plan_stats(A, B, nonzero_a=za, nonzero_b=zb).matched_pairs == len(pairs)
    _say(f"[naive] sparse gpu ({len(pairs)} of 512 products)")
    C = ctx.spmspm_naive_sparse(A, B, za, zb)
    _say("[naive] sparse oracle")
    ref = spmspm.spmspm(op, keys, OA, OB, workers=WORKERS, pairs=pairs)
    assert (ctx.export(C, 0) == ref[0].data).all()
    assert np.abs(ctx.decrypt_decode(sk, C) - a @ b).max() < 1e-5
    C.close()
    # every flag set: the naive dense plan, bit for bit
    ones_a, ones_b = np.ones_like(za), np.ones_like(zb)
    Cs, Cd = ctx.spmspm_naive_sparse(A, B, ones_a, ones_b), ctx.spmspm(A, B)
    assert (ctx.export(Cs, 0) == ctx.export(Cd, 0)).all()
    # a missing flag array is refused
    with pytest.raises(fhe.FheError) as ei:
        fhe._check(fhe._lib.fhe_spmspm_naive_sparse(ctx._ptr, A._ptr, B._ptr, None, None, None,
                                                    fhe.ctypes.byref(fhe.c_vp())))
    assert ei.value.code == -1
