"""GPU parity: the HIP library against the CPU oracle, bit-exact in the coefficient domain.

Each test prints the case it runs (flushed) before touching the GPU.
"""
import sys

import numpy as np
import pytest

from oracle import ckks, spmspm
from paper_2604_11659_amd import synth

pytestmark = pytest.mark.gpu

# (log_n, n_q, n_p, alpha, rot_digits): a small set with two-prime digits, two special primes and
# two-step rotations, and the single-prime-digit set of the 16x16 workload at a smaller ring.
OP_PARAMS = [(12, 5, 2, 2, 2), (13, 4, 1, 1, 1)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fhe():
    from paper_2604_11659_amd import fhe as f
    return f


_CACHE = {}


def _setup(fhe, prm):
    if prm not in _CACHE:
        log_n, n_q, n_p, alpha, D = prm
        _say(f"[setup] params {prm}")
        op = ckks.Params(log_n=log_n, n_q=n_q, n_p=n_p, alpha=alpha, rot_digits=D)
        ctx = fhe.Context(log_n, n_q, n_p, alpha, D)
        okeys = ckks.Keys(op, 42)
        sk = ctx.keygen(42)
        _CACHE[prm] = (op, okeys, ctx, sk)
    return _CACHE[prm]


def _rand_ct(op, nl, seed, ncomp=2):
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([rng.integers(0, op.q[i], op.N, dtype=np.uint64) for i in range(nl)])
                     for _ in range(ncomp)])


@pytest.mark.parametrize("prm", OP_PARAMS)
def test_primes_match(fhe, prm):
    op, _, ctx, _ = _setup(fhe, prm)
    assert ctx.primes == list(op.q) + list(op.p)


@pytest.mark.parametrize("prm", OP_PARAMS)
def test_ntt_roundtrip_and_add(fhe, prm):
    op, _, ctx, _ = _setup(fhe, prm)
    _say(f"[ntt/add] {prm}")
    a, b = _rand_ct(op, op.n_q, 1), _rand_ct(op, op.n_q, 2)
    ca, cb = ctx.ct_import(a, 1.0), ctx.ct_import(b, 1.0)
    assert (ctx.ct_export(ca) == a).all()
    got = ctx.ct_export(ctx.ct_add(ca, cb))
    ref = ckks.add(op, ckks.Ct(a, 1.0), ckks.Ct(b, 1.0)).data
    assert (got == ref).all()


@pytest.mark.parametrize("prm", OP_PARAMS)
@pytest.mark.parametrize("ncomp", [2, 3])
def test_rescale_parity(fhe, prm, ncomp):
    op, _, ctx, _ = _setup(fhe, prm)
    for nl in range(2, op.n_q + 1):
        _say(f"[rescale] {prm} ncomp={ncomp} nl={nl}")
        a = _rand_ct(op, nl, 10 + nl, ncomp)
        got = ctx.ct_export(ctx.ct_rescale(ctx.ct_import(a, 1.0)))
        ref = ckks.rescale(op, ckks.Ct(a, 1.0)).data
        assert (got == ref).all(), f"nl={nl}"


@pytest.mark.parametrize("prm", OP_PARAMS)
def test_mult_relin_parity(fhe, prm):
    op, okeys, ctx, _ = _setup(fhe, prm)
    for nl in sorted({op.n_q, 2, op.n_q - 1}):
        _say(f"[mult_relin] {prm} nl={nl}")
        a, b = _rand_ct(op, nl, 20 + nl), _rand_ct(op, nl, 30 + nl)
        got = ctx.ct_export(ctx.ct_mult_relin(ctx.ct_import(a, 1.0), ctx.ct_import(b, 1.0)))
        ref = ckks.mult_relin(op, okeys, ckks.Ct(a, 1.0), ckks.Ct(b, 1.0)).data
        assert (got == ref).all(), f"nl={nl}"


@pytest.mark.parametrize("prm", OP_PARAMS)
def test_rotate_parity(fhe, prm):
    op, okeys, ctx, sk = _setup(fhe, prm)
    amounts = [1, 5, op.S - 1, 3 * (1 << op.rot_step_bits()) + 7, 0]
    if op.rot_digits == 1:
        ctx.keygen_rotations(sk, amounts)
    for nl in sorted({op.n_q, op.n_q - 2}):
        a = _rand_ct(op, nl, 40 + nl)
        ca = ctx.ct_import(a, 1.0)
        for r in amounts:
            _say(f"[rotate] {prm} nl={nl} r={r}")
            got = ctx.ct_export(ctx.ct_rotate(ca, r))
            ref = ckks.rotate(op, okeys, ckks.Ct(a, 1.0), r).data
            assert (got == ref).all(), f"nl={nl} r={r}"


@pytest.mark.parametrize("prm", OP_PARAMS)
def test_mask_parity(fhe, prm):
    op, _, ctx, _ = _setup(fhe, prm)
    nl = op.n_q - 1
    a = _rand_ct(op, nl, 50)
    ca = ctx.ct_import(a, 1.0)
    for slot in [0, 1, 77, op.S - 1]:
        _say(f"[mask] {prm} slot={slot}")
        got = ctx.ct_export(ctx.ct_mask(ca, slot))
        ref = ckks.mul_plain(op, ckks.Ct(a, 1.0), ckks.mask(op, slot), op.delta_mask).data
        assert (got == ref).all(), f"slot={slot}"


@pytest.mark.parametrize("prm", OP_PARAMS)
def test_encryption_parity(fhe, prm):
    """Encoding, sampling and encryption reproduce the oracle's ciphertexts bit for bit."""
    op, okeys, ctx, sk = _setup(fhe, prm)
    _say(f"[encrypt] {prm}")
    a = synth.sparse_dense(6, 9, 0.5, "uniform", 5, 6)
    ip, ix, va = synth.to_csr(a)
    A = ctx.encrypt_csr(sk, 6, 9, ip, ix, va, seed=43)
    OA = spmspm.encrypt_csr(op, okeys, 6, 9, ip, ix, va, seed=43)
    assert (ctx.export(A, 0) == OA.chunks[0].data).all()
    b = synth.sparse_dense(9, 4, 0.5, "halfnormal", 7, 8)
    ip, ix, vb = synth.to_csc(b)
    B = ctx.encrypt_csc(sk, 9, 4, ip, ix, vb, seed=44)
    OB = spmspm.encrypt_csc(op, okeys, 9, 4, ip, ix, vb, seed=44)
    assert (ctx.export(B, 0) == OB.chunks[0].data).all()
    dec = ctx.decrypt_decode(sk, A)[: len(va)]
    assert np.abs(dec - va).max() < 1e-6


def _matmul_case(fhe, prm, m, k, n, sp_a, sp_b, seeds, workers=1):
    op, okeys, ctx, sk = _setup(fhe, prm)
    a = synth.sparse_dense(m, k, sp_a, "uniform", seeds[0], seeds[2])
    b = synth.sparse_dense(k, n, sp_b, "uniform", seeds[1], seeds[3])
    ipa, ixa, va = synth.to_csr(a)
    ipb, ixb, vb = synth.to_csc(b)
    A = ctx.encrypt_csr(sk, m, k, ipa, ixa, va, seed=43)
    B = ctx.encrypt_csc(sk, k, n, ipb, ixb, vb, seed=44)
    if op.rot_digits == 1:
        ctx.keygen_rotations(sk, ctx.plan_rotations(A, B))
    _say(f"[spmspm] {prm} {m}x{k}x{n} gpu")
    C = ctx.spmspm(A, B)
    OA = spmspm.encrypt_csr(op, okeys, m, k, ipa, ixa, va, seed=43)
    OB = spmspm.encrypt_csc(op, okeys, k, n, ipb, ixb, vb, seed=44)
    _say(f"[spmspm] {prm} {m}x{k}x{n} oracle")
    ref = spmspm.spmspm(op, okeys, OA, OB, workers=workers)
    for c, rct in enumerate(ref):
        assert (ctx.export(C, c) == rct.data).all(), f"chunk {c}"
    dec = ctx.decrypt_decode(sk, C)
    assert np.abs(dec - a @ b).max() < 1e-5
    return ctx, A, B


def test_spmspm_parity_small(fhe):
    _matmul_case(fhe, OP_PARAMS[0], 5, 6, 7, 0.5, 0.5, (0, 1, 2, 3))


def test_spmspm_parity_single_digit(fhe):
    _matmul_case(fhe, OP_PARAMS[1], 6, 5, 4, 0.4, 0.6, (4, 5, 6, 7))


def test_released_result_block_reused(fhe):
    """A released result's device block is kept by its context and handed to the next result of the
    same size: a product of other values written into it equals the oracle's (the block is cleared
    before accumulation), and so does the first product recomputed into a kept block."""
    prm = OP_PARAMS[0]
    op, okeys, ctx, sk = _setup(fhe, prm)
    m, k, n = 5, 6, 7
    cases = []
    for t, seeds in enumerate(((30, 31, 32, 33), (34, 35, 36, 37))):
        a = synth.sparse_dense(m, k, 0.5, "uniform", seeds[0], seeds[2])
        b = synth.sparse_dense(k, n, 0.5, "uniform", seeds[1], seeds[3])
        ipa, ixa, va = synth.to_csr(a)
        ipb, ixb, vb = synth.to_csc(b)
        A = ctx.encrypt_csr(sk, m, k, ipa, ixa, va, seed=43 + 2 * t)
        B = ctx.encrypt_csc(sk, k, n, ipb, ixb, vb, seed=44 + 2 * t)
        _say(f"[reuse] case {t} oracle")
        ref = spmspm.spmspm(op, okeys, spmspm.encrypt_csr(op, okeys, m, k, ipa, ixa, va, seed=43 + 2 * t),
                            spmspm.encrypt_csc(op, okeys, k, n, ipb, ixb, vb, seed=44 + 2 * t))
        cases.append((A, B, ref))
    for t in (0, 1, 0):
        A, B, ref = cases[t]
        _say(f"[reuse] case {t} gpu")
        C = ctx.spmspm(A, B)
        for c, rct in enumerate(ref):
            assert (ctx.export(C, c) == rct.data).all(), f"case {t} chunk {c}"
        C.close()  # its block goes back to the context for the next result of this size


def test_unfused_split_fallback(fhe, monkeypatch):
    """An NTT split outside the fused column kernels' compiled ones (k1 = 5 at N = 2^12) runs the
    unfused ModUp / ModDown / rescale sequence and row-phase kernels with run-time stage counts;
    the matmul stays bit-exact against the oracle."""
    prm = OP_PARAMS[0]
    op, okeys, _, _ = _setup(fhe, prm)
    monkeypatch.setenv("FHE_NTT_K1", "5")
    ctx = fhe.Context(*prm)
    monkeypatch.delenv("FHE_NTT_K1")
    sk = ctx.keygen(42)
    m, k, n = 4, 5, 6
    a = synth.sparse_dense(m, k, 0.4, "uniform", 21, 23)
    b = synth.sparse_dense(k, n, 0.4, "uniform", 22, 24)
    ipa, ixa, va = synth.to_csr(a)
    ipb, ixb, vb = synth.to_csc(b)
    _say("[fallback] k1=5 gpu")
    C = ctx.spmspm(ctx.encrypt_csr(sk, m, k, ipa, ixa, va, seed=43), ctx.encrypt_csc(sk, k, n, ipb, ixb, vb, seed=44))
    _say("[fallback] k1=5 oracle")
    ref = spmspm.spmspm(op, okeys, spmspm.encrypt_csr(op, okeys, m, k, ipa, ixa, va, seed=43),
                        spmspm.encrypt_csc(op, okeys, k, n, ipb, ixb, vb, seed=44))
    for c, rct in enumerate(ref):
        assert (ctx.export(C, c) == rct.data).all(), f"chunk {c}"


def test_autotune_keeps_results_bit_exact(fhe):
    """The autotuner tries every admissible NTT split and keeps the fastest; the transform is the same
    for all of them, so a matmul afterwards is still bit-exact against the oracle."""
    prm = OP_PARAMS[0]
    op, okeys, _, _ = _setup(fhe, prm)
    ctx = fhe.Context(*prm)
    sk = ctx.keygen(42)
    _say("[autotune] synthetic key switches")
    rep = ctx.autotune(batch=4)
    log_n = prm[0]
    splits = range(max(1, log_n - 9), min(9, log_n - 1) + 1)
    assert set(rep["tried"]) == {f"{k1}/{rows}" for k1 in splits for rows in (512, 256)}
    assert f"{rep['k1']}/{rep['row_threads']}" in rep["tried"] and rep["ms"] > 0
    m, k, n = 3, 4, 5
    a = synth.sparse_dense(m, k, 0.3, "uniform", 31, 33)
    b = synth.sparse_dense(k, n, 0.3, "uniform", 32, 34)
    ipa, ixa, va = synth.to_csr(a)
    ipb, ixb, vb = synth.to_csc(b)
    A = ctx.encrypt_csr(sk, m, k, ipa, ixa, va, seed=43)
    B = ctx.encrypt_csc(sk, k, n, ipb, ixb, vb, seed=44)
    _say("[autotune] plan prefix")
    rep2 = ctx.autotune(A, B, pairs=6)
    assert rep2["mode"] == "plan" and f"{rep2['k1']}/{rep2['row_threads']}" in rep2["tried"] and rep2["ms"] > 0
    _say(f"[autotune] k1={rep2['k1']} rows={rep2['row_threads']} matmul")
    C = ctx.spmspm(A, B)
    ref = spmspm.spmspm(op, okeys, spmspm.encrypt_csr(op, okeys, m, k, ipa, ixa, va, seed=43),
                        spmspm.encrypt_csc(op, okeys, k, n, ipb, ixb, vb, seed=44))
    for c, rct in enumerate(ref):
        assert (ctx.export(C, c) == rct.data).all(), f"chunk {c}"


def test_row_shape_256_matmul_bit_exact(fhe, monkeypatch):
    """Row-phase workgroups of 256 threads x 16 elements (FHE_ROWS_NT=256, one of the autotuner's
    candidates: row transforms, the combine and the rescale rows in 4-stage rounds) give the same
    matmul, bit-exact against the oracle."""
    prm = OP_PARAMS[0]
    op, okeys, _, _ = _setup(fhe, prm)
    monkeypatch.setenv("FHE_ROWS_NT", "256")
    ctx = fhe.Context(*prm)
    monkeypatch.delenv("FHE_ROWS_NT")
    sk = ctx.keygen(42)
    m, k, n = 5, 4, 6
    a = synth.sparse_dense(m, k, 0.3, "uniform", 41, 43)
    b = synth.sparse_dense(k, n, 0.3, "uniform", 42, 44)
    ipa, ixa, va = synth.to_csr(a)
    ipb, ixb, vb = synth.to_csc(b)
    _say("[rows 256] matmul gpu")
    C = ctx.spmspm(ctx.encrypt_csr(sk, m, k, ipa, ixa, va, seed=43), ctx.encrypt_csc(sk, k, n, ipb, ixb, vb, seed=44))
    _say("[rows 256] matmul oracle")
    ref = spmspm.spmspm(op, okeys, spmspm.encrypt_csr(op, okeys, m, k, ipa, ixa, va, seed=43),
                        spmspm.encrypt_csc(op, okeys, k, n, ipb, ixb, vb, seed=44))
    for c, rct in enumerate(ref):
        assert (ctx.export(C, c) == rct.data).all(), f"chunk {c}"


@pytest.mark.parametrize("log_n", [15, 16])
def test_row_shape_256_rows_of_512_bit_exact(fhe, monkeypatch, log_n):
    """The 256-thread row shape on rows of 2^9 elements (N >= 2^15): mult + relinearise, a rotation
    and a rescale bit-exact against the oracle."""
    prm = (log_n, 3, 1, 1, 1)
    op, okeys, _, _ = _setup(fhe, prm)
    monkeypatch.setenv("FHE_ROWS_NT", "256")
    ctx = fhe.Context(*prm)
    monkeypatch.delenv("FHE_ROWS_NT")
    sk = ctx.keygen(42)
    _say(f"[rows 256] {prm}")
    a, b = _rand_ct(op, 3, 80 + log_n), _rand_ct(op, 3, 90 + log_n)
    ca, cb = ctx.ct_import(a, 1.0), ctx.ct_import(b, 1.0)
    got = ctx.ct_export(ctx.ct_mult_relin(ca, cb))
    assert (got == ckks.mult_relin(op, okeys, ckks.Ct(a, 1.0), ckks.Ct(b, 1.0)).data).all()
    r = op.S // 5 + 3
    ctx.keygen_rotations(sk, [r])
    got = ctx.ct_export(ctx.ct_rotate(ca, r))
    assert (got == ckks.rotate(op, okeys, ckks.Ct(a, 1.0), r).data).all()
    got = ctx.ct_export(ctx.ct_rescale(ca))
    assert (got == ckks.rescale(op, ckks.Ct(a, 1.0)).data).all()


@pytest.mark.parametrize("log_n", [14, 15, 16, 17])
def test_ring_size_sweep(fhe, log_n):
    """Every supported ring size (two-phase NTT with 2-3 register rounds per phase, FP64 and integer
    arithmetic): mult + relinearise and one rotation bit-exact against the oracle."""
    prm = (log_n, 3, 1, 1, 1)
    op, okeys, ctx, sk = _setup(fhe, prm)
    _say(f"[sweep] {prm}")
    a, b = _rand_ct(op, 3, 60 + log_n), _rand_ct(op, 3, 70 + log_n)
    ca, cb = ctx.ct_import(a, 1.0), ctx.ct_import(b, 1.0)
    assert (ctx.ct_export(ca) == a).all()
    got = ctx.ct_export(ctx.ct_mult_relin(ca, cb))
    assert (got == ckks.mult_relin(op, okeys, ckks.Ct(a, 1.0), ckks.Ct(b, 1.0)).data).all()
    r = op.S // 3 + 1
    ctx.keygen_rotations(sk, [r])
    got = ctx.ct_export(ctx.ct_rotate(ca, r))
    assert (got == ckks.rotate(op, okeys, ckks.Ct(a, 1.0), r).data).all()


def test_spmspm_batch_matches_individual_and_oracle(fhe):
    """Uneven matmuls merged into one launch stream give bit-identical results to one-at-a-time runs."""
    op, okeys, ctx, sk = _setup(fhe, OP_PARAMS[0])
    shapes = [(3, 4, 5, 0.5, 0.5), (6, 6, 2, 0.3, 0.7), (1, 5, 1, 0.0, 0.0), (4, 4, 4, 1.0, 0.2), (5, 3, 6, 0.6, 0.4)]
    As, Bs, dense = [], [], []
    for t, (m, k, n, sa, sb) in enumerate(shapes):
        a = synth.sparse_dense(m, k, sa, "uniform", 100 + t, 200 + t)
        b = synth.sparse_dense(k, n, sb, "uniform", 300 + t, 400 + t)
        As.append(ctx.encrypt_csr(sk, m, k, *synth.to_csr(a), seed=43 + 10 * t))
        Bs.append(ctx.encrypt_csc(sk, k, n, *synth.to_csc(b), seed=44 + 10 * t))
        dense.append((a, b))
    _say("[batch] merged")
    Cb = ctx.spmspm_batch(As, Bs)
    for t in range(len(shapes)):
        _say(f"[batch] single {t}")
        Ci = ctx.spmspm(As[t], Bs[t])
        info = Ci.info()
        for c in range(info["chunks"]):
            assert (ctx.export(Cb[t], c) == ctx.export(Ci, c)).all(), (t, c)
        a, b = dense[t]
        assert np.abs(ctx.decrypt_decode(sk, Cb[t]) - a @ b).max() < 1e-5
    # one of them against the oracle as well
    a, b = dense[0]
    m, k, n = shapes[0][:3]
    OA = spmspm.encrypt_csr(op, okeys, m, k, *synth.to_csr(a), seed=43)
    OB = spmspm.encrypt_csc(op, okeys, k, n, *synth.to_csc(b), seed=44)
    ref = spmspm.spmspm(op, okeys, OA, OB)
    assert (ctx.export(Cb[0], 0) == ref[0].data).all()


def test_spmspm_batch_pair_ranges_match_single_ranges(fhe):
    """Batched form restricted to per-matmul pair ranges equals fhe_spmspm_pairs on the same ranges."""
    op, okeys, ctx, sk = _setup(fhe, OP_PARAMS[0])
    shapes = [(5, 6, 4, 0.3, 0.4), (4, 7, 5, 0.5, 0.2), (6, 3, 6, 0.2, 0.5)]
    As, Bs = [], []
    for t, (m, k, n, sa, sb) in enumerate(shapes):
        a = synth.sparse_dense(m, k, sa, "uniform", 150 + t, 250 + t)
        b = synth.sparse_dense(k, n, sb, "uniform", 350 + t, 450 + t)
        As.append(ctx.encrypt_csr(sk, m, k, *synth.to_csr(a), seed=73 + 10 * t))
        Bs.append(ctx.encrypt_csc(sk, k, n, *synth.to_csc(b), seed=74 + 10 * t))
    F = [ctx.plan_stats(A, B).matched_pairs for A, B in zip(As, Bs)]
    ranges = [(0, F[0] // 2), (F[1] // 3, F[1]), (2, 2)]  # prefix, suffix, empty
    _say(f"[batch-ranges] F={F} ranges={ranges}")
    Cb = ctx.spmspm_batch(As, Bs, pair_ranges=ranges)
    for t, (lo, hi) in enumerate(ranges):
        Ci = ctx.spmspm_pairs(As[t], Bs[t], lo, hi)
        for c in range(Ci.info()["chunks"]):
            assert (ctx.export(Cb[t], c) == ctx.export(Ci, c)).all(), (t, c)
    assert (ctx.export(Cb[2], 0) == 0).all()
    with pytest.raises(fhe.FheError):
        ctx.spmspm_batch(As[:1], Bs[:1], pair_ranges=[(3, 1)])


def test_spmspm_full_sparsity_is_zero(fhe):
    op, _, ctx, sk = _setup(fhe, OP_PARAMS[0])
    z = np.zeros((4, 4))
    ip, ix, v = synth.to_csr(z)
    A = ctx.encrypt_csr(sk, 4, 4, ip, ix, v, seed=43)
    B = ctx.encrypt_csc(sk, 4, 4, ip, ix, v, seed=44)
    C = ctx.spmspm(A, B)
    assert (ctx.export(C, 0) == 0).all()
    assert (ctx.decrypt_decode(sk, C) == 0).all()
