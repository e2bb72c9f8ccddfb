"""Oracle for the paper's sparse x sparse ciphertext matmul (test infrastructure only).

Algorithm 1 (CSR x CSC traversal with rotation-minimising alignment) and
Algorithm 2 (per matched pair: EvalMult, Relinearize, Rescale, one-hot mask,
Rescale, EvalRotate to the target slot, EvalAdd) are followed step by step for
every matched pair, with no sharing of work between pairs.

Readings where the paper is silent (listed in the design notes):
  * loops run i in [0, m), j in [0, n); ``size`` in the target index is n;
  * values of an operand longer than S = N/2 slots are packed into chunks of
    S consecutive values; a position splits into (chunk, local slot);
  * the result is packed row-major, chunked the same way, and each result
    chunk starts as the all-zero ciphertext two levels below the top;
  * rotations are cyclic over all S slots, a rotation by 0 is the identity,
    the Relinearize after the plaintext mask multiply is the identity.

A second, grouped form (``grouped=True``) follows the paper's aim of issuing as few
rotations as possible (Section 3.2, mitigating the overhead of rotations): the
Isolation step leaves each masked product in one slot, so products bound for the
same result chunk with the same target rotation can be added before a single
second rescale and a single rotation. Its ciphertext bits differ from the
per-pair form (fewer roundings and key switches); its decryption does not
beyond noise.
"""
from __future__ import annotations

import multiprocessing as mp
from dataclasses import dataclass

import numpy as np

from . import ckks
from .ckks import Ct, Keys, Params


@dataclass
class EncSparse:
    """An encrypted sparse matrix: public pattern, encrypted values in slot chunks."""
    rows: int
    cols: int
    indptr: np.ndarray
    indices: np.ndarray
    chunks: list


def _encrypt_values(params: Params, keys: Keys, values: np.ndarray, seed: int, scale: float) -> list:
    S = params.S
    out = []
    nchunks = max(1, -(-len(values) // S))
    for c in range(nchunks):
        z = values[c * S:(c + 1) * S]
        m = ckks.encode(z, scale, params.N)
        out.append(ckks.encrypt(params, keys, m, seed, c, scale))
    return out


def encrypt_csr(params: Params, keys: Keys, rows, cols, indptr, indices, values, seed: int) -> EncSparse:
    """Left operand in CSR, values encoded at 2^log_delta."""
    values = np.asarray(values, dtype=np.float64)
    return EncSparse(rows, cols, np.asarray(indptr), np.asarray(indices),
                     _encrypt_values(params, keys, values, seed, params.delta_a))


def encrypt_csc(params: Params, keys: Keys, rows, cols, indptr, indices, values, seed: int) -> EncSparse:
    """Right operand in CSC, values encoded at exactly q_top."""
    values = np.asarray(values, dtype=np.float64)
    return EncSparse(rows, cols, np.asarray(indptr), np.asarray(indices),
                     _encrypt_values(params, keys, values, seed, params.delta_b))


def matched_pairs(m: int, n: int, indptr_a, indices_a, indptr_b, indices_b) -> list:
    """Algorithm 1's traversal: for every (row i, column j), merge the column ids of
    row i of A with the row ids of column j of B; every equal id is one matched
    pair (i, j, a_pos, b_pos), positions being indices into the value arrays."""
    pairs = []
    for i in range(m):
        for j in range(n):
            a_pos, a_end = int(indptr_a[i]), int(indptr_a[i + 1])
            b_pos, b_end = int(indptr_b[j]), int(indptr_b[j + 1])
            while a_pos < a_end and b_pos < b_end:
                a_col, b_row = int(indices_a[a_pos]), int(indices_b[b_pos])
                if a_col == b_row:
                    pairs.append((i, j, a_pos, b_pos))
                    a_pos += 1
                    b_pos += 1
                elif a_col < b_row:
                    a_pos += 1
                else:
                    b_pos += 1
    return pairs


def naive_sparse_pairs(m: int, n: int, indptr_a, indices_a, indptr_b, indices_b, nonzero_a, nonzero_b) -> list:
    """The naive sparse method of the paper's evaluation (Section 4, method (ii)): the multiplication
    stays element-wise over the stored entries, and a product is skipped only when BOTH of its values
    are zero. The operands store every entry they may multiply (for the method as evaluated, all m k
    and k n entries, zeros included); nonzero_a / nonzero_b flag the stored entries (packing order)
    whose value is nonzero, which is public. Returns the matched pairs of Algorithm 1's traversal over
    the stored patterns, less those whose two entries are both flagged zero, in traversal order."""
    return [pr for pr in matched_pairs(m, n, indptr_a, indices_a, indptr_b, indices_b)
            if nonzero_a[pr[2]] or nonzero_b[pr[3]]]


def alignment(params: Params, a_pos: int, b_pos: int):
    """(chunk of A, chunk of B, rotation of A, rotation of B, min local position).
    Only the operand whose value sits at the larger local slot is rotated, by the
    difference; equal slots need no rotation."""
    S = params.S
    ca, la = divmod(a_pos, S)
    cb, lb = divmod(b_pos, S)
    if la < lb:
        return ca, cb, 0, lb - la, la
    if lb < la:
        return ca, cb, la - lb, 0, lb
    return ca, cb, 0, 0, la


def target(params: Params, i: int, j: int, n: int, min_pos: int):
    """(result chunk, rotation amount) moving slot min_pos to slot (i n + j) mod S."""
    cr, lt = divmod(i * n + j, params.S)
    return cr, (min_pos - lt) % params.S


_HOIST = {"on": False}


def masked_product(params: Params, keys: Keys, A: EncSparse, B: EncSparse, a_pos: int, b_pos: int) -> Ct:
    """Algorithm 1's alignment, then Algorithm 2 up to the mask: EvalMult, Relinearize, Rescale and
    the product with the one-hot mask at min_pos (one level below the top, before the second rescale).
    With hoisting on (spmspm(..., hoist=True)) the alignment rotations use rotate_hoisted."""
    ca, cb, ra, rb, mn = alignment(params, a_pos, b_pos)
    vA, vB = A.chunks[ca], B.chunks[cb]
    rot = ckks.rotate_hoisted if _HOIST["on"] else ckks.rotate
    if rb:
        vB = rot(params, keys, vB, rb)
    if ra:
        vA = rot(params, keys, vA, ra)
    d = ckks.mult_relin(params, keys, vA, vB)
    d = ckks.rescale(params, d)
    return ckks.mul_plain(params, d, ckks.mask(params, mn), params.delta_mask)


def pair_contribution(params: Params, keys: Keys, A: EncSparse, B: EncSparse, i: int, j: int, a_pos: int,
                      b_pos: int) -> tuple:
    # Algorithm 2 for one matched pair: masked product, second rescale, target rotation
    d = masked_product(params, keys, A, B, a_pos, b_pos)
    d = ckks.rescale(params, d)
    mn = alignment(params, a_pos, b_pos)[4]
    cr, rot = target(params, i, j, B.cols, mn)
    d = ckks.rotate(params, keys, d, rot)
    return cr, d


def target_groups(params: Params, pairs: list, n: int) -> list:
    """Matched pairs grouped by (result chunk, target rotation), in order of first appearance:
    [((chunk, rot), [pairs...]), ...]. Within a group the isolated slots min_pos differ exactly when
    the targets differ (min_pos = (lt + rot) mod S), so the masked products of a group occupy
    distinct slots unless they belong to the same output entry, where they are meant to add up."""
    groups: dict = {}
    for pair in pairs:
        i, j, a_pos, b_pos = pair
        mn = alignment(params, a_pos, b_pos)[4]
        groups.setdefault(target(params, i, j, n, mn), []).append(pair)
    return list(groups.items())


def group_contribution(params: Params, keys: Keys, A: EncSparse, B: EncSparse, rot: int, members: list) -> Ct:
    """Grouped form of Algorithm 2's tail: the masked products of all pairs sharing (result chunk,
    target rotation) are added (exactly, mod q), then rescaled once and rotated once. Rotation and
    rescale act on the sum as on each term up to rounding, and the masks keep the terms in distinct
    slots, so the decrypted contribution is the same as the per-pair sequence's; the ciphertext bits
    are not (one rounding and one key switch per group instead of per pair)."""
    acc = None
    for (_, _, a_pos, b_pos) in members:
        d = masked_product(params, keys, A, B, a_pos, b_pos)
        acc = d if acc is None else ckks.add(params, acc, d)
    acc = ckks.rescale(params, acc)
    return ckks.rotate(params, keys, acc, rot)


def result_chunks(params: Params, m: int, n: int) -> int:
    return max(1, -(-(m * n) // params.S))


def digit_tree_sum(params, items: list, nres: int, rotate, add) -> list:
    """Sum of Rot_rot(x) over items (chunk, rot, x) per result chunk, sharing rotations digit by digit.

    A rotation by r = sum_t r_t 2^(b t) is the composition of its digit steps (t ascending, zero
    digits skipped, as for every rotation here). Level 0 rotates each x by its lowest digit and adds
    the results of equal (chunk, r >> b); level t rotates each partial sum by its digit t and adds
    those of equal (chunk, digits above t). After the last digit one sum per chunk is left.
    ``rotate(x, step)`` and ``add(x, y)`` are the ring operations (ciphertexts here; plaintext slot
    vectors in the tests). Returns [sum or None per chunk]."""
    b = params.rot_step_bits()
    low = (1 << b) - 1
    level = {}
    for (cr, rot, x) in items:
        if rot & low:
            x = rotate(x, rot & low)
        key = (cr, rot >> b)
        level[key] = x if key not in level else add(level[key], x)
    for t in range(1, params.rot_digits):
        nxt = {}
        for (cr, rest), x in sorted(level.items(), key=lambda kv: kv[0]):
            if rest & low:
                x = rotate(x, (rest & low) << (b * t))
            key = (cr, rest >> b)
            nxt[key] = x if key not in nxt else add(nxt[key], x)
        level = nxt
    res = [None] * nres
    for (cr, rest), x in level.items():
        assert rest == 0
        res[cr] = x
    return res


def digit_tree_level0(params: Params, keys: Keys, A: EncSparse, B: EncSparse, groups: list) -> dict:
    """First level of the digit tree on ciphertexts: each group's masked sum is rescaled once and
    rotated by the lowest digit of its target rotation; the results are added per (result chunk,
    remaining digits). {(chunk, rot >> b): ciphertext data}."""
    b = params.rot_step_bits()
    low = (1 << b) - 1
    out = {}
    for ((cr, rot), members) in groups:
        acc = None
        for (_, _, a_pos, b_pos) in members:
            d = masked_product(params, keys, A, B, a_pos, b_pos)
            acc = d if acc is None else ckks.add(params, acc, d)
        acc = ckks.rescale(params, acc)
        if rot & low:
            acc = ckks.rotate_single(params, keys, acc, rot & low)
        key = (cr, rot >> b)
        out[key] = acc if key not in out else ckks.add(params, out[key], acc)
    return {k: v.data for k, v in out.items()}


def digit_tree_finish(params: Params, keys: Keys, level: dict, nres: int) -> list:
    """The remaining levels (digits 1 and up) of ``digit_tree_sum`` on the level-0 partial sums."""
    b = params.rot_step_bits()
    items = [(cr, rest << b, Ct(v, params.delta_out)) for (cr, rest), v in level.items()]
    out = digit_tree_sum(params, items, nres, lambda x, r: ckks.rotate_single(params, keys, x, r),
                         lambda x, y: ckks.add(params, x, y))
    return [None if x is None else x.data for x in out]


def _accumulate(params: Params, keys: Keys, A: EncSparse, B: EncSparse, pairs: list) -> list:
    res = [None] * result_chunks(params, A.rows, B.cols)
    for (i, j, a_pos, b_pos) in pairs:
        cr, d = pair_contribution(params, keys, A, B, i, j, a_pos, b_pos)
        res[cr] = d if res[cr] is None else ckks.add(params, res[cr], d)
    return [None if r is None else r.data for r in res]


def _accumulate_groups(params: Params, keys: Keys, A: EncSparse, B: EncSparse, groups: list) -> list:
    res = [None] * result_chunks(params, A.rows, B.cols)
    for ((cr, rot), members) in groups:
        d = group_contribution(params, keys, A, B, rot, members)
        res[cr] = d if res[cr] is None else ckks.add(params, res[cr], d)
    return [None if r is None else r.data for r in res]


_G = {}


def _worker(idx):
    g = _G
    if g["tree"]:
        return digit_tree_level0(g["params"], g["keys"], g["A"], g["B"], g["parts"][idx])
    if g["grouped"]:
        return _accumulate_groups(g["params"], g["keys"], g["A"], g["B"], g["parts"][idx])
    return _accumulate(g["params"], g["keys"], g["A"], g["B"], g["parts"][idx])


def _keygen_worker(gval):
    k = _G["keys"]
    return gval, k.rot_key(gval)


def rotation_elements(params: Params, A: EncSparse, B: EncSparse, pairs: list) -> set:
    gs = set()
    for (i, j, a_pos, b_pos) in pairs:
        _, _, ra, rb, mn = alignment(params, a_pos, b_pos)
        _, rt = target(params, i, j, B.cols, mn)
        for r in (ra, rb, rt):
            for step in ckks.rotation_steps(params, r):
                gs.add(pow(5, step, 2 * params.N))
    return gs


def spmspm(params: Params, keys: Keys, A: EncSparse, B: EncSparse, workers: int = 1, pairs: list | None = None,
           grouped: bool = False, tree: bool = False, hoist: bool = False) -> list:
    """See _spmspm; hoist: every alignment rotation step is hoisted (ckks.rotate_single_hoisted: the
    automorphism applied to the ModUp digits of the step's input), in any plan mode."""
    _HOIST["on"] = hoist
    try:
        return _spmspm(params, keys, A, B, workers, pairs, grouped, tree)
    finally:
        _HOIST["on"] = False


def _spmspm(params: Params, keys: Keys, A: EncSparse, B: EncSparse, workers: int = 1, pairs: list | None = None,
            grouped: bool = False, tree: bool = False) -> list:
    """Encrypted C = A B as a list of result-chunk ciphertexts (row-major slots).

    ``pairs`` restricts the sum to a subset of matched pairs (default: all).
    ``grouped``: pairs sharing (result chunk, target rotation) go through one second rescale and one
    target rotation together (``group_contribution``); groups are formed over ``pairs``.
    ``tree`` (implies grouped): the groups' target rotations are further shared digit by digit
    (``digit_tree_level0``, ``digit_tree_finish``): a rotation by r = sum_t r_t 2^(b t) is the
    product of its digit steps, and rotation is linear, so the groups whose rotations agree above
    digit t are added before their common digit-t step.
    With workers > 1 the pairs (or groups) are split across processes and the partial results are
    added; addition mod q is exact, so the result does not depend on the split."""
    assert A.cols == B.rows
    grouped = grouped or tree
    if pairs is None:
        pairs = matched_pairs(A.rows, B.cols, A.indptr, A.indices, B.indptr, B.indices)
    units = target_groups(params, pairs, B.cols) if grouped else pairs
    out_nl = params.n_q - 2
    nres = result_chunks(params, A.rows, B.cols)
    if tree:
        if workers <= 1 or len(units) < 2:
            levels = [digit_tree_level0(params, keys, A, B, units)]
        else:
            gs = sorted(rotation_elements(params, A, B, pairs) - set(keys._rot))
            ctx = mp.get_context("fork")
            _G.update(params=params, keys=keys, A=A, B=B, grouped=True, tree=True)
            if gs:
                with ctx.Pool(workers) as pool:
                    for gval, key in pool.imap_unordered(_keygen_worker, gs):
                        keys._rot[gval] = key
            _G["parts"] = [units[w::workers] for w in range(workers)]
            with ctx.Pool(workers) as pool:
                levels = pool.map(_worker, range(workers))
            _G.clear()
        level = {}
        for part in levels:
            for k, v in part.items():
                level[k] = v if k not in level else ckks.add(params, Ct(level[k], params.delta_out),
                                                            Ct(v, params.delta_out)).data
        parts = [digit_tree_finish(params, keys, level, nres)]
    elif workers <= 1 or len(units) < 2:
        parts = [_accumulate_groups(params, keys, A, B, units) if grouped else _accumulate(params, keys, A, B, units)]
    else:
        gs = sorted(rotation_elements(params, A, B, pairs) - set(keys._rot))
        ctx = mp.get_context("fork")
        _G.update(params=params, keys=keys, A=A, B=B, grouped=grouped, tree=False)
        if gs:
            with ctx.Pool(workers) as pool:
                for gval, key in pool.imap_unordered(_keygen_worker, gs):
                    keys._rot[gval] = key
        _G["parts"] = [units[w::workers] for w in range(workers)]
        with ctx.Pool(workers) as pool:
            parts = pool.map(_worker, range(workers))
        _G.clear()
    res = []
    for c in range(nres):
        acc = ckks.zero_ct(params, out_nl, params.delta_out)
        for part in parts:
            if part[c] is not None:
                acc = ckks.add(params, acc, Ct(part[c], params.delta_out))
        res.append(acc)
    return res


def decrypt_result(params: Params, keys: Keys, res: list, m: int, n: int) -> np.ndarray:
    S = params.S
    out = np.zeros(m * n)
    for c, ct in enumerate(res):
        lo, hi = c * S, min((c + 1) * S, m * n)
        if hi > lo:
            out[lo:hi] = ckks.decrypt_decode(params, keys, ct, np.arange(hi - lo))
    return out.reshape(m, n)
