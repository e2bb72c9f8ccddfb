"""Seeded synthetic sparse operands (no CKKS arithmetic lives here).

The paper evaluates on random square matrices at several sparsity levels
(Section 4); the workloads below keep that recipe at the shapes of the
benchmark configurations. Zeros are placed exactly: round(sparsity * size)
positions chosen by a seeded permutation; values come from a seeded numpy
PCG64 stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def sparse_dense(rows: int, cols: int, sparsity: float, dist: str, seed_values: int, seed_mask: int,
                 lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rv = np.random.Generator(np.random.PCG64(seed_values))
    if dist == "uniform":
        vals = rv.uniform(lo, hi, size=(rows, cols))
    elif dist == "halfnormal":
        vals = np.abs(rv.standard_normal(size=(rows, cols)))
    else:
        raise ValueError(dist)
    rm = np.random.Generator(np.random.PCG64(seed_mask))
    nzero = int(round(sparsity * rows * cols))
    perm = rm.permutation(rows * cols)
    flat = vals.reshape(-1).copy()
    flat[perm[:nzero]] = 0.0
    return flat.reshape(rows, cols)


def to_csr(d: np.ndarray):
    """(indptr int32[rows+1], indices int32[nnz] column ids ascending per row, values f64[nnz])."""
    rows, _ = d.shape
    indptr = np.zeros(rows + 1, np.int32)
    idx, val = [], []
    for i in range(rows):
        nz = np.nonzero(d[i])[0]
        idx.extend(nz.tolist())
        val.extend(d[i, nz].tolist())
        indptr[i + 1] = len(idx)
    return indptr, np.asarray(idx, np.int32), np.asarray(val, np.float64)


def to_csc(d: np.ndarray):
    """(indptr int32[cols+1], indices int32[nnz] row ids ascending per column, values f64[nnz])."""
    return to_csr(np.ascontiguousarray(d.T))


def full_csr(d: np.ndarray):
    """The CSR arrays of d with every entry stored, zeros included (the naive dense plan: every
    (i, k, j) product is computed whatever the values)."""
    rows, cols = d.shape
    indptr = (np.arange(rows + 1, dtype=np.int32) * cols).astype(np.int32)
    indices = np.tile(np.arange(cols, dtype=np.int32), rows)
    return indptr, indices, np.ascontiguousarray(d, dtype=np.float64).reshape(-1)


def full_csc(d: np.ndarray):
    return full_csr(np.ascontiguousarray(d.T))


def stored_nonzero_csr(d: np.ndarray) -> np.ndarray:
    """One flag per entry of full_csr(d) in its packing order (row-major): 1 where the value is nonzero."""
    return (np.ascontiguousarray(d) != 0).reshape(-1).astype(np.uint8)


def stored_nonzero_csc(d: np.ndarray) -> np.ndarray:
    """One flag per entry of full_csc(d) in its packing order (column-major)."""
    return stored_nonzero_csr(np.ascontiguousarray(d.T))


@dataclass(frozen=True)
class Workload:
    name: str
    log_n: int
    n_q: int
    n_p: int
    alpha: int
    rot_digits: int
    m: int
    k: int
    n: int
    sparsity_a: float
    sparsity_b: float
    dist_a: tuple
    dist_b: tuple

    def operands(self, seeds=(0, 1, 2, 3)):
        a = sparse_dense(self.m, self.k, self.sparsity_a, self.dist_a[0], seeds[0], seeds[2], *self.dist_a[1:])
        b = sparse_dense(self.k, self.n, self.sparsity_b, self.dist_b[0], seeds[1], seeds[3], *self.dist_b[1:])
        return a, b


WORKLOADS = {
    # 16x16 x 16x16, 75% zeros each, N = 2^13, 4 x 50-bit Q primes, 1 x 60-bit P prime
    "plain": Workload("plain", 13, 4, 1, 1, 1, 16, 16, 16, 0.75, 0.75, ("uniform", -1.0, 1.0), ("uniform", -1.0, 1.0)),
    # DNN layer: W 128x128 (90% zeros, U[-0.1,0.1]) times X 128x64 (50% zeros, |N(0,1)|), N = 2^15
    "dnn": Workload("dnn", 15, 10, 2, 2, 2, 128, 128, 64, 0.90, 0.50, ("uniform", -0.1, 0.1), ("halfnormal",)),
    # 512x512 (95% zeros) times 512x512 (60% zeros), N = 2^16, 24 Q primes, 3 P primes
    "large": Workload("large", 16, 24, 3, 3, 3, 512, 512, 512, 0.95, 0.60, ("uniform", -0.1, 0.1), ("halfnormal",)),
}


@dataclass(frozen=True)
class BatchWorkload:
    """Many independent square matmuls of uneven size and sparsity under one parameter set."""
    name: str
    log_n: int
    n_q: int
    n_p: int
    alpha: int
    rot_digits: int
    count: int
    sizes: tuple
    sparsity: tuple  # (low, high) of the per-operand uniform draw
    seed: int

    def specs(self):
        """[(n, sparsity_a, sparsity_b)] for every matmul, from one seeded stream."""
        r = np.random.Generator(np.random.PCG64(self.seed))
        out = []
        for _ in range(self.count):
            n = int(r.choice(self.sizes))
            sa, sb = (float(x) for x in r.uniform(self.sparsity[0], self.sparsity[1], size=2))
            out.append((n, sa, sb))
        return out

    def operands(self, i: int, spec=None):
        n, sa, sb = spec if spec is not None else self.specs()[i]
        s = self.seed * 100000 + 4 * i
        a = sparse_dense(n, n, sa, "uniform", s, s + 2)
        b = sparse_dense(n, n, sb, "uniform", s + 1, s + 3)
        return a, b


BATCH_WORKLOADS = {
    # 64 matmuls, square sizes from {32, 64, 128, 256}, per-operand sparsity U[0.5, 0.95], values
    # U[-1, 1]; N = 2^16, 24 x 50-bit Q primes, 3 x 60-bit P primes, alpha = 3, 3 rotation digits
    "batch": BatchWorkload("batch", 16, 24, 3, 3, 3, 64, (32, 64, 128, 256), (0.5, 0.95), 1),
    # the same batch shape at the 16x16 workload's parameters: 64 matmuls of square size 8 or 16 at
    # N = 2^13, 4 Q + 1 P primes, alpha = 1, per-amount rotation keys (small plans, where launches
    # of one matmul do not fill the GPU)
    "batch_small": BatchWorkload("batch_small", 13, 4, 1, 1, 1, 64, (8, 16), (0.5, 0.95), 1),
}


def poisson_arrivals(rate: float, window_s: float, seed: int) -> np.ndarray:
    """Arrival times in [0, window_s) of a Poisson process of the given rate (seeded)."""
    r = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += float(r.exponential(1.0 / rate))
        if t >= window_s:
            return np.asarray(out)
        out.append(t)
