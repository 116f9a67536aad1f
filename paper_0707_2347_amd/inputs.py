"""Seeded synthetic inputs: uniform residues, shared by tests, oracle runs and
the benchmark.  This module holds none of the method's arithmetic.

Recipe: numpy ``Generator(PCG64(seed))`` draws A, then B, then C (when the
workload accumulates) with ``integers(0, p, size, dtype=int64)``, row-major.
Binary64 storage is the exact cast of those integers.  The batch workload
draws its sizes and primes from ``PCG64(5)`` and product i's matrices from
``PCG64([5, i])``.
"""
import math

import numpy as np

PRIMES = (65521, 1048573, 8388593)

# Named workloads (sizes, modulus, operation, schedules, recursion depth).
WORKLOADS = {
    "t1_512_p65521_l1_i64": dict(seed=1, m=512, k=512, n=512, p=65521, alpha=1, beta=0,
                                 dtype="i64", schedules=("two_temp",), levels=1),
    "acc_4096_p65521_l3": dict(seed=2, m=4096, k=4096, n=4096, p=65521, alpha=1, beta=1,
                               dtype="f64", schedules=("two_temp", "overwrite"), levels=3),
    "ipmm_8192x4096x8192_p8388593": dict(seed=3, m=8192, k=4096, n=8192, p=8388593,
                                         alpha=1, beta=0, dtype="f64",
                                         schedules=("readonly_inplace", "two_temp"),
                                         levels=1),
    "t1_16384_p1048573": dict(seed=4, m=16384, k=16384, n=16384, p=1048573, alpha=1,
                              beta=0, dtype="f64", schedules=("two_temp",), levels=None),
    # the largest shape of the paper's rectangular timings (m = n < k)
    "overwrite_8192x16384x8192_p8388593": dict(seed=6, m=8192, k=16384, n=8192, p=8388593,
                                               alpha=1, beta=0, dtype="f64",
                                               schedules=("overwrite",), levels=1),
}


def uniform(seed, m, k, n, p, with_c=False):
    """A (m x k), B (k x n) and optionally C (m x n), int64 residues in [0, p)."""
    g = np.random.Generator(np.random.PCG64(seed))
    A = g.integers(0, p, size=(m, k), dtype=np.int64)
    B = g.integers(0, p, size=(k, n), dtype=np.int64)
    C = g.integers(0, p, size=(m, n), dtype=np.int64) if with_c else None
    return A, B, C


def uniform_f64(seed, m, k, n, p, with_c=False):
    """Same draws as :func:`uniform`, cast to float64 one matrix at a time."""
    g = np.random.Generator(np.random.PCG64(seed))
    A = g.integers(0, p, size=(m, k), dtype=np.int64).astype(np.float64)
    B = g.integers(0, p, size=(k, n), dtype=np.int64).astype(np.float64)
    C = (g.integers(0, p, size=(m, n), dtype=np.int64).astype(np.float64)
         if with_c else None)
    return A, B, C


def batch_problems(count=2000, seed=5, lo=64, hi=2048):
    """Sizes and primes of the batch workload: each of m, k, n is
    round(exp(U(ln lo, ln hi))), p uniform over PRIMES."""
    g = np.random.Generator(np.random.PCG64(seed))
    dims = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=(count, 3))))
    dims = dims.astype(np.int64)
    ps = g.integers(0, len(PRIMES), size=count)
    return [dict(m=int(d[0]), k=int(d[1]), n=int(d[2]), p=PRIMES[int(j)], index=i)
            for i, (d, j) in enumerate(zip(dims, ps))]


def batch_inputs(prob, seed=5):
    """A and B of one batch product (float64 holding residues)."""
    g = np.random.Generator(np.random.PCG64([seed, prob["index"]]))
    A = g.integers(0, prob["p"], size=(prob["m"], prob["k"]), dtype=np.int64)
    B = g.integers(0, prob["p"], size=(prob["k"], prob["n"]), dtype=np.int64)
    return A.astype(np.float64), B.astype(np.float64)
