"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
runs.  This module draws stream ids, jump exponents, request mixes and the
like from numpy's PCG64; it contains none of the generators' arithmetic.

Master seed 13075869; every workload mixes in its own tag so that the draws
of one never depend on another.
"""
import numpy as np

MASTER_SEED = 13075869
ID_BOUND = 10**19          # stream ids are uniform in [0, 10^19)

# jump exponents k (distance 2^k) drawn per generator for the stream-init
# workload: 10 .. the largest exponent the generator's stream table supports
JUMP_EXP_RANGE = {
    0: (10, 511),    # MT19937
    1: (10, 76),     # MRG32K3A
    2: (10, 112),    # LFSR113
    3: (10, 37),     # GM19
    4: (10, 57),     # GM29
    5: (10, 61),     # GM31
    6: (10, 101),    # GM55
    7: (10, 121),    # GM61
    8: (10, 57),     # GQ58.1
    9: (10, 57),     # GQ58.3
    10: (10, 57),    # GQ58.4
}


def rng(tag):
    return np.random.Generator(np.random.PCG64([MASTER_SEED, tag]))


def stream_ids(count, gen, tag=1):
    """count stream ids uniform in [0, 10^19) for generator gen."""
    return rng(tag * 100 + gen).integers(0, ID_BOUND, size=count, dtype=np.uint64)


def jump_exponents(count, gen, tag=3):
    lo, hi = JUMP_EXP_RANGE[gen]
    return rng(tag * 100 + gen).integers(lo, hi + 1, size=count)


def small_jumps(count, gen, tag=33, bound=2**16):
    """Distances n <= 2^16 for the brute-force check of the jump workload."""
    return rng(tag * 100 + gen).integers(1, bound + 1, size=count, dtype=np.uint64)


def batched_tasks(count=20000, tag=4, lo=1e3, hi=1e7):
    """(gen, id, length) for the batched launch: gen uniform over 11, id
    uniform in [0, 10^19), length log-uniform in [lo, hi]."""
    r = rng(tag)
    gens = r.integers(0, 11, size=count)
    ids = r.integers(0, ID_BOUND, size=count, dtype=np.uint64)
    lens = np.rint(np.exp(r.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    return gens, ids, lens


def serving_requests(rate=2000.0, seconds=60.0, tag=5, lo=1e3, hi=1e8):
    """Poisson arrivals: (arrival time s, gen, id, n, dtype)."""
    r = rng(tag)
    gaps = r.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 100)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    m = t.size
    gens = r.integers(0, 11, size=m)
    ids = r.integers(0, ID_BOUND, size=m, dtype=np.uint64)
    ns = np.rint(np.exp(r.uniform(np.log(lo), np.log(hi), size=m))).astype(np.int64)
    dts = r.integers(0, 3, size=m)
    return t, gens, ids, ns, dts
