"""Pins of the oracle's seed expansion: the builder-defined reading for the
seeds the paper does not fix (the GM/GQ ensembles of Table 2 at every seed,
MRG32K3A outside 1 <= seed < m2, LFSR113 outside 128 <= seed < 2^32).

The reading: SplitMix64 (Steele, Lea & Flood) whose start state is the first
SplitMix64 output from seed XOR gamma * (generator + 1), gamma being the
SplitMix64 Weyl increment;
GM/GQ elements i = 0 .. s - 1 draw (x^(n-1), x^(n)) in that order, each value
from the top ceil(log2 g) bits of a draw, redrawn while >= g, the pair redrawn
while both are 0 mod p; MRG32K3A draws x_n, x_{n-1}, x_{n-2} below m1, then the
y triple below m2, a triple redrawn while all zero; LFSR113 takes the top 32
bits of one draw per component, redrawn while the component's top-k bit field
is zero.

What pins it, other than the oracle itself:
 * the Weyl increment is the odd integer nearest 2^64 / golden ratio, computed
   here from an integer square root;
 * the output function is the 64-bit finalizer that pandas applies in
   ``pandas.util.hash_array`` to uint64 data (an implementation that shares
   nothing with the oracle), and mix(gamma), the first output of SplitMix64
   from state 0, is the value its authors publish for that state;
 * the draws are re-derived from those two pieces and compared with the
   oracle's states element for element, over many seeds and every generator;
 * properties a slip anywhere in the expansion would break: element pairs of
   one state pairwise distinct (a reused draw repeats a pair), uniform values
   (a wrong shift in the bounded draw halves or skews the range), states of
   different generators and of neighbouring seeds unrelated (a dropped or
   shared tag makes the 8- and 32-element GQ58 ensembles share elements).
"""
import math

import numpy as np
import pytest
from pandas.util import hash_array

from oracle.oracle import gm_arrays

MASK = (1 << 64) - 1
GM_GENS = list(range(3, 11))
# (k, q, g, p, s) of Table 2 (g = p * 2^t) and the ensemble sizes of the
# launch-shape table
GM = {
    3: (15, 28, 524287, 524287, 32),
    4: (4, 2, 536870909, 536870909, 32),
    5: (11, 14, 2147483647, 2147483647, 32),
    6: (256, 176, 2251799813685119 * 16, 2251799813685119, 8),
    7: (24, 74, 2305843009213693951, 2305843009213693951, 32),
    8: (8, 48, 536870909 << 29, 536870909, 32),
    9: (8, 48, 536870909 << 29, 536870909, 12),
    10: (8, 48, 536870909 << 29, 536870909, 8),
}
M1, M2 = 4294967087, 4294944443


def golden_gamma():
    """Odd integer nearest 2^64 * (sqrt(5) - 1) / 2 = 2^64 / golden ratio."""
    r = (math.isqrt(5 << 128) - (1 << 64)) // 2     # floor(2^64 (sqrt 5 - 1) / 2)
    return r if r & 1 else r + 1


GAMMA = golden_gamma()


def mix(states):
    """The SplitMix64 output function, through pandas' implementation."""
    return [int(v) for v in hash_array(np.array(states, dtype=np.uint64))]


class Stream:
    """SplitMix64 draws from a 64-bit start state: state += gamma, output
    mix(state).  Draws are produced in batches."""

    def __init__(self, state):
        self.state, self.buf = state & MASK, []

    def next(self):
        if not self.buf:
            ss = [(self.state + GAMMA * (j + 1)) & MASK for j in range(64)]
            self.state = ss[-1]
            self.buf = mix(ss)[::-1]
        return self.buf.pop()

    def below(self, bound):
        nb = (bound - 1).bit_length()
        while True:
            r = self.next() >> (64 - nb)
            if r < bound:
                return r


def tag(gen):
    return (GAMMA * (gen + 1)) & MASK


def start(seed, gen):
    """Start state of a seed's expansion: one SplitMix64 output from
    seed ^ tag(gen)."""
    return mix([((seed ^ tag(gen)) + GAMMA) & MASK])[0]


def expected_gm(gen, seed):
    k, q, g, p, s = GM[gen]
    sm = Stream(start(seed, gen))
    xp, xc = [], []
    for _ in range(s):
        while True:
            a, b = sm.below(g), sm.below(g)
            if not (a % p == 0 and b % p == 0):
                break
        xp.append(a)
        xc.append(b)
    return xp, xc


def test_gamma_closed_form():
    assert GAMMA == 0x9E3779B97F4A7C15


def test_first_output_from_state_zero():
    # the value SplitMix64's authors give for the first output from state 0
    assert mix([GAMMA])[0] == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("gen", GM_GENS)
def test_gm_states_are_the_defined_draws(oracle, gen):
    s = GM[gen][4]
    for seed in list(range(0, 40)) + [2**32 - 1, 2**32, 0x0123456789ABCDEF, 2**64 - 1]:
        xp, xc, off = gm_arrays(oracle.seed(gen, seed))
        exp_p, exp_c = expected_gm(gen, seed)
        assert off == 0
        assert [int(v) for v in xp[:s]] == exp_p, f"gen {gen} seed {seed} x^(n-1)"
        assert [int(v) for v in xc[:s]] == exp_c, f"gen {gen} seed {seed} x^(n)"


@pytest.mark.parametrize("gen", GM_GENS)
def test_gm_default_is_seed_zero(oracle, gen):
    assert np.array_equal(oracle.init_default(gen), oracle.seed(gen, 0))


@pytest.mark.parametrize("seed", [0, 2**32 + 5, 4294944443, 2**64 - 1])
def test_mrg_expanded_branch_is_the_defined_draws(oracle, seed):
    st = oracle.seed(1, seed).view(np.uint32)
    sm = Stream(start(seed, 1))
    while True:
        x = [sm.below(M1) for _ in range(3)]
        if any(x):
            break
    while True:
        y = [sm.below(M2) for _ in range(3)]
        if any(y):
            break
    assert [int(v) for v in st[:3]] == x and [int(v) for v in st[3:6]] == y


@pytest.mark.parametrize("seed", [0, 1, 127, 2**32, 2**40 + 3, 2**64 - 1])
def test_lfsr_expanded_branch_is_the_defined_draws(oracle, seed):
    st = oracle.seed(2, seed).view(np.uint32)
    sm = Stream(start(seed, 2))
    for c, k in enumerate((31, 29, 28, 25)):
        while True:
            z = sm.next() >> 32
            if z >> (32 - k):
                break
        assert int(st[c]) == z, f"component {c}"


def test_verbatim_branches(oracle):
    for seed in (1, 12345, M2 - 1):
        assert list(oracle.seed(1, seed).view(np.uint32)) == [seed] * 6
    for seed in (128, 12345, 2**32 - 1):
        assert list(oracle.seed(2, seed).view(np.uint32)) == [seed] * 4


@pytest.mark.parametrize("gen", GM_GENS)
def test_gm_element_pairs_distinct_and_in_range(oracle, gen):
    """Seeds 0..999: every state's s element pairs are distinct, in range and
    not both 0 mod p; no two states share a pair."""
    k, q, g, p, s = GM[gen]
    seen = set()
    for seed in range(1000):
        xp, xc, _ = gm_arrays(oracle.seed(gen, seed))
        pairs = [(int(a), int(b)) for a, b in zip(xp[:s], xc[:s])]
        assert all(a < g and b < g and not (a % p == 0 and b % p == 0) for a, b in pairs)
        assert len(set(pairs)) == s, f"seed {seed}"
        assert not np.any(xp[s:]) and not np.any(xc[s:])
        seen.update(pairs)
    assert len(seen) == 1000 * s


def chi2_uniform(u, bins=64):
    """Pearson statistic of values in [0, 1) over equal bins and its
    Wilson-Hilferty z-score (about N(0, 1) for a uniform sample)."""
    h = np.bincount(np.minimum((np.asarray(u) * bins).astype(int), bins - 1), minlength=bins)
    e = len(u) / bins
    x = float(((h - e) ** 2 / e).sum())
    d = bins - 1
    return (((x / d) ** (1 / 3)) - (1 - 2 / (9 * d))) / math.sqrt(2 / (9 * d))


@pytest.mark.parametrize("gen", GM_GENS)
def test_gm_values_uniform(oracle, gen):
    """Element values / g over seeds 0..999 (both state slots): the histogram
    of 64 bins, and of the top and bottom halves of the range, is flat; the
    lag-1 correlation between consecutive draws is near zero."""
    k, q, g, p, s = GM[gen]
    vals = []
    for seed in range(1000):
        xp, xc, _ = gm_arrays(oracle.seed(gen, seed))
        for a, b in zip(xp[:s], xc[:s]):
            vals += [int(a) / g, int(b) / g]
    u = np.array(vals)
    assert abs(chi2_uniform(u)) < 5.0
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / len(u))
    assert abs((u < 0.5).mean() - 0.5) < 5 * 0.5 / math.sqrt(len(u))
    c = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(c) < 5 / math.sqrt(len(u))


def test_generators_and_neighbouring_seeds_unrelated(oracle):
    """States of the three GQ58 generators (same modulus, 32, 12 and 8
    elements) share no element for one seed; the first elements of different
    generators are uncorrelated over seeds, and so are neighbouring seeds."""
    for seed in range(200):
        sets = [set(int(v) for v in gm_arrays(oracle.seed(gen, seed))[1][:GM[gen][4]]) for gen in (8, 9, 10)]
        assert not (sets[0] & sets[1]) and not (sets[0] & sets[2]) and not (sets[1] & sets[2])
    first = {gen: np.array([int(gm_arrays(oracle.seed(gen, seed))[1][0]) / GM[gen][2] for seed in range(2000)])
             for gen in GM_GENS}
    lim = 5 / math.sqrt(2000)
    for a in GM_GENS:
        assert abs(np.corrcoef(first[a][:-1], first[a][1:])[0, 1]) < lim
        for b in GM_GENS:
            if a < b:
                assert abs(np.corrcoef(first[a], first[b])[0, 1]) < lim, (a, b)


def test_expanded_mrg_lfsr_states_distinct_and_in_range(oracle):
    mrg, lfsr = set(), set()
    for seed in [0] + [2**32 + i for i in range(500)]:
        m = tuple(int(v) for v in oracle.seed(1, seed).view(np.uint32))
        assert all(v < M1 for v in m[:3]) and all(v < M2 for v in m[3:]) and any(m[:3]) and any(m[3:])
        mrg.add(m)
        z = tuple(int(v) for v in oracle.seed(2, seed).view(np.uint32))
        assert z[0] >= 2 and z[1] >= 8 and z[2] >= 16 and z[3] >= 128
        lfsr.add(z)
    assert len(mrg) == 501 and len(lfsr) == 501
