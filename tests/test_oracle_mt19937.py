"""Pins of the oracle's MT19937 (generator, seeding, jump-ahead) against things
other than itself: independent implementations (numpy, CPython, libstdc++),
brute force, and algebraic facts of the jump of the paper's MT19937 section
(equation g_v: A^v Y = g_v(A) Y with g_v = x^v mod phi)."""
import os
import random
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.oracle import mt_words

MT = 0


def numpy_raw(seed, n):
    bg = np.random.RandomState(seed)._bit_generator
    return bg.random_raw(n).astype(np.uint32)


@pytest.mark.parametrize("seed", [5489, 0, 1, 12345, 2**32 - 1])
def test_init_genrand_matches_numpy_legacy(oracle, seed):
    st = oracle.seed(MT, seed)
    words, mti = mt_words(st)
    key = np.random.RandomState(seed).get_state()[1]
    assert mti == 624
    assert np.array_equal(words, key.astype(np.uint32))
    assert np.array_equal(oracle.generate(MT, st, 2000), numpy_raw(seed, 2000))


def test_default_is_5489(oracle):
    a = oracle.generate(MT, oracle.init_default(MT), 100)
    assert np.array_equal(a, numpy_raw(5489, 100))


@pytest.mark.parametrize("seed", [2**32, 2**32 + 7, 0xDEADBEEFCAFEF00D, 2**64 - 1])
def test_init_by_array_matches_cpython(oracle, seed):
    st = oracle.seed(MT, seed)
    words, mti = mt_words(st)
    r = random.Random(seed)          # CPython seeds ints >= 2^32 via init_by_array
    state = r.getstate()[1]
    assert list(words) == list(state[:624]) and mti == state[624]
    ours = oracle.generate(MT, st, 1500)
    theirs = [r.getrandbits(32) for _ in range(1500)]
    assert list(ours) == theirs
    # numpy's legacy seeding by a key array is init_by_array as well
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
    bg = np.random.RandomState(key)._bit_generator
    assert np.array_equal(bg.random_raw(100).astype(np.uint32), oracle.generate(MT, oracle.seed(MT, seed), 100))


def test_arbitrary_mid_block_states_match_cpython(oracle):
    """Load oracle states with any index into CPython's generator."""
    st = oracle.seed(MT, 987654321)
    for consumed in [1, 226, 227, 396, 397, 623, 624, 700]:
        s = st.copy()
        oracle.generate(MT, s, consumed)
        words, mti = mt_words(s)
        r = random.Random()
        r.setstate((3, tuple(int(w) for w in words) + (mti,), None))
        ours = oracle.generate(MT, s, 1300)
        assert list(ours) == [r.getrandbits(32) for _ in range(1300)]


CXX_SRC = r"""
#include <random>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  std::mt19937 d;                 // default-constructed: seed 5489
  unsigned v = 0;
  for (int i = 0; i < 10000; i++) v = d();
  std::printf("%u\n", v);
  std::mt19937 s((unsigned)std::strtoul(argv[1], 0, 10));
  for (int i = 0; i < 1000; i++) std::printf("%u\n", (unsigned)s());
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_matches_libstdcxx(oracle):
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "m.cpp"), os.path.join(d, "m")
        open(src, "w").write(CXX_SRC)
        subprocess.check_call(["g++", "-O1", "-o", exe, src])
        out = subprocess.check_output([exe, "4242"]).decode().split()
    vals = [int(x) for x in out]
    ours = oracle.generate(MT, oracle.init_default(MT), 10000)
    assert ours[-1] == vals[0]
    assert list(oracle.generate(MT, oracle.seed(MT, 4242), 1000)) == vals[1:]


def _brute(oracle, st, n, k):
    s = st.copy()
    if n:
        oracle.generate(MT, s, n)
    return oracle.generate(MT, s, k)


@pytest.mark.parametrize("consumed", [0, 1, 313, 623, 624, 1000])
@pytest.mark.parametrize("n", [0, 1, 2, 310, 311, 623, 624, 625, 1247, 19937, 123457])
def test_jump_equals_brute_force(oracle, consumed, n):
    st = oracle.seed(MT, 20240601)
    oracle.generate(MT, st, consumed)
    j = st.copy()
    oracle.skipahead(MT, j, n)
    assert np.array_equal(oracle.generate(MT, j, 700), _brute(oracle, st, n, 700))


def test_jump_large_brute_force(oracle):
    st = oracle.init_default(MT)
    n = 2_000_003
    j = st.copy()
    oracle.skipahead(MT, j, n)
    assert np.array_equal(oracle.generate(MT, j, 1000), _brute(oracle, st, n, 1000))


def test_jump_result_is_canonical(oracle):
    st = oracle.init_default(MT)
    oracle.skipahead(MT, st, 5000)
    words, mti = mt_words(st)
    assert mti == 624 and (int(words[0]) & 0x7FFFFFFF) == 0


@pytest.mark.parametrize("a,b", [(2**100 + 3, 2**300 + 12345), (10**19 * 2**432, 2**432 + 99),
                                 (623, 2**64 - 1), (7, 11)])
def test_jump_composition(oracle, a, b):
    s1 = oracle.seed(MT, 77)
    oracle.skipahead(MT, s1, a)
    oracle.skipahead(MT, s1, b)
    s2 = oracle.seed(MT, 77)
    oracle.skipahead(MT, s2, a + b)
    assert np.array_equal(oracle.generate(MT, s1, 800), oracle.generate(MT, s2, 800))


def test_jump_doubling(oracle):
    for k in [20, 77, 200, 433, 510]:
        s1 = oracle.init_default(MT)
        oracle.skipahead(MT, s1, 2**k)
        oracle.skipahead(MT, s1, 2**k)
        s2 = oracle.init_default(MT)
        oracle.skipahead(MT, s2, 2**(k + 1))
        assert np.array_equal(s1, s2)


def _bits_of_outputs(oracle, seed, bit, n):
    out = oracle.generate(MT, oracle.seed(MT, seed), n)
    b = ((out >> bit) & 1).astype(np.uint8)
    return int.from_bytes(np.packbits(b, bitorder="little").tobytes(), "little")


@pytest.mark.parametrize("seed,bit", [(1234567, 17), (2**40 + 5, 31), (5489, 0)])
def test_charpoly_annihilates_output_bits(oracle, seed, bit):
    """phi(A) = 0: every output-bit sequence satisfies the recurrence whose
    characteristic polynomial is phi (checked on functionals and seeds other
    than the one the polynomial was derived from)."""
    phi = oracle.mt_charpoly()
    assert phi.bit_length() - 1 == 19937
    assert phi & 1 == 1 and bin(phi).count("1") % 2 == 1   # phi(0) = phi(1) = 1
    s = _bits_of_outputs(oracle, seed, bit, 19937 + 3000)
    for j in range(0, 3000, 37):
        assert bin(phi & (s >> j)).count("1") % 2 == 0


def test_charpoly_is_not_annihilating_a_shorter_recurrence(oracle):
    """A dropped or wrong coefficient breaks the recurrence somewhere."""
    phi = oracle.mt_charpoly()
    s = _bits_of_outputs(oracle, 99, 5, 19937 + 400)
    for flip in [0, 1, 5000, 19936]:
        bad = phi ^ (1 << flip)
        assert any(bin(bad & (s >> j)).count("1") % 2 for j in range(0, 400))


def test_jump_poly_closed_forms(oracle):
    phi = oracle.mt_charpoly()
    for n in [0, 1, 63, 64, 1000, 19936]:
        assert oracle.mt_jump_poly(n) == 1 << n
    assert oracle.mt_jump_poly(19937) == phi ^ (1 << 19937)


def test_word_reduction_equals_bitwise(oracle):
    rng = np.random.default_rng(5)
    for _ in range(3):
        a = int.from_bytes(rng.bytes(4984), "little") & ((1 << (2 * 19937 - 1)) - 1)
        assert oracle.mt_reduce(a, True) == oracle.mt_reduce(a, False)


@pytest.mark.slow
def test_charpoly_irreducible_rabin(oracle):
    """19937 is prime: phi is irreducible iff x^(2^19937) = x mod phi and phi
    has no root in F2 (the latter checked in the annihilation test)."""
    assert oracle.mt_frobenius(19937) == 2
