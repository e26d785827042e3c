"""Pins of block splitting (section "Parallel streams of pseudorandom numbers":
stream id starts id * L outputs into the base sequence) and of the stream table
(Table 4), plus the fixed integer-to-float maps."""
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NAMES = ["mt19937", "mrg32k3a", "lfsr113", "gm19", "gm29", "gm31", "gm55", "gm61", "gq58x1", "gq58x3", "gq58x4"]
VARIANT = {"init_sequence_": 1, "init_short_sequence_": 2, "init_medium_sequence_": 3, "init_long_sequence_": 4}
# words per ensemble step: GQ58.3 yields 9 words per 8 steps, the rest one
WORDS_PER_STEP = {"gq58x3": Fraction(9, 8)}
PERIOD = {
    "mt19937": 2**19937 - 1,
    "mrg32k3a": (2**32 - 209)**3 * (2**32 - 22853)**3 // 2,
    "lfsr113": (2**31 - 1) * (2**29 - 1) * (2**28 - 1) * (2**25 - 1),
    "gm19": (2**19 - 1)**2 - 1, "gm29": (2**29 - 3)**2 - 1, "gm31": (2**31 - 1)**2 - 1,
    "gm55": (2**51 - 129)**2 - 1, "gm61": (2**61 - 1)**2 - 1,
    "gq58x1": (2**29 - 3)**2 - 1, "gq58x3": ((2**29 - 3)**2 - 1) * 9 // 8, "gq58x4": (2**29 - 3)**2 - 1,
}


def table4():
    rows = []
    for line in open(os.path.join(GOLD, "table4_streams.txt")):
        if line.startswith("#") or not line.strip():
            continue
        fn, nseq, maxlen = line.split()
        gen_name, rest = fn.split("_", 1)
        rows.append((NAMES.index(gen_name), VARIANT[rest], float(nseq), float(maxlen)))
    return rows


@pytest.mark.parametrize("gen,variant,nseq,maxlen", table4())
def test_block_length_covers_table4(oracle, gen, variant, nseq, maxlen):
    e = oracle.block_log2(gen, variant)
    assert e > 0
    L = oracle.stream_distance(gen, variant, 1)
    assert L >= maxlen                              # each stream holds its maximal length
    # all Table 4 streams fit in one period without overlap
    assert int(nseq) * L <= PERIOD[NAMES[gen]]
    # the block is 2^e ensemble steps (outputs for the single-word generators)
    assert L == 2**e * WORDS_PER_STEP.get(NAMES[gen], 1)


def test_unlisted_variants_unsupported(oracle):
    listed = {(g, v) for g, v, _, _ in table4()}
    for g in range(11):
        for v in range(1, 5):
            if (g, v) not in listed:
                assert oracle.block_log2(g, v) == -2
        # the default variant is one of the listed ones
        e = oracle.block_log2(g, 0)
        assert any(oracle.block_log2(g, v) == e for v in range(1, 5) if (g, v) in listed)


@pytest.mark.parametrize("gen", range(11))
def test_blocks_are_consecutive_slices_of_the_base_sequence(oracle, gen):
    """Stream k from distance k*B equals words [kB, (k+1)B) of the base stream."""
    B, K = 1024, 12
    base = oracle.init_default(gen)
    ref = oracle.generate(gen, base.copy(), B * K)
    for k in range(K):
        st = base.copy()
        oracle.skipahead(gen, st, k * B)
        assert np.array_equal(oracle.generate(gen, st, B), ref[k * B:(k + 1) * B])


def test_gm19_stream_one_follows_stream_zero(oracle):
    """GM19's block is 2^23 outputs: stream 1 begins where stream 0's block ends."""
    gen = 3
    L = oracle.stream_distance(gen, 1, 1)
    assert L == 2**23
    s0 = oracle.init_stream(gen, 1, 0)
    assert np.array_equal(s0, oracle.init_default(gen))
    oracle.generate(gen, s0, L)
    s1 = oracle.init_stream(gen, 1, 1)
    assert np.array_equal(oracle.generate(gen, s0, 64), oracle.generate(gen, s1, 64))


@pytest.mark.parametrize("gen", range(11))
def test_init_stream_is_jump_of_id_times_block(oracle, gen):
    for sid in [0, 1, 5, 10**19 - 1]:
        a = oracle.init_stream(gen, 0, sid)
        b = oracle.init_default(gen)
        oracle.skipahead(gen, b, sid * oracle.stream_distance(gen, 0, 1))
        assert np.array_equal(a, b)
        assert oracle.stream_distance(gen, 0, sid) == sid * oracle.stream_distance(gen, 0, 1)


def test_stream_init_from_explicit_base(oracle):
    gen = 1
    base = oracle.seed(gen, 777)
    a = oracle.init_stream(gen, 0, 3, base=base)
    b = base.copy()
    oracle.skipahead(gen, b, 3 * 2**127)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("gen", range(11))
def test_conversions(oracle, gen):
    st = oracle.seed(gen, 2024)
    w = oracle.generate(gen, st.copy(), 50000)
    f32 = oracle.generate(gen, st.copy(), 50000, oracle.F32)
    f64 = oracle.generate(gen, st.copy(), 50000, oracle.F64)
    assert np.array_equal(f32, (w >> 8).astype(np.float32) * np.float32(2.0**-24))
    assert f32.min() >= 0.0 and f32.max() < 1.0
    if gen == 1:
        assert np.array_equal(f64, w.astype(np.float64) * np.float64(1.0 / 4294967088.0))
        assert f64.min() > 0.0
    else:
        assert np.array_equal(f64, w.astype(np.float64) * 2.0**-32)
    assert f64.max() < 1.0


@pytest.mark.parametrize("gen", range(11))
def test_generate_in_pieces_equals_one_call(oracle, gen):
    st = oracle.seed(gen, 31)
    ref = oracle.generate(gen, st.copy(), 3000)
    s = st.copy()
    parts = [oracle.generate(gen, s, n) for n in [1, 2, 623, 624, 625, 7, 1118]]
    assert np.array_equal(np.concatenate(parts), ref)


def test_bad_arguments(oracle):
    assert oracle.lib.or_state_bytes(11) < 0
    assert oracle.lib.or_block_log2(0, 5) < 0
    st = oracle.new_state(0)
    assert oracle.lib.or_generate(0, oracle._ptr(st), 3, None, 0) < 0
