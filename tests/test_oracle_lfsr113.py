"""Pins of the oracle's LFSR113 against the paper's bit-level definition
(relations lfsrRel1 and lfsrOutput, section on jumping ahead for LFSR113), the
paper's 2^n table method of jumping, brute force, primitivity of the
component trinomials and the Table 2 period."""
import numpy as np
import pytest
import sympy

LFSR = 2
COMPS = [(31, 6, 18), (29, 2, 2), (28, 13, 7), (25, 3, 13)]


def top_bits(z, p):
    """x_0..x_{p-1}: the top p bits of a 32-bit word, most significant first."""
    return [(z >> (31 - i)) & 1 for i in range(p)]


def bit_sequence(x0, p, q, length):
    """x_n = x_{n-p} + x_{n-p+q} mod 2 (relation lfsrRel1)."""
    x = list(x0)
    while len(x) < length:
        n = len(x)
        x.append(x[n - p] ^ x[n - p + q])
    return x


def word_at(x, start):
    """sum_{i=1..32} x_{start+i-1} 2^{-i} scaled by 2^32 (relation lfsrOutput)."""
    w = 0
    for i in range(32):
        w = (w << 1) | x[start + i]
    return w


@pytest.mark.parametrize("p,q,s", COMPS + [(20, 3, 2)])
def test_word_step_is_the_bit_recurrence(oracle, p, q, s):
    rng = np.random.default_rng(p)
    for _ in range(20):
        z = int(rng.integers(1, 2**32))
        if not (z >> (32 - p)):
            continue
        x = bit_sequence(top_bits(z, p), p, q, s * 60 + 40)
        for n in range(1, 50):
            z = oracle.lfsr_comp_step(z, p, q, s)
            assert z == word_at(x, n * s)


def test_output_is_xor_of_components(oracle):
    st = oracle.seed(LFSR, 987654)
    z = [int(v) for v in st.view(np.uint32)]
    out = oracle.generate(LFSR, st, 40)
    for n in range(40):
        z = [oracle.lfsr_comp_step(z[c], *COMPS[c]) for c in range(4)]
        assert out[n] == z[0] ^ z[1] ^ z[2] ^ z[3]


def test_seed_constraints_and_default(oracle):
    assert list(oracle.init_default(LFSR).view(np.uint32)) == [12345] * 4
    for seed in [0, 1, 127, 2**32, 2**64 - 1]:
        z = oracle.seed(LFSR, seed).view(np.uint32)
        for c, (p, _, _) in enumerate(COMPS):
            assert int(z[c]) >> (32 - p) != 0


def test_low_seed_bits_irrelevant(oracle):
    """Only the top p bits of a component seed enter the sequence (s+q <= 2p-32)."""
    st = oracle.seed(LFSR, 5555555)
    alt = st.copy()
    w = alt.view(np.uint32)
    for c, (p, _, _) in enumerate(COMPS):
        w[c] ^= np.uint32((1 << (32 - p)) - 1)
    assert np.array_equal(oracle.generate(LFSR, st, 100), oracle.generate(LFSR, alt, 100))


@pytest.mark.parametrize("p,q,s", COMPS)
def test_trinomials_primitive_and_component_period(oracle, p, q, s):
    x = sympy.symbols("x")
    poly = sympy.Poly(x**p + x**q + 1, x, modulus=2)
    assert poly.is_irreducible
    order = 2**p - 1
    z = oracle.lfsr_comp_step(0xDEADBEEF, p, q, s)       # a consistent state
    assert oracle.lfsr_comp_jump(z, p, q, s, order) == z
    for r in sympy.factorint(order):
        assert oracle.lfsr_comp_jump(z, p, q, s, order // r) != z


def test_table2_period():
    per = 1
    for p, _, _ in COMPS:
        per *= 2**p - 1
    assert f"{per:.1e}" == "1.0e+34"


def test_tiny_variant_brute_force_period(oracle):
    """(p,q,s) = (20,3,2): x^20+x^3+1 is primitive, so the brute-force period
    of the word sequence is 2^20-1."""
    p, q, s = 20, 3, 2
    z0 = oracle.lfsr_comp_step(0x12345678, p, q, s)
    z, n = oracle.lfsr_comp_step(z0, p, q, s), 1
    while z != z0:
        z, n = oracle.lfsr_comp_step(z, p, q, s), n + 1
    assert n == 2**20 - 1
    assert oracle.lfsr_comp_jump(z0, p, q, s, n) == z0


@pytest.mark.parametrize("p,q,s", COMPS)
def test_jump_equals_brute_force(oracle, p, q, s):
    z0 = 0x9E3779B9
    z = z0
    for n in range(0, 300):
        assert oracle.lfsr_comp_jump(z0, p, q, s, n) == z
        z = oracle.lfsr_comp_step(z, p, q, s)


def paper_table_jump_word(z0, p, q, s, n):
    """The paper's method for the word u_{2^n}: 32 tables, one per starting
    bit i, each with rows r = 0..n holding x'_{2^r p} .. x'_{2^r (2p-1)} of the
    shifted sequence x'_j = x_{j+i}; row r follows from earlier entries by
    x_{2^r (p+l)} = x_{2^r l} + x_{2^r (l+q)} (relation lfsrRel2)."""
    base = bit_sequence(top_bits(z0, p), p, q, 32 + 2 * p)
    word = 0
    for i in range(32):
        xs = base[i:i + p]                       # x'_0 .. x'_{p-1}
        x_first = bit_sequence(xs, p, q, 2 * p)  # row 0 = x'_p .. x'_{2p-1}
        rows = [x_first[p:2 * p]]

        def value(r, j):
            """x'_{2^r j} for 0 <= j < 2p using rows 0..r."""
            if j == 0:
                return xs[0]
            while j < p:                         # x'_{2^r j} = x'_{2^(r-1) 2j}
                if r == 0:
                    return xs[j] if j < p else rows[0][j - p]
                r, j = r - 1, 2 * j
            return rows[r][j - p]

        for r in range(1, n + 1):
            row = []
            for l in range(p):
                a = value(r, l) if l > 0 else xs[0]
                lq = l + q
                b = row[lq - p] if lq >= p else value(r, lq)
                row.append(a ^ b)
            rows.append(row)
        # x'_{s 2^n}: find j with s 2^j in [p, 2p)
        j, t = 0, s
        while t < p:
            t, j = 2 * t, j + 1
        bit = rows[n - j][t - p] if n >= j else None
        if bit is None:
            bit = bit_sequence(xs, p, q, s * 2**n + 1)[s * 2**n]
        word = (word << 1) | bit
    return word


@pytest.mark.parametrize("p,q,s", COMPS)
def test_jump_matches_papers_table_method(oracle, p, q, s):
    z0 = 0xC0FFEE11 | (1 << 31)
    for n in [0, 1, 2, 5, 6, 10, 33, 64, 100, 127]:
        assert oracle.lfsr_comp_jump(z0, p, q, s, 2**n) == paper_table_jump_word(z0, p, q, s, n)


def test_generator_jump_equals_brute_force(oracle):
    st = oracle.seed(LFSR, 31337)
    for n in [0, 1, 2, 77, 1000, 65535]:
        j = st.copy()
        oracle.skipahead(LFSR, j, n)
        b = st.copy()
        if n:
            oracle.generate(LFSR, b, n)
        assert np.array_equal(oracle.generate(LFSR, j, 50), oracle.generate(LFSR, b, 50))


def test_jump_composition(oracle):
    for a, b in [(2**34, 5 * 2**34), (2**80 * 12345, 2**100 + 1)]:
        s1 = oracle.init_default(LFSR)
        oracle.skipahead(LFSR, s1, a)
        oracle.skipahead(LFSR, s1, b)
        s2 = oracle.init_default(LFSR)
        oracle.skipahead(LFSR, s2, a + b)
        assert np.array_equal(s1, s2)
