"""Pins of the oracle's MRG32K3A against the paper's matrices A, B (section on
jumping ahead for MRG32K3A), its Table 2 period, brute force and number-theoretic
facts.  The paper prints no output values for MRG32K3A, so value parity rests on
the definition itself (matrices + output reading)."""
import numpy as np
import pytest
import sympy

from oracle.oracle import to_limbs  # noqa: F401  (import check)

MRG = 1
M1 = 2**32 - 209
M2 = 2**32 - 22853
A = [[0, 1403580, -810728], [1, 0, 0], [0, 1, 0]]
B = [[527612, 0, -1370589], [1, 0, 0], [0, 1, 0]]
I3 = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]


def words(st):
    w = st.view(np.uint32)
    return [int(v) for v in w[:3]], [int(v) for v in w[3:6]]


def mat_vec(M, v, m):
    return [sum(M[i][k] * v[k] for k in range(3)) % m for i in range(3)]


def mat_mul(P, Q, m):
    return [[sum(P[i][k] * Q[k][j] for k in range(3)) % m for j in range(3)] for i in range(3)]


def test_moduli_prime():
    assert sympy.isprime(M1) and sympy.isprime(M2)


def test_seed_12345_fills_all_six_words(oracle):
    x, y = words(oracle.seed(MRG, 12345))
    assert x == [12345] * 3 and y == [12345] * 3
    assert np.array_equal(oracle.init_default(MRG), oracle.seed(MRG, 12345))


def test_step_is_the_papers_matrix_product(oracle):
    st = oracle.seed(MRG, 2**63 + 11)       # expanded (non-trivial) seed
    for _ in range(50):
        x, y = words(st)
        z = int(oracle.generate(MRG, st, 1)[0])
        x2, y2 = words(st)
        assert x2 == mat_vec(A, x, M1) and y2 == mat_vec(B, y, M2)
        # output reading: difference modulo m1, taken in [1, m1]
        assert z == ((x2[0] - y2[0]) % M1 or M1)


@pytest.mark.parametrize("mat,m", [(A, M1), (B, M2)])
def test_matrices_primitive(oracle, mat, m):
    """A^(m^3-1) = I and no proper divisor of m^3-1 gives I: the period of
    each component is m^3-1, as the Table 2 period requires."""
    order = m**3 - 1
    assert oracle.mat3_pow(mat, m, order) == I3
    for r in sympy.factorint(order):
        assert oracle.mat3_pow(mat, m, order // r) != I3


def test_table2_period(oracle):
    per = (M1**3 - 1) * (M2**3 - 1) // 2
    # Table 2 prints 3.1e57
    assert f"{per:.1e}" == "3.1e+57"


def test_matpow_equals_repeated_products_tiny_prime(oracle):
    """A 3x3 companion matrix of a primitive cubic over F_7: the oracle's
    matrix power equals repeated multiplication, and its order is 7^3-1."""
    p = 7
    found = None
    for a in range(p):
        for b in range(1, p):
            M = [[0, a, b], [1, 0, 0], [0, 1, 0]]
            P, n = M, 1
            while P != I3 and n <= p**3:
                P, n = mat_mul(P, M, p), n + 1
            if n == p**3 - 1:
                found = M
                break
        if found:
            break
    assert found is not None
    P = I3
    for n in range(0, 400):
        assert oracle.mat3_pow(found, p, n) == P
        P = mat_mul(P, found, p)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 100, 1000, 4095, 65536])
def test_jump_equals_brute_force(oracle, n):
    st = oracle.seed(MRG, 987654321987)
    j = st.copy()
    oracle.skipahead(MRG, j, n)
    b = st.copy()
    if n:
        oracle.generate(MRG, b, n)
    assert np.array_equal(j, b)
    assert np.array_equal(oracle.generate(MRG, j, 64), oracle.generate(MRG, b, 64))


def test_jump_composition(oracle):
    for a, b in [(2**76, 3 * 2**76), (10**19 * 2**127, 2**190 + 5), (12345, 2**64 - 1)]:
        s1 = oracle.init_default(MRG)
        oracle.skipahead(MRG, s1, a)
        oracle.skipahead(MRG, s1, b)
        s2 = oracle.init_default(MRG)
        oracle.skipahead(MRG, s2, a + b)
        assert np.array_equal(s1, s2)


def test_jump_by_component_period_is_identity(oracle):
    """X jumps with A^(m1^3-1) = I; Y with B^(m2^3-1) = I.  The combined state
    returns after lcm of both, which equals the Table 2 period times 2."""
    st = oracle.seed(MRG, 4242)
    j = st.copy()
    oracle.skipahead(MRG, j, (M1**3 - 1) * (M2**3 - 1))
    assert np.array_equal(j, st)


def test_outputs_and_conversions(oracle):
    st = oracle.seed(MRG, 12345)
    z = oracle.generate(MRG, st.copy(), 200000).astype(np.int64)
    assert z.min() >= 1 and z.max() <= M1
    f64 = oracle.generate(MRG, st.copy(), 200000, oracle.F64)
    assert np.array_equal(f64, z.astype(np.float64) * np.float64(1.0 / 4294967088.0))
    assert f64.min() > 0.0 and f64.max() < 1.0
    f32 = oracle.generate(MRG, st.copy(), 200000, oracle.F32)
    assert np.array_equal(f32, (z >> 8).astype(np.float32) * np.float32(2.0**-24))
    assert f32.max() < 1.0
