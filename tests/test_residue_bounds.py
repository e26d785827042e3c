"""The integer facts the GM/GQ device steps rely on (paper, equation rec1;
k, q, g of Table 2), checked in exact integer arithmetic on the CPU.

After the collapse the kernels keep each element as a redundant residue z in
[0, zmax] (some shifted by a constant: the exact value is z + shift mod the
prime m) and never reduce it fully: each step forms a non-negative product
sum that fits its machine word, folds it once with 2^e = c (mod m), and the
digit is read off z directly.  For every form this test checks, on random
and boundary inputs: the sum and its pieces fit the widths the kernels use,
the result stays in [0, zmax], it is congruent to k x - q x_prev (mod m), and
the digit equals floor(2^v x / m) of the exact value.  The v = 3/4 digit
formula is also checked on every value within 64 of each place where either
the exact digit or one of the formula's shifts changes.

GM19 instead keeps a centred residue in FP32 and steps it with FMAs: that
form is checked exhaustively over every product sum its inputs can give,
with the FP32 roundings emulated exactly in integers."""
import random

import numpy as np
import pytest

M32 = (1 << 32) - 1
M64 = (1 << 64) - 1


def fits(x, bits):
    assert 0 <= x < (1 << bits), (x, bits)
    return x


def gm29_step(zc, zp):
    g = (1 << 29) - 3
    a = fits(2 * zc + (g + 19) - zp, 31)
    return 2 * (a & ((1 << 28) - 1)) + 3 * (a >> 28)


def gm31_step(zc, zp):
    g = (1 << 31) - 1
    t = fits(11 * zc + 14 * fits(2 * g - zp, 32), 64)
    return (t & g) + (t >> 31)


def gm61_step(zc, zp):
    g = (1 << 61) - 1
    s = fits(2 * g - zp, 62)
    b = fits((zc >> 32) * 24 + (s >> 32) * 74, 38)
    a = fits((zc & M32) * 24 + (s & M32) * 74 + (b >> 29), 64)
    hi = fits((a >> 32) + (b & ((1 << 29) - 1)), 32)
    return (hi << 32) | (a & M32)


def gq1_step(zc, zp):
    p = (1 << 29) - 3
    u = fits(zc + 6 * fits(p + 205 - zp, 32), 32)
    return ((u << 3) & ((1 << 29) - 1)) + 3 * (u >> 26)


def gq34_step(zc, zp):
    p = (1 << 29) - 3
    u = fits(zc + 6 * fits(p + 11184779 - zp, 32), 32)
    return ((u << 3) & ((1 << 29) - 1)) + 3 * (u >> 26)


def gm55_step(zc, zp):
    p = (1 << 51) - 129
    s = fits((zc << 8) + 176 * (2 * p - zp), 61)
    return (s & ((1 << 51) - 1)) + 129 * (s >> 51)


P19, P29, P31, P61 = (1 << 19) - 1, (1 << 29) - 3, (1 << 31) - 1, (1 << 61) - 1
P51 = (1 << 51) - 129


def v1_digit(lo, hi):
    return lambda z: int(lo <= z < hi)


def gq1_digit(z):
    return int(((z - 240) & M32) >= 268435455)


def gq_digit(v):
    def d(z):
        d0 = z >> (29 - v)
        return (((z + ((3 * d0 + 3 + (37 << v)) >> v)) & M32) >> (29 - v)) & ((1 << v) - 1)
    return d


def gm55_digit(z):
    num = (z << 4) & M64
    d0 = num >> 51
    return (d0 + ((d0 + 1) * P51 <= num)) & 15


FORMS = [
    # name, m, k, q, v, shift (exact = z + shift), zmax, step, digit
    ("GM29", P29, 4, 2, 1, 38, P29 + 19, gm29_step, v1_digit((P29 + 1) // 2 - 38, P29 - 38)),
    ("GM31", P31, 11, 14, 1, 0, P31 + 39, gm31_step, v1_digit(1 << 30, P31)),
    ("GM61", P61, 24, 74, 1, 0, (1 << 61) + 98 * (1 << 32) - 1, gm61_step, v1_digit(1 << 60, P61)),
    ("GQ58.1", P29, 8, 48, 1, -240, P29 + 184, gq1_step, gq1_digit),
    ("GQ58.3", P29, 8, 48, 3, 37, P29 + 166, gq34_step, gq_digit(3)),
    ("GQ58.4", P29, 8, 48, 4, 37, P29 + 166, gq34_step, gq_digit(4)),
    ("GM55", P51, 256, 176, 4, 0, P51 + 78560, gm55_step, gm55_digit),
]


def exact(m, shift, z):
    return (z + shift) % m


def true_digit(m, v, x):
    return (x << v) // m


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_step_range_congruence_digit(form):
    name, m, k, q, v, shift, zmax, step, digit = form
    rnd = random.Random(1307)
    edges = [z for z in (list(range(300)) + [m - i for i in range(1, 300)] + [m + i for i in range(300)]
                         + [zmax - i for i in range(300)]) if 0 <= z <= zmax]
    for _ in range(20000):
        zc = rnd.choice(edges) if rnd.random() < 0.3 else rnd.randint(0, zmax)
        zp = rnd.choice(edges) if rnd.random() < 0.3 else rnd.randint(0, zmax)
        z = step(zc, zp)
        assert 0 <= z <= zmax, (name, zc, zp, z)
        x = (k * exact(m, shift, zc) - q * exact(m, shift, zp)) % m
        assert exact(m, shift, z) == x, (name, zc, zp)
        assert digit(z) == true_digit(m, v, x), (name, z)
    for z in edges:
        assert digit(z) == true_digit(m, v, exact(m, shift, z)), (name, z)


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_long_runs_from_exact_states(form):
    name, m, k, q, v, shift, zmax, step, digit = form
    rnd = random.Random(58)
    for _ in range(50):
        xc, xp = rnd.randrange(m), rnd.randrange(m)
        zc, zp = (xc - shift) % m, (xp - shift) % m   # the kernels' conversion into the stored form
        for _ in range(400):
            z = step(zc, zp)
            x = (k * xc - q * xp) % m
            assert exact(m, shift, z) == x and digit(z) == true_digit(m, v, x), name
            zp, zc, xp, xc = zc, z, xc, x


@pytest.mark.parametrize("v", [3, 4])
def test_gq_digit_near_every_boundary(v):
    """Around every exact digit boundary ceil(j p / 2^v) (in stored form) and
    every multiple of 2^(29-v) (where d0 and the final shift change)."""
    m, shift, zmax = P29, 37, P29 + 166
    d = gq_digit(v)
    centres = set()
    for j in range(0, (1 << v) + 1):
        centres.add((-(-j * m // (1 << v)) - shift) % m)
        centres.add(j << (29 - v))
    centres |= {0, m, zmax}
    for c in centres:
        for z in range(max(0, c - 64), min(zmax, c + 64) + 1):
            assert d(z) == true_digit(m, v, exact(m, shift, z)), (v, z)


def fold_max(t_max, e, c, mult=1):
    """max over 0 <= t <= t_max of mult (t mod 2^e) + c floor(t / 2^e)."""
    hi, lo = t_max >> e, t_max & ((1 << e) - 1)
    best = mult * lo + c * hi
    if hi:
        best = max(best, mult * ((1 << e) - 1) + c * (hi - 1))
    return best


def test_worst_case_bounds():
    """Every fold's largest possible result over all stored inputs in
    [0, zmax] stays within zmax (the product sums are largest at zp = 0)."""
    z = {f[0]: f[6] for f in FORMS}
    assert fold_max(2 * z["GM29"] + P29 + 19, 28, 3, 2) <= z["GM29"]
    assert fold_max(11 * z["GM31"] + 14 * 2 * P31, 31, 1) <= z["GM31"]
    u1 = z["GQ58.1"] + 6 * (P29 + 205)
    assert u1 < 1 << 32 and fold_max(u1, 26, 3, 8) <= z["GQ58.1"]
    u3 = z["GQ58.3"] + 6 * (P29 + 11184779)
    assert u3 < 1 << 32 and fold_max(u3, 26, 3, 8) <= z["GQ58.3"]
    s55 = (z["GM55"] << 8) + 176 * 2 * P51
    assert s55 < 1 << 61 and fold_max(s55, 51, 129) <= z["GM55"]
    # GM61: B < 2^38 gives floor(B / 2^29) < 2^9; A below 98 2^32 + 2^9; the
    # result adds at most 2^29 - 1 to A's high word
    zc_hi, s_hi = z["GM61"] >> 32, (2 * P61) >> 32
    b_max = 24 * zc_hi + 74 * s_hi
    a_max = 98 * M32 + (b_max >> 29)
    r_max = (((a_max >> 32) + (1 << 29) - 1) << 32) | M32
    assert b_max < 1 << 38 and r_max <= z["GM61"] and 2 * P61 - z["GM61"] > 0


# ---------------------------------------------------------------- GM19, FP32
# The kernel's GM19 step on centred residues r in [-(g-1)/2, (g-1)/2] held as
# floats: t = fma(15, zc, -28 zp); K = fma(t, RN(1/g), 1.5 2^23); k = K -
# 1.5 2^23; r = fma(-k, g, t); digit = (r < 0).
G19 = P19
HALF19 = (G19 - 1) // 2
ROUND = 3 << 22          # 1.5 2^23
INV_NUM = (1 << 19) + 1  # RN_f32(1/g) = INV_NUM / 2^38 (pinned below)


def test_gm19_f32_inverse_constant():
    """the float nearest 1/g is 2^-19 (1 + 2^-19), within 2^-38 relative"""
    inv = np.float32(1.0) / np.float32(G19)
    assert float(inv) == INV_NUM / 2.0 ** 38
    assert abs(float(inv) * G19 - 1.0) < 2.0 ** -37


def gm19_f32_from_t(t):
    """The kernel's step from the product sum t (int64 array), every FP32
    operation emulated exactly: returns (k, r, digit)."""
    # t = 15 zc - 28 zp and the product 28 zp are exact FP32 values
    assert np.all(np.abs(t) < 1 << 24)
    # K = RN_f32(t / 2^38 * INV_NUM + ROUND): the exact value lies in
    # [2^23, 2^24), where FP32 spacing is 1, so K is that value rounded to
    # the nearest integer, ties to even
    num = t * INV_NUM + (ROUND << 38)
    q, rem = num >> 38, num & ((1 << 38) - 1)
    assert np.all((q >= 1 << 23) & (q + 1 < 1 << 24))
    half = 1 << 37
    K = q + (rem > half) + ((rem == half) & (q & 1))
    k = K - ROUND                       # exact: integers below 2^24
    assert np.all(np.abs(k * G19) < 1 << 24)
    r = t - k * G19                     # fma(-k, g, t): exact
    return k, r, r < 0


def test_gm19_f32_step_exhaustive():
    """Every product sum t of two centred residues: k is the nearest integer
    to t / g, r = t - k g is the centred residue of t, and the digit read off
    its sign is floor(2 x / g) of x = t mod g."""
    tmax = 15 * HALF19 + 28 * HALF19
    for lo in range(-tmax, tmax + 1, 1 << 22):
        t = np.arange(lo, min(lo + (1 << 22), tmax + 1), dtype=np.int64)
        k, r, digit = gm19_f32_from_t(t)
        assert np.array_equal(k, (2 * t + G19) // (2 * G19))   # nearest: t/g is never a half-integer
        assert np.all(np.abs(r) <= HALF19)
        x = np.mod(t, G19)
        assert np.array_equal(np.mod(r, G19), x)
        assert np.array_equal(digit, (2 * x) // G19 == 1)


def test_gm19_f32_runs_and_conversions():
    """Runs from exact states through the kernel's conversions and steps."""
    rnd = random.Random(19)
    for x0 in [0, 1, HALF19, HALF19 + 1, G19 - 1] + [rnd.randrange(G19) for _ in range(40)]:
        xc, xp = x0, rnd.randrange(G19)
        zc = xc - (G19 if xc > HALF19 else 0)      # to_fast
        zp = xp - (G19 if xp > HALF19 else 0)
        for _ in range(300):
            t = np.array([15 * zc - 28 * zp], dtype=np.int64)
            _, r, digit = gm19_f32_from_t(t)
            x = (15 * xc - 28 * xp) % G19
            assert int(r[0]) % G19 == x and bool(digit[0]) == ((2 * x) // G19 == 1)
            zp, zc, xp, xc = zc, int(r[0]), xc, x
        assert (zc + G19 if zc < 0 else zc) == xc     # from_fast
