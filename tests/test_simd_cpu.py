"""CPU SIMD generation (section "Generation with SSE": rng_get_sse_state_
and rng_sse_generate_), host only: prand_get_simd_state / prand_simd_next /
prand_simd_fill against the oracle, on both code paths (AVX2 and the scalar
one that PRAND_SIMD_DISABLE selects), for every generator, from seeded
states, states inside a block (MT19937, GQ58.3), block-split streams (GM/GQ
composite moduli already collapsed) and freshly seeded composite states
(GM55, GQ58: exact steps before the collapse), over several buffer refills
and ragged lengths."""
import os

import numpy as np
import pytest

from paper_1307_5869_amd import prand as P

GENS = list(range(11))


def have_avx2():
    try:
        flags = open("/proc/cpuinfo").read()
    except OSError:
        return False
    return " avx2" in flags and " fma" in flags


@pytest.fixture(params=["vector", "scalar"])
def path(request, monkeypatch):
    if request.param == "scalar":
        monkeypatch.setenv("PRAND_SIMD_DISABLE", "1")
    else:
        monkeypatch.delenv("PRAND_SIMD_DISABLE", raising=False)
        if not have_avx2():
            pytest.skip("no AVX2/FMA on this host")
    return request.param


def start_states(oracle, gen):
    """(label, state) pairs covering the ways a state reaches the SIMD code"""
    out = [("seed 7", oracle.seed(gen, 7)), ("seed 2^63+1", oracle.seed(gen, 2**63 + 1))]
    st = oracle.seed(gen, 11)
    oracle.generate(gen, st, 5)
    out.append(("after 5 outputs", st))
    out.append(("stream 123456", oracle.init_stream(gen, P.SEQ_DEFAULT, 123456)))
    st = oracle.seed(gen, 13)
    oracle.skipahead(gen, st, 10**12 + 3)
    out.append(("jumped 10^12+3", st))
    return out


@pytest.mark.parametrize("gen", GENS)
def test_simd_fill_matches_oracle(oracle, gen, path):
    n = 9000 if gen <= P.LFSR113 else 2600
    for label, st in start_states(oracle, gen):
        s = P.SimdState(gen, st)
        assert s.vectorized == (path == "vector")
        got = s.fill(P.U32, n)
        np.testing.assert_array_equal(got, oracle.generate(gen, st.copy(), n), err_msg=f"{P.NAMES[gen]} {label}")


@pytest.mark.parametrize("gen", GENS)
def test_simd_next_and_fill_interleaved(oracle, gen, path):
    """single outputs, ragged fills and a copied blob continue one sequence"""
    st = oracle.seed(gen, 31337)
    s = P.SimdState(gen, st)
    parts = [np.array([s.next() for _ in range(3)], dtype=np.uint32), s.fill(P.U32, 1), s.fill(P.U32, 2047)]
    copy = P.SimdState.__new__(P.SimdState)
    copy.blob = s.blob.copy()
    parts.append(np.array([s.next() for _ in range(700)], dtype=np.uint32))
    parts.append(s.fill(P.U32, 4099))
    got = np.concatenate(parts)
    ref = oracle.generate(gen, st.copy(), got.size)
    np.testing.assert_array_equal(got, ref, err_msg=P.NAMES[gen])
    # the copy taken after 2051 outputs continues from there
    np.testing.assert_array_equal(copy.fill(P.U32, 500), ref[2051:2551], err_msg=f"{P.NAMES[gen]} copy")


@pytest.mark.parametrize("dtype", [P.F32, P.F64])
@pytest.mark.parametrize("gen", GENS)
def test_simd_conversions(oracle, gen, dtype, path):
    st = oracle.seed(gen, 2024)
    got = P.SimdState(gen, st).fill(dtype, 3001)
    np.testing.assert_array_equal(got, oracle.generate(gen, st.copy(), 3001, dtype), err_msg=P.NAMES[gen])


def test_simd_errors():
    lib = P.load()
    st = np.zeros(P.state_bytes(P.LFSR113), dtype=np.uint8)
    blob = np.zeros(lib.prand_simd_state_bytes(), dtype=np.uint8)
    assert lib.prand_get_simd_state(11, st.ctypes.data, blob.ctypes.data) == P.EINVAL
    assert lib.prand_get_simd_state(-1, st.ctypes.data, blob.ctypes.data) == P.EINVAL
    assert lib.prand_get_simd_state(P.LFSR113, None, blob.ctypes.data) == P.EINVAL
    assert lib.prand_get_simd_state(P.LFSR113, st.ctypes.data, None) == P.EINVAL
    # a blob that was never made a SIMD state
    out = np.zeros(4, dtype=np.uint32)
    assert lib.prand_simd_next(blob.ctypes.data) == 0
    assert lib.prand_simd_fill(blob.ctypes.data, P.U32, out.ctypes.data, 4) == P.EINVAL
    assert lib.prand_simd_vectorized(blob.ctypes.data) == P.EINVAL
    # bad dtype and null output on a valid state
    from oracle import Oracle

    good = P.SimdState(P.LFSR113, Oracle().seed(P.LFSR113, 5))
    assert lib.prand_simd_fill(good.blob.ctypes.data, 3, out.ctypes.data, 4) == P.EINVAL
    assert lib.prand_simd_fill(good.blob.ctypes.data, P.U32, None, 4) == P.EINVAL
    assert lib.prand_simd_fill(good.blob.ctypes.data, P.U32, None, 0) == P.OK


def test_simd_state_is_self_contained(oracle):
    """the blob holds no pointers: a byte copy moved to another buffer works"""
    st = oracle.seed(P.MT19937, 1)
    a = P.SimdState(P.MT19937, st)
    a.fill(P.U32, 1000)
    b = P.SimdState.__new__(P.SimdState)
    b.blob = np.frombuffer(bytes(a.blob), dtype=np.uint8).copy()
    np.testing.assert_array_equal(a.fill(P.U32, 2000), b.fill(P.U32, 2000))
