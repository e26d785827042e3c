"""Host-array generation (prand_generate_array, the paper's
rng_generate_array_) and mixing the CPU and GPU interfaces on one stream
(section "Function call interface": a generator advanced on the CPU and
continued on the GPU from the same state, and back).

The CPU interface here is include/prand_device.h compiled for the host (the
test-side loop in tests/devapi/user_kernel.hip); the GPU side is the library.
"""
import numpy as np
import pytest

import devapi_lib
from paper_1307_5869_amd import prand as P

pytestmark = pytest.mark.gpu

NPDT = {P.U32: np.uint32, P.F32: np.float32, P.F64: np.float64}


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def host_advance(gen, dtype, state, n):
    """n values drawn on the CPU with the header's host build; state advanced"""
    lib = devapi_lib.load()
    out = np.empty(n, dtype=NPDT[dtype])
    assert lib.hostapi_draw(gen, dtype, state.ctypes.data, 1, n, out.ctypes.data) == 0
    return out


@pytest.mark.parametrize("gen", range(11))
@pytest.mark.parametrize("dtype", [P.U32, P.F32, P.F64])
def test_generate_array_matches_oracle(ctx, oracle, gen, dtype):
    for seed, n in ((3, 1), (5, 999), (8, 70001)):
        st = oracle.seed(gen, seed)
        if gen in (P.MT19937, P.GQ58X3):
            oracle.generate(gen, st, 5)       # start inside a block
        mine = st.copy()
        got = ctx.generate_array(gen, mine, dtype, n)
        np.testing.assert_array_equal(got, oracle.generate(gen, st, n, dtype), err_msg=f"{P.NAMES[gen]} n {n}")
        assert np.array_equal(mine, st)


@pytest.mark.parametrize("gen", [P.MT19937, P.MRG32K3A, P.LFSR113, P.GM55, P.GQ58X3])
def test_generate_array_in_chunks(ctx, oracle, gen):
    """More than one 2^26-value chunk: the whole array equals one device
    fill of the same state, and the values around the chunk boundary and
    at the end equal the oracle's"""
    import torch

    n = (1 << 26) + 12345
    st = oracle.seed(gen, 4242)
    a = st.copy()
    got = ctx.generate_array(gen, a, P.U32, n)
    b = st.copy()
    dev = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.generate(gen, b, P.U32, dev, n)
    torch.cuda.synchronize()
    assert np.array_equal(got, dev.cpu().numpy().view(np.uint32))
    assert np.array_equal(a, b)
    for at in (0, (1 << 26) - 100, n - 200):
        o = oracle.skipahead(gen, st.copy(), at)
        np.testing.assert_array_equal(got[at:at + 200], oracle.generate(gen, o, 200), err_msg=f"at {at}")
    o = st.copy()
    oracle.skipahead(gen, o, n)
    if gen != P.MT19937:      # a jumped MT19937 window is a canonical form of the same point
        assert np.array_equal(a, o)
    assert np.array_equal(oracle.generate(gen, a.copy(), 1300), oracle.generate(gen, o, 1300))


@pytest.mark.parametrize("gen", range(11))
def test_cpu_then_gpu_then_cpu(ctx, oracle, gen):
    """Advance on the CPU, continue on the GPU from the same state (host
    array and device array), then on the CPU again: the concatenation is
    the sequential stream"""
    import torch

    st = oracle.init_stream(gen, 0, 12345) if gen != P.MT19937 else oracle.seed(gen, 12345)
    ref_state = st.copy()
    m1, m2, m3, m4 = 777, 5003, 20000, 1001
    s = st.copy()
    part1 = host_advance(gen, P.U32, s, m1)
    part2 = ctx.generate_array(gen, s, P.U32, m2)
    dev = torch.empty(m3, dtype=torch.int32, device="cuda")
    ctx.generate(gen, s, P.U32, dev, m3)
    torch.cuda.synchronize()
    part3 = dev.cpu().numpy().view(np.uint32)
    part4 = host_advance(gen, P.U32, s, m4)
    ref = oracle.generate(gen, ref_state, m1 + m2 + m3 + m4)
    np.testing.assert_array_equal(np.concatenate([part1, part2, part3, part4]), ref)
    assert np.array_equal(s, ref_state)


def test_generate_array_degenerate(ctx, oracle):
    st = oracle.seed(P.LFSR113, 1)
    before = st.copy()
    assert ctx.generate_array(P.LFSR113, st, P.U32, 0).size == 0
    assert np.array_equal(st, before)
    small = np.zeros(4, dtype=np.uint32)
    with pytest.raises(P.PrandError) as ei:
        ctx._call("prand_generate_array", P.LFSR113, P._ptr(st), P.U32, P._ptr(small), (1 << 40) + 1)
    assert ei.value.code == P.ERANGE
    with pytest.raises(P.PrandError) as ei:
        ctx._call("prand_generate_array", P.LFSR113, P._ptr(st), P.U32, None, 5)
    assert ei.value.code == P.EINVAL
    assert np.array_equal(st, before)
