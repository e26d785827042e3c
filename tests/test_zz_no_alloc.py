"""The allocation-free fill (prand_generate_noalloc) against prand_generate,
through the C ABI: the same host state filled by both entry points gives the
same outputs and the same advanced state, call after call (the second call
of each pair is shorter than the first and starts where the first ended).
Lengths above what the static scratch array holds with prand_generate's own
section plan make the allocation-free call plan fewer, longer sections; the
result must not change."""
import numpy as np
import pytest
import torch

from paper_1307_5869_amd import prand as P

pytestmark = pytest.mark.gpu

TDT = {P.U32: torch.int32, P.F32: torch.float32, P.F64: torch.float64}


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def _pair(ctx, gen, dtype, state, n):
    """Fill n values from copies of `state` with both entry points; return
    (outputs equal, states after each call)."""
    sa, sb = state.copy(), state.copy()
    oa = torch.empty(n, dtype=TDT[dtype], device="cuda")
    ob = torch.full((n,), -1, dtype=TDT[dtype], device="cuda")
    ctx.generate(gen, sa, dtype, oa, n)
    ctx.generate_noalloc(gen, sb, dtype, ob, n)
    torch.cuda.synchronize()
    same = bool(torch.equal(oa.view(torch.uint8), ob.view(torch.uint8)))
    return same, sa, sb, oa


def test_mt19937_needs_its_tables_first():
    c = P.Context(0)
    try:
        st = c.init_default(P.MRG32K3A)
        out = torch.empty(1000, dtype=torch.int32, device="cuda")
        # a generator without lazily built tables works at once
        c.generate_noalloc(P.MRG32K3A, st, P.U32, out, 1000)
        mt = c.init_default(P.MT19937)
        with pytest.raises(P.PrandError) as ei:
            c.generate_noalloc(P.MT19937, mt, P.U32, out, 1000)
        assert ei.value.code == P.ENOTREADY
        c.init_stream(P.MT19937, P.SEQ_DEFAULT, 3)   # builds the MT19937 tables
        c.generate_noalloc(P.MT19937, mt, P.U32, out, 1000)
    finally:
        c.close()


@pytest.mark.parametrize("gen", range(P.NUM_GENERATORS))
@pytest.mark.parametrize("dtype", [P.U32, P.F32, P.F64])
def test_noalloc_equals_generate(ctx, oracle, gen, dtype):
    st = ctx.init_stream(gen, P.SEQ_DEFAULT, 987654321)
    n1 = 3_000_017 if gen == P.MT19937 else 1_000_003
    n2 = 77_777
    for n in (n1, n2):
        same, sa, sb, oa = _pair(ctx, gen, dtype, st, n)
        assert same, (P.NAMES[gen], dtype, n)
        assert np.array_equal(sa, sb), (P.NAMES[gen], dtype, n)
        st = sa
    # the second call's values and state from the oracle, continued from the
    # oracle's own state after n1 values
    o = oracle.init_stream(gen, 0, 987654321)
    oracle.generate(gen, o, n1, dtype)
    ref = oracle.generate(gen, o, n2, dtype)
    got = oa.cpu().numpy().view(ref.dtype)
    assert np.array_equal(got, ref)
    assert np.array_equal(o, st)


@pytest.mark.parametrize("gen", range(P.NUM_GENERATORS))
def test_noalloc_beyond_the_default_plan(ctx, gen):
    """Lengths whose prand_generate plan holds more sections than the static
    array (MT19937 above 1662 * 2^18 outputs, the others above a few 10^7):
    the allocation-free call uses longer sections, with the same result."""
    st = ctx.init_stream(gen, P.SEQ_DEFAULT, 5)
    n1 = 450_000_001 if gen == P.MT19937 else 50_000_017
    for n in (n1, 1_234_567):
        same, sa, sb, _ = _pair(ctx, gen, P.U32, st, n)
        assert same, (P.NAMES[gen], n)
        assert np.array_equal(sa, sb), (P.NAMES[gen], n)
        st = sa
    torch.cuda.empty_cache()


def test_noalloc_rejects_and_degenerate(ctx):
    st = ctx.init_default(P.LFSR113)
    before = st.copy()
    out = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(P.PrandError) as ei:
        ctx.generate_noalloc(P.LFSR113, st, P.U32, out, (1 << 40) + 1)
    assert ei.value.code == P.ERANGE
    ctx.generate_noalloc(P.LFSR113, st, P.U32, out, 0)
    assert np.array_equal(st, before)
    with pytest.raises(P.PrandError) as ei:
        ctx.generate_noalloc(11, st, P.U32, out, 8)
    assert ei.value.code == P.EINVAL
    with pytest.raises(P.PrandError) as ei:
        ctx.generate_noalloc(P.LFSR113, st, 3, out, 8)
    assert ei.value.code == P.EINVAL
    ctx.generate_noalloc(P.LFSR113, st, P.U32, out, 8)
    ref = before.copy()
    ref_out = torch.empty(8, dtype=torch.int32, device="cuda")
    ctx.generate(P.LFSR113, ref, P.U32, ref_out, 8)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out) and np.array_equal(st, ref)
