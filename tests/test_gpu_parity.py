"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle:
seeding, generation in every dtype, sections, jumps, block-splitting stream
initialisation, ragged sizes and degenerate cases."""
import numpy as np
import pytest
import torch

from paper_1307_5869_amd import prand as P

pytestmark = pytest.mark.gpu

GENS = list(range(11))
DTYPES = [P.U32, P.F32, P.F64]
TDT = {P.U32: torch.int32, P.F32: torch.float32, P.F64: torch.float64}
NPDT = {P.U32: np.uint32, P.F32: np.float32, P.F64: np.float64}


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def to_dev(states):
    return torch.from_numpy(np.concatenate(states)).cuda()


def from_dev(t, gen):
    a = t.cpu().numpy()
    sb = P.state_bytes(gen)
    return [a[i * sb:(i + 1) * sb] for i in range(a.size // sb)]


def out_np(t, dtype):
    return t.cpu().numpy().view(NPDT[dtype])


def gpu_generate_streams(ctx, gen, states, n, dtype):
    d = to_dev(states)
    out = torch.empty(len(states) * n, dtype=TDT[dtype], device="cuda")
    ctx.generate_streams(gen, d, len(states), n, dtype, out)
    torch.cuda.synchronize()
    return out_np(out, dtype), from_dev(d, gen)


SEEDS = [0, 1, 127, 128, 12345, 2**32 - 1, 2**32, 2**63 + 5, 2**64 - 1]


@pytest.mark.parametrize("gen", GENS)
def test_seed_and_default_match_oracle(ctx, oracle, gen):
    for s in SEEDS:
        assert np.array_equal(ctx.seed(gen, s), oracle.seed(gen, s)), s
    assert np.array_equal(ctx.init_default(gen), oracle.init_default(gen))
    seeds = torch.tensor(np.array(SEEDS, dtype=np.uint64).view(np.int64), device="cuda")
    d = torch.zeros(len(SEEDS) * P.state_bytes(gen), dtype=torch.uint8, device="cuda")
    ctx.seed_dev(gen, seeds, len(SEEDS), d)
    torch.cuda.synchronize()
    for s, st in zip(SEEDS, from_dev(d, gen)):
        assert np.array_equal(st, oracle.seed(gen, s))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("gen", GENS)
@pytest.mark.parametrize("count,n", [(1, 1), (3, 3), (37, 1000), (5, 4101), (64, 257), (33, 4132), (130, 8192),
                                     (7, 20000)])
def test_generate_streams(ctx, oracle, gen, dtype, count, n):
    states = [oracle.seed(gen, 1000 + 7 * i) for i in range(count)]
    got, got_states = gpu_generate_streams(ctx, gen, states, n, dtype)
    for i, st in enumerate(states):
        ref = oracle.generate(gen, st, n, dtype)
        np.testing.assert_array_equal(got[i * n:(i + 1) * n], ref, err_msg=f"stream {i}")
        assert np.array_equal(got_states[i], st), f"state {i}"


def test_gm19_states_at_the_centred_range_edges(ctx, oracle):
    """GM19 steps on centred residues in [-(g-1)/2, (g-1)/2]: states whose
    elements sit where the conversion into that form changes side (and at
    the ends of [0, g)), in every dtype, with a ragged last block."""
    g = (1 << 19) - 1
    edge = [0, 1, 2, (g - 1) // 2 - 1, (g - 1) // 2, (g + 1) // 2, (g + 1) // 2 + 1, g - 2, g - 1]
    rng = np.random.default_rng(19)
    states = []
    for i in range(40):
        st = oracle.seed(P.GM19, 500 + i).copy()
        st.view(np.uint64)[:64] = rng.choice(edge, 64)   # xc[32], xp[32]
        states.append(st)
    n = 3000
    for dtype in DTYPES:
        got, got_states = gpu_generate_streams(ctx, P.GM19, [st.copy() for st in states], n, dtype)
        for i, st in enumerate(states):
            ref_state = st.copy()
            ref = oracle.generate(P.GM19, ref_state, n, dtype)
            np.testing.assert_array_equal(got[i * n:(i + 1) * n], ref, err_msg=f"stream {i}")
            assert np.array_equal(got_states[i], ref_state), f"state {i}"


@pytest.mark.parametrize("gen", GENS)
def test_generate_in_pieces_continues_the_stream(ctx, oracle, gen):
    states = [oracle.seed(gen, 77 + i) for i in range(6)]
    d = to_dev(states)
    parts = []
    for n in [5, 619, 1, 700, 624, 33]:
        out = torch.empty(len(states) * n, dtype=torch.int32, device="cuda")
        ctx.generate_streams(gen, d, len(states), n, P.U32, out)
        parts.append(out_np(out, P.U32).reshape(len(states), n))
    torch.cuda.synchronize()
    got = np.concatenate(parts, axis=1)
    for i, st in enumerate(states):
        assert np.array_equal(got[i], oracle.generate(gen, st, got.shape[1]))
        assert np.array_equal(from_dev(d, gen)[i], st)


@pytest.mark.parametrize("gen", GENS)
def test_degenerate_calls(ctx, oracle, gen):
    st = [oracle.seed(gen, 5)]
    d = to_dev(st)
    out = torch.empty(8, dtype=torch.int32, device="cuda")
    ctx.generate_streams(gen, d, 1, 0, P.U32, out)        # n = 0: nothing happens
    ctx.generate_streams(gen, d, 0, 8, P.U32, out)        # count = 0
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(d, gen)[0], st[0])
    with pytest.raises(P.PrandError):
        ctx.generate_streams(gen, d, 1, 4, 3, out)         # bad dtype
    with pytest.raises(P.PrandError):
        ctx.generate_streams(gen, d, 1, 4, P.U32, None)    # no output


def distances_for(gen):
    base = [0, 1, 2, 5, 623, 624, 625, 9999, 2**40 + 3, 5 * 2**127 + 11, 2**300 + 1, 2**511 + 2**200]
    return base if gen != 0 else [0, 1, 623, 625, 100000, 2**128 + 7, 2**511]


@pytest.mark.parametrize("gen", GENS)
def test_skipahead_host(ctx, oracle, gen):
    for dist in distances_for(gen):
        st = oracle.seed(gen, 4242)
        if gen == 0:
            oracle.generate(gen, st, 100)       # start mid-block
        mine = ctx.skipahead(gen, st.copy(), dist)
        ref = oracle.skipahead(gen, st.copy(), dist)
        assert np.array_equal(mine, ref), dist


@pytest.mark.parametrize("gen", GENS)
def test_skipahead_dev_per_stream_and_shared(ctx, oracle, gen):
    rng = np.random.default_rng(gen)
    count = 24 if gen == 0 else 96
    states = [oracle.seed(gen, 900 + i) for i in range(count)]
    for i in range(0, count, 5):
        oracle.generate(gen, states[i], 17 * i)   # various offsets / indices
    dists = [int(rng.integers(0, 2**63)) >> int(rng.integers(0, 60)) for _ in range(count)]
    if gen != 0:
        dists[1] = 2**200 + 12345
        dists[2] = 2**511
    d = to_dev(states)
    L = torch.tensor(np.stack([P.limbs(x) for x in dists]).view(np.int64), device="cuda")
    ctx.skipahead_dev(gen, d, count, L, 8, True)
    torch.cuda.synchronize()
    for i, st in enumerate(from_dev(d, gen)):
        assert np.array_equal(st, oracle.skipahead(gen, states[i].copy(), dists[i])), i
    # one shared distance of 2 limbs
    d = to_dev(states)
    shared = 3 * 2**70 + 99
    L2 = torch.tensor(P.limbs(shared)[:2].view(np.int64), device="cuda")
    ctx.skipahead_dev(gen, d, count, L2, 2, False)
    torch.cuda.synchronize()
    for i, st in enumerate(from_dev(d, gen)[:8]):
        assert np.array_equal(st, oracle.skipahead(gen, states[i].copy(), shared))


VARIANTS = {g: [v for v in range(5) if P.block_log2(g, v) >= 0] for g in GENS}


@pytest.mark.parametrize("gen", GENS)
def test_init_streams_match_oracle(ctx, oracle, gen):
    ids = [0, 1, 2, 3, 10**19 - 1, 2**64 - 1, 123456789012345678]
    if gen == 0:
        # digit boundaries of the MT19937 tables: 16-bit digits below bit 48,
        # precomputed states above it
        ids = [0, 1, 10**19 - 1, 987654321, 2**64 - 1, 1 << 48, (1 << 48) - 1, 1 << 32, 65535]
    for v in VARIANTS[gen]:
        t = torch.tensor(np.array(ids, dtype=np.uint64).view(np.int64), device="cuda")
        d = torch.empty(len(ids) * P.state_bytes(gen), dtype=torch.uint8, device="cuda")
        ctx.init_streams_dev(gen, v, None, t, len(ids), d)
        torch.cuda.synchronize()
        for sid, st in zip(ids, from_dev(d, gen)):
            assert np.array_equal(st, oracle.init_stream(gen, v, sid)), (v, sid)
        assert np.array_equal(ctx.init_stream(gen, v, ids[-1]), oracle.init_stream(gen, v, ids[-1]))
    bad = [v for v in range(1, 5) if v not in VARIANTS[gen]]
    for v in bad:
        with pytest.raises(P.PrandError):
            ctx.init_stream(gen, v, 1)


@pytest.mark.parametrize("gen", GENS[1:])
def test_init_streams_byte_tables(ctx, oracle, gen):
    """Default-variant block splitting through the byte tables (one matrix
    per nonzero byte of the id): ids with one byte set at every position and
    edge values, mixed and random ids, from the default state."""
    ids = [d << (8 * j) for j in range(8) for d in (1, 2, 127, 128, 255)]
    rng = np.random.default_rng(1307)
    ids += [int(x) for x in rng.integers(0, 2**63, 8, dtype=np.int64)] + [2**63, 2**63 + 1, 0x00FF00FF00FF00FF]
    t = torch.tensor(np.array(ids, dtype=np.uint64).view(np.int64), device="cuda")
    d = torch.empty(len(ids) * P.state_bytes(gen), dtype=torch.uint8, device="cuda")
    ctx.init_streams_dev(gen, P.SEQ_DEFAULT, None, t, len(ids), d)
    torch.cuda.synchronize()
    for sid, st in zip(ids, from_dev(d, gen)):
        assert np.array_equal(st, oracle.init_stream(gen, P.SEQ_DEFAULT, sid)), hex(sid)


@pytest.mark.parametrize("consumed", [0, 100])
@pytest.mark.parametrize("gen", GENS)
def test_init_streams_from_explicit_base(ctx, oracle, gen, consumed):
    base = oracle.seed(gen, 31337)
    if consumed:
        oracle.generate(gen, base, consumed)    # a base in the middle of its sequence
    ids = [0, 5, 77, 0x0102030405060708]
    t = torch.tensor(np.array(ids, dtype=np.uint64).view(np.int64), device="cuda")
    db = torch.from_numpy(base.copy()).cuda()
    d = torch.empty(len(ids) * P.state_bytes(gen), dtype=torch.uint8, device="cuda")
    ctx.init_streams_dev(gen, 0, db, t, len(ids), d)
    torch.cuda.synchronize()
    for sid, st in zip(ids, from_dev(d, gen)):
        assert np.array_equal(st, oracle.init_stream(gen, 0, sid, base=base)), sid


@pytest.mark.parametrize("kind", ["ids", "distances"])
def test_mt19937_jump_launch_shapes_agree(ctx, oracle, kind):
    """MT19937 jumps run with 12 or 8 wavefronts per stream (coefficient
    ranges scanned apart, partial windows XORed) in launches of few streams
    and with one wavefront per stream in larger ones.  Launches of 300, 1500
    and 2500 streams over the same inputs (a prefix of one another, one launch
    of each shape) agree on every shared stream, and sampled streams of each
    launch, the first, the last and one in between, equal the oracle.  ids:
    block splitting from the default state (digit tables); distances:
    per-stream skip-ahead from states at various places in their blocks
    (ladder polynomials)."""
    gen, sb = P.MT19937, P.state_bytes(P.MT19937)
    rng = np.random.default_rng(5869)
    total = 2500
    if kind == "ids":
        ids = rng.integers(0, 2**63, total, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
        ids[:4] = [0, 1, 2**64 - 1, 1 << 48]
        dev_ids = torch.from_numpy(ids.view(np.int64)).cuda()
        bases = None
    else:
        bases = [oracle.seed(gen, 4000 + i) for i in range(5)]
        for i, b in enumerate(bases):
            oracle.generate(gen, b, [0, 1, 300, 623, 624][i])
        dists = [int(x) >> int(y) for x, y in zip(rng.integers(1, 2**63, total), rng.integers(0, 40, total))]
        dists[:3] = [0, 1, 624 * 2**12]
        limbs = torch.from_numpy(np.stack([P.limbs(x)[:2] for x in dists]).view(np.int64)).cuda()
        start = np.concatenate([bases[i % 5] for i in range(total)])
    results = {}
    for count in (300, 1500, 2500):
        if kind == "ids":
            d = torch.empty(count * sb, dtype=torch.uint8, device="cuda")
            ctx.init_streams_dev(gen, P.SEQ_DEFAULT, None, dev_ids, count, d)
        else:
            d = torch.from_numpy(start[:count * sb].copy()).cuda()
            ctx.skipahead_dev(gen, d, count, limbs, 2, True)
        torch.cuda.synchronize()
        results[count] = d.cpu().numpy()
    for count in (300, 1500):
        assert np.array_equal(results[count], results[2500][:count * sb]), count
    for count in (300, 1500, 2500):
        for i in (0, count // 2 + 1, count - 1):
            got = results[count][i * sb:(i + 1) * sb]
            if kind == "ids":
                ref = oracle.init_stream(gen, P.SEQ_DEFAULT, int(ids[i]))
            else:
                ref = oracle.skipahead(gen, bases[i % 5].copy(), dists[i])
            assert np.array_equal(got, ref), (count, i)


SECTIONED_N = {0: 3 * 2**18 + 7, 1: 300001, 2: 300001}


@pytest.mark.parametrize("dtype", [P.U32, P.F64])
@pytest.mark.parametrize("gen", GENS)
def test_generate_single_stream_sections(ctx, oracle, gen, dtype):
    n = SECTIONED_N.get(gen, 3 * 4096 + 5)
    st = oracle.seed(gen, 2718)
    if gen in (0, 9):
        oracle.generate(gen, st, 13)
    mine = st.copy()
    out = torch.empty(n, dtype=TDT[dtype], device="cuda")
    ctx.generate(gen, mine, dtype, out, n)
    ref = oracle.generate(gen, st, n, dtype)
    np.testing.assert_array_equal(out_np(out, dtype), ref)
    assert np.array_equal(mine, st)


@pytest.mark.parametrize("consumed", [0, 13, 624])
@pytest.mark.parametrize("n", [1000, 2**19, 611 + 624 * 900, 611 + 624 * 900 + 1, 3 * 2**18 + 7])
def test_mt19937_sections_leave_the_sequential_state(ctx, oracle, consumed, n):
    """The final section of a long MT19937 fill starts on a twist-block
    boundary, so the returned state is the sequential one byte for byte."""
    gen, dtype = P.MT19937, P.U32
    st = oracle.seed(gen, 99991)
    if consumed:
        oracle.generate(gen, st, consumed)
    mine = st.copy()
    out = torch.empty(n, dtype=TDT[dtype], device="cuda")
    ctx.generate(gen, mine, dtype, out, n)
    ref = oracle.generate(gen, st, n, dtype)
    np.testing.assert_array_equal(out_np(out, dtype), ref)
    assert np.array_equal(mine, st)


def test_mrg32k3a_block_split_4096_streams_full(ctx, oracle):
    """4096 streams from all-12345 seeds, stream k jumped k * 2^76; every u32
    word and its float64 conversion compared with the oracle."""
    gen, count, n = P.MRG32K3A, 4096, 4096
    base = ctx.seed(gen, 12345)
    assert np.array_equal(base, oracle.seed(gen, 12345))
    d = to_dev([base] * count)
    L = torch.tensor(np.stack([P.limbs(k * 2**76) for k in range(count)]).view(np.int64), device="cuda")
    ctx.skipahead_dev(gen, d, count, L, 8, True)
    d2 = d.clone()
    u = torch.empty(count * n, dtype=torch.int32, device="cuda")
    f = torch.empty(count * n, dtype=torch.float64, device="cuda")
    ctx.generate_streams(gen, d, count, n, P.U32, u)
    ctx.generate_streams(gen, d2, count, n, P.F64, f)
    torch.cuda.synchronize()
    U, F = out_np(u, P.U32).reshape(count, n), out_np(f, P.F64).reshape(count, n)
    assert F.min() > 0.0 and F.max() < 1.0
    for k in range(count):
        st = oracle.seed(gen, 12345)
        oracle.skipahead(gen, st, k * 2**76)
        s2 = st.copy()
        assert np.array_equal(U[k], oracle.generate(gen, st, n)), k
        assert np.array_equal(F[k], oracle.generate(gen, s2, n, P.F64)), k


@pytest.mark.parametrize("gen", [P.MRG32K3A, P.LFSR113])
def test_generate_streams_captured_then_eager(ctx, oracle, gen):
    """Many-stream generation captured into a HIP graph with a section length
    no earlier call used (no section-start table may be built under capture:
    the sections jump through the ladder), replayed three times with eager
    work and synchronisations between the replays; then the same call made
    eagerly (which builds and uses the table).  Every replay and the eager
    call continue each stream exactly as the oracle does."""
    count, n = 9, 64 * 331 + 5
    states = [oracle.init_stream(gen, 0, 1000 + i) for i in range(count)]
    d = to_dev(states)
    out = torch.empty(count * n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.generate_streams(gen, d, count, n, P.U32, out, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = np.concatenate([oracle.generate(gen, st, n) for st in states])
        np.testing.assert_array_equal(out_np(out, P.U32), ref, err_msg=f"replay {rep}")
        got = from_dev(d, gen)
        for i in range(count):
            assert np.array_equal(got[i], states[i]), (rep, i)
    del g
    ctx.generate_streams(gen, d, count, n, P.U32, out)
    torch.cuda.synchronize()
    ref = np.concatenate([oracle.generate(gen, st, n) for st in states])
    np.testing.assert_array_equal(out_np(out, P.U32), ref, err_msg="eager after capture")


def test_mt19937_whole_section_jumps(ctx, oracle):
    """Section starts as the serving loop makes them: each state jumped by a
    number of whole sections of 624 * 2^10 outputs, through the whole-block
    table from a block boundary (below 2^22 sections) and through the ladder
    otherwise (mid-block states, 2^22 sections and more).  Every state equals
    the oracle's skip-ahead by the same number of outputs, in a launch of 12
    wavefronts per stream and, repeated, of one wavefront per stream."""
    import ctypes
    gen, sb, sec = P.MT19937, P.state_bytes(P.MT19937), 624 << 10
    lib = P.load()
    f = lib.prand_internal_mt_jump_sections
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    counts = [0, 1, 2, 3, 5, 149, 255, 2**21 + 3, 2**22 - 1, 2**22, 2**40 + 7]
    starts, dists = [], []
    for i, consumed in enumerate([0, 300, 624, 1]):
        st = oracle.seed(gen, 777 + i)
        if consumed:
            oracle.generate(gen, st, consumed)
        for d in counts:
            starts.append(st.copy())
            dists.append(d)
    n = len(starts)
    refs = [oracle.skipahead(gen, s.copy(), d * sec) for s, d in zip(starts, dists)]
    for reps in (1, 3000 // n + 1):
        count = n * reps
        d_states = torch.from_numpy(np.concatenate(starts * reps)).cuda()
        d_secs = torch.tensor(np.array(dists * reps, dtype=np.uint64).view(np.int64), device="cuda")
        assert f(ctx.handle, d_states.data_ptr(), count, d_secs.data_ptr(), None) == P.OK
        torch.cuda.synchronize()
        got = d_states.cpu().numpy()
        for k in range(count):
            assert np.array_equal(got[k * sb:(k + 1) * sb], refs[k % n]), (count, k, dists[k % n])
