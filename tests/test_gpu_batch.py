"""Batched launch: every task's output and advanced state equal
the oracle's sequential generation and the plain per-stream launches, for
mixed generators, dtypes and uneven lengths, across configurations and HIP
graph replays."""
import numpy as np
import pytest
import torch

from paper_1307_5869_amd import prand as P
from paper_1307_5869_amd import workloads as W

pytestmark = pytest.mark.gpu

TDT = {P.U32: torch.int32, P.F32: torch.float32, P.F64: torch.float64}
NPDT = {P.U32: np.uint32, P.F32: np.float32, P.F64: np.float64}


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def make_tasks(oracle, specs, seed0=500):
    """specs: list of (gen, dtype, n) -> device buffers + oracle references."""
    tasks, refs = [], []
    for k, (gen, dt, n) in enumerate(specs):
        st = oracle.seed(gen, seed0 + k)
        if gen in (0, 9) and k % 3 == 1:
            oracle.generate(gen, st, 5 + k % 7)   # start inside a block
        sin = torch.from_numpy(st.copy()).cuda()
        # garbage in the output state: every byte of the blob must be written
        sout = torch.full_like(sin, 0xA5)
        out = torch.empty(max(n, 1), dtype=TDT[dt], device="cuda")
        ref_state = st.copy()
        ref = oracle.generate(gen, ref_state, n, dt) if n else np.empty(0, NPDT[dt])
        tasks.append((gen, dt, n, sin, sout, out))
        refs.append((ref, ref_state, st))
    return tasks, refs


def check(tasks, refs):
    for k, ((gen, dt, n, sin, sout, out), (ref, ref_state, st0)) in enumerate(zip(tasks, refs)):
        got = out.cpu().numpy().view(NPDT[dt])[:n]
        np.testing.assert_array_equal(got, ref, err_msg=f"task {k} gen {gen} dtype {dt} n {n}")
        assert np.array_equal(sout.cpu().numpy(), ref_state), f"state of task {k} gen {gen} n {n}"
        assert np.array_equal(sin.cpu().numpy(), st0), f"input state of task {k} changed"


def mixed_specs():
    rng = np.random.default_rng(11)
    specs = []
    for gen in range(11):
        for dt in (P.U32, P.F32, P.F64):
            for n in (0, 1, 31, 33, 1000, int(rng.integers(2000, 30000))):
                specs.append((gen, dt, n))
    specs += [(g, P.U32, 150001) for g in range(11)]
    return specs


@pytest.mark.parametrize("cfg", [None, (2, 512, 1024, 1, 16, 0), (4, 8192, 16384, 0, 32, 1), (1, 32, 32, 1, 16, 1),
                                 (4, 2048, 4096, 1, 16, 0), (4, 2048, 4096, 1, 32, 1), (4, 8192, 16384, 1, 16, 2),
                                 (2, 512, 1024, 0, 32, 2)])
def test_batch_matches_oracle(ctx, oracle, cfg):
    tasks, refs = make_tasks(oracle, mixed_specs())
    conf = P.BatchConfig(*cfg) if cfg else None
    b = P.Batch(ctx, tasks, conf)
    assert b.tiles() > len(tasks)
    b.launch()
    torch.cuda.synchronize()
    check(tasks, refs)
    b.close()


# batches holding only some families: either register class (or both) may
# be empty, and within the light class any of MT19937, v = 1 GM/GQ and
# MRG32K3A/LFSR113
SUBSETS = {
    "mt_only": [(P.MT19937, dt, n) for dt in (P.U32, P.F64) for n in (0, 1, 700, 5000)],
    "v1_only": [(g, dt, n) for g in (P.GM19, P.GM61, P.GQ58X1) for dt in (P.U32, P.F32) for n in (1, 64, 3001)],
    "mt_and_v1": [(P.MT19937, P.F32, 2500), (P.GM29, P.F32, 2500), (P.GM31, P.U32, 77), (P.MT19937, P.U32, 0)],
    "no_mt_no_v1": [(g, P.U32, n) for g in (P.MRG32K3A, P.GM55, P.GQ58X3) for n in (5, 4000)],
    "copies_only": [(g, P.U32, 0) for g in range(11)],
}


def mt_state_at(oracle, seed, kind):
    """A seeded MT19937 state at a chosen place in its 624-word block:
    block used up (624), 300 or 1 words used, or a renewed block with none
    used (index 0: the oracle's state after 624 outputs, index reset)."""
    st = oracle.seed(P.MT19937, seed)
    if kind == "mid":
        oracle.generate(P.MT19937, st, 300)
    elif kind == "one":
        oracle.generate(P.MT19937, st, 1)
    elif kind == "zero":
        oracle.generate(P.MT19937, st, 624)
        st.view(np.uint32)[624] = 0
    return st


@pytest.mark.parametrize("graph", [1, 0])
def test_batch_long_mt_sections(ctx, oracle, graph):
    """MT19937 tasks longer than 2^24 outputs are cut into sections of
    624 * 2^10 outputs, each started by a whole-block jump of the task state
    that keeps its place in the block; outputs and final states (bit for bit)
    equal the oracle's sequential ones, whatever the start index."""
    L, T = 624 << 10, 1 << 24
    specs = [("aligned", P.U32, T + 1), ("mid", P.F32, T + 3 * L - 5), ("one", P.U32, T + 2 * L),
             ("zero", P.F64, T + 2 * L + 1877), ("zero", P.U32, T + 624), ("mid", P.U32, T),
             ("one", P.U32, 27 * L)]   # a whole number of sections
    tasks, refs = [], []
    for k, (kind, dt, n) in enumerate(specs):
        st = mt_state_at(oracle, 4000 + k, kind)
        sin = torch.from_numpy(st.copy()).cuda()
        sout = torch.full_like(sin, 0xA5)
        out = torch.empty(n, dtype=TDT[dt], device="cuda")
        ref_state = st.copy()
        ref = oracle.generate(P.MT19937, ref_state, n, dt)
        tasks.append((P.MT19937, dt, n, sin, sout, out))
        refs.append((ref, ref_state, st))
    b = P.Batch(ctx, tasks, P.BatchConfig(4, 2048, 4096, graph))
    assert b.tiles() == sum((n + L - 1) // L if n > T else 1 for _, _, n in specs)
    for _ in range(2):
        for (_, _, _, _, sout, out) in tasks:
            out.zero_()
            sout.fill_(0x5A)
        b.launch()
        torch.cuda.synchronize()
        check(tasks, refs)
    b.close()


@pytest.mark.parametrize("graph", [1, 0])
@pytest.mark.parametrize("subset", sorted(SUBSETS))
def test_batch_family_subsets(ctx, oracle, subset, graph):
    tasks, refs = make_tasks(oracle, SUBSETS[subset], seed0=1300)
    b = P.Batch(ctx, tasks, P.BatchConfig(4, 2048, 4096, graph))
    for _ in range(2):
        b.launch()
        torch.cuda.synchronize()
        check(tasks, refs)
    b.close()


def test_batch_graph_replays(ctx, oracle):
    """Replays of the captured graph, with eager work between them, all give
    the same result (the input states are never written)."""
    tasks, refs = make_tasks(oracle, mixed_specs()[::3], seed0=900)
    b = P.Batch(ctx, tasks, P.BatchConfig(4, 2048, 4096, 1))
    for rep in range(4):
        for (_, _, _, _, sout, out) in tasks:
            out.zero_()
            sout.fill_(0x5A)
        b.launch()
        torch.cuda.synchronize()
        check(tasks, refs)
        torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
    b.close()


def test_batch_equals_plain_launches(ctx, oracle):
    """The batched launch reproduces the plain per-stream launches."""
    gens, ids, lens = W.batched_tasks(count=200, lo=1e3, hi=2e5)
    tasks, plain = [], []
    for g, sid, n in zip(gens, ids, lens):
        g, n = int(g), int(n)
        sb = P.state_bytes(g)
        st = torch.empty(sb, dtype=torch.uint8, device="cuda")
        t_ids = torch.from_numpy(np.array([sid], dtype=np.uint64).view(np.int64)).cuda()
        ctx.init_streams_dev(g, P.SEQ_DEFAULT, None, t_ids, 1, st)
        sout = torch.zeros_like(st)
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        tasks.append((g, P.F32, n, st, sout, out))
        pst = st.clone()
        pout = torch.empty(n, dtype=torch.float32, device="cuda")
        ctx.generate_streams(g, pst, 1, n, P.F32, pout)
        plain.append((pst, pout))
    b = P.Batch(ctx, tasks)
    b.launch()
    torch.cuda.synchronize()
    for (g, _, n, _, sout, out), (pst, pout) in zip(tasks, plain):
        assert torch.equal(out, pout), (g, n)
        assert torch.equal(sout, pst), (g, n)
    # and a sample against the oracle
    for k in range(0, len(tasks), 17):
        g, _, n, sin, sout, out = tasks[k]
        st = sin.cpu().numpy().copy()
        ref = oracle.generate(g, st, n, P.F32)
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
    b.close()


def test_batch_rejects_bad_tasks(ctx):
    st = torch.zeros(P.state_bytes(1), dtype=torch.uint8, device="cuda")
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(P.PrandError):
        P.Batch(ctx, [(11, P.U32, 16, st, st.clone(), out)])      # bad generator
    with pytest.raises(P.PrandError):
        P.Batch(ctx, [(1, 3, 16, st, st.clone(), out)])           # bad dtype
    with pytest.raises(P.PrandError):
        P.Batch(ctx, [(1, P.U32, 16, st, st.clone(), None)])      # no output
    empty = P.Batch(ctx, [])
    empty.launch()
    assert empty.tiles() == 0


def test_autotune_returns_a_working_config(ctx, oracle, tmp_path, monkeypatch):
    monkeypatch.setenv("PRAND_TUNE_CACHE", str(tmp_path / "tune.txt"))
    specs = [(g, P.F32, 20000 + 1000 * g) for g in range(11)]
    tasks, refs = make_tasks(oracle, specs, seed0=1300)
    best = P.autotune(ctx, tasks)
    assert best.waves_per_block in (2, 4) and best.use_graph == 1
    again = P.autotune(ctx, tasks)          # second call: from the cache file
    assert (again.waves_per_block, again.reg_section, again.gm_section) == \
        (best.waves_per_block, best.reg_section, best.gm_section)
    assert (tmp_path / "tune.txt").read_text().count("\n") == 1
    b = P.Batch(ctx, tasks, best)
    b.launch()
    torch.cuda.synchronize()
    check(tasks, refs)
    b.close()
