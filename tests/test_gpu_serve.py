"""Serving loop: a request's output and final state are the same whether it
is served alone or in a mix of generators, dtypes and lengths, across many
loop iterations (chunked continuation); admission keeps within the HBM
budget and rejects what can never fit."""
import ctypes
import time

import numpy as np
import pytest
import torch

from paper_1307_5869_amd import prand as P

pytestmark = pytest.mark.gpu

NPDT = {P.U32: np.uint32, P.F32: np.float32, P.F64: np.float64}
TDT = {P.U32: torch.int32, P.F32: torch.float32, P.F64: torch.float64}
_hip = None


def dev_to_host(ptr, nbytes):
    """Copy device memory the server owns to a host array (test helper)."""
    global _hip
    if _hip is None:
        # the HIP runtime already in the process (the one libprand and torch use)
        path = next(ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln)
        _hip = ctypes.CDLL(path)
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    buf = np.empty(nbytes, dtype=np.uint8)
    assert _hip.hipMemcpy(buf.ctypes.data, ptr, nbytes, 2) == 0   # device to host
    return buf


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def alone(ctx, gen, sid, n, dtype, variant=P.SEQ_DEFAULT):
    st = torch.empty(P.state_bytes(gen), dtype=torch.uint8, device="cuda")
    ids = torch.from_numpy(np.array([sid], dtype=np.uint64).view(np.int64)).cuda()
    ctx.init_streams_dev(gen, variant, None, ids, 1, st)
    out = torch.empty(n, dtype=TDT[dtype], device="cuda")
    ctx.generate_streams(gen, st, 1, n, dtype, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(NPDT[dtype]), st.cpu().numpy()


def drain(srv, count, timeout_s=120):
    got = {}
    t0 = time.time()
    while len(got) < count:
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {count} completed"
        for c in srv.poll(wait_ms=50):
            got[c.ticket] = c
    return got


def check_completion(ctx, c, gen, sid, n, dtype, variant=P.SEQ_DEFAULT):
    es = 8 if dtype == P.F64 else 4
    out = dev_to_host(c.out, n * es).view(NPDT[dtype])
    st = dev_to_host(c.state, P.state_bytes(gen))
    ref_out, ref_st = alone(ctx, gen, sid, n, dtype, variant)
    np.testing.assert_array_equal(out, ref_out, err_msg=f"gen {gen} id {sid} n {n} dtype {dtype}")
    assert np.array_equal(st, ref_st), f"state gen {gen} id {sid} n {n}"


def mixed_requests(count, seed, lo=1e3, hi=1e5):
    r = np.random.default_rng(seed)
    gens = r.integers(0, 11, size=count)
    ids = r.integers(0, 10**19, size=count, dtype=np.uint64)
    ns = np.rint(np.exp(r.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    dts = r.integers(0, 3, size=count)
    return [(int(g), int(i), int(n), int(d)) for g, i, n, d in zip(gens, ids, ns, dts)]


def test_serve_alone_equals_mix(ctx):
    # small iterations: most requests span several loop iterations
    cfg = P.ServerConfig(hbm_budget=1 << 30, iter_numbers=1 << 20, min_chunk=1 << 12, mt_chunk=1 << 13)
    srv = P.Server(ctx, cfg)
    reqs = mixed_requests(500, seed=21)
    tickets = {}
    for k, (g, sid, n, dt) in enumerate(reqs):
        tickets[srv.submit(g, sid, n, dt, tag=k)] = k
        if k % 50 == 49:
            time.sleep(0.002)   # arrivals in bursts while the loop runs
    got = drain(srv, len(reqs))
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["iterations"] > 5
    for t, c in got.items():
        k = tickets[t]
        assert c.tag == k
        g, sid, n, dt = reqs[k]
        assert (c.gen, c.n, c.dtype) == (g, n, dt)
        assert c.t_submit <= c.t_admit <= c.t_done
        check_completion(ctx, c, g, sid, n, dt)
        srv.release(t)
    srv.close()


def test_serve_long_requests_continue_exactly(ctx, oracle):
    """Requests far longer than an iteration's share, every generator, with
    MT19937 chunks that end inside a twist block."""
    cfg = P.ServerConfig(hbm_budget=1 << 30, iter_numbers=1 << 18, min_chunk=1000, mt_chunk=5000)
    srv = P.Server(ctx, cfg)
    reqs = [(g, 10**18 + 7919 * g, 200003 + 17 * g, (P.U32, P.F32, P.F64)[g % 3]) for g in range(11)]
    tickets = {srv.submit(g, sid, n, dt): k for k, (g, sid, n, dt) in enumerate(reqs)}
    got = drain(srv, len(reqs))
    for t, c in got.items():
        g, sid, n, dt = reqs[tickets[t]]
        check_completion(ctx, c, g, sid, n, dt)
        # and the first words against the oracle's stream
        st = oracle.init_stream(g, 0, sid)
        ref = oracle.generate(g, st, 1000, dt)
        es = 8 if dt == P.F64 else 4
        np.testing.assert_array_equal(dev_to_host(c.out, 1000 * es).view(NPDT[dt]), ref)
        srv.release(t)
    srv.close()


def test_serve_long_mt_requests_in_sections(ctx):
    """MT19937 requests above the section threshold are cut into sections of
    624 * 2^k words that start from jumped states; outputs and the final
    state equal one sequential stream.  Both the configured threshold 2^22 and
    the default (2^20, sections from 624 * 2^10 words)."""
    sec = 624 << 12
    cfg = P.ServerConfig(hbm_budget=1 << 30, mt_section=1 << 22, mt_chunk=1 << 19)
    srv = P.Server(ctx, cfg)
    reqs = [(P.MT19937, 4242, (1 << 22) + 1, P.U32), (P.MT19937, 10**19 - 3, 2 * sec, P.F64),
            (P.MT19937, 7, 3 * sec + 12345, P.F32), (P.MT19937, 1 << 50, 1 << 22, P.U32)]
    tickets = {srv.submit(g, sid, n, dt): k for k, (g, sid, n, dt) in enumerate(reqs)}
    got = drain(srv, len(reqs))
    for t, c in got.items():
        g, sid, n, dt = reqs[tickets[t]]
        check_completion(ctx, c, g, sid, n, dt)
        srv.release(t)
    srv.close()
    # default threshold; the last request takes 150 sections (section starts
    # from the whole-block table up to section number 149)
    srv = P.Server(ctx, P.ServerConfig(hbm_budget=1 << 30))
    reqs = [(P.MT19937, 99, (1 << 20) + 1, P.U32), (P.MT19937, 2**63 + 1, 5 * (624 << 10) - 1, P.F32),
            (P.MT19937, 31337, 150 * (624 << 10) - 17, P.U32)]
    tickets = {srv.submit(g, sid, n, dt): k for k, (g, sid, n, dt) in enumerate(reqs)}
    got = drain(srv, len(reqs))
    for t, c in got.items():
        g, sid, n, dt = reqs[tickets[t]]
        check_completion(ctx, c, g, sid, n, dt)
        srv.release(t)
    srv.close()


def test_serve_variants(ctx):
    srv = P.Server(ctx, P.ServerConfig(hbm_budget=1 << 28))
    reqs = [(P.LFSR113, P.SEQ_LONG, 5, 3000), (P.GM29, P.SEQ_MEDIUM, 9, 3000), (P.GM55, P.SEQ_LONG, 2, 3000),
            (P.GQ58X3, P.SEQ_MEDIUM, 11, 3001)]
    tickets = {srv.submit(g, sid, n, P.U32, variant=v): k for k, (g, v, sid, n) in enumerate(reqs)}
    with pytest.raises(P.PrandError):
        srv.submit(P.MT19937, 1, 100, P.U32, variant=P.SEQ_SHORT)   # not offered for MT19937
    got = drain(srv, len(reqs))
    for t, c in got.items():
        g, v, sid, n = reqs[tickets[t]]
        check_completion(ctx, c, g, sid, n, P.U32, v)
    srv.close()


def test_serve_admission_by_hbm_budget(ctx):
    budget = 8 << 20
    srv = P.Server(ctx, P.ServerConfig(hbm_budget=budget, max_queue=64))
    n = (2 << 20) // 4          # 2 MiB of u32 per request: at most 3 fit with their states
    with pytest.raises(P.PrandError) as e:
        srv.submit(P.MRG32K3A, 1, budget, P.F64)                 # can never fit
    assert e.value.code == P.ERANGE
    tickets = [srv.submit(P.GM31, 100 + k, n, P.U32) for k in range(10)]
    first = drain(srv, 3)
    time.sleep(0.2)
    st = srv.stats()
    assert st["completed"] == 3 and st["waiting"] == 7, st
    assert st["hbm_used"] <= budget and st["hbm_peak"] <= budget
    for t, c in first.items():
        check_completion(ctx, c, P.GM31, 100 + tickets.index(t), n, P.U32)
        srv.release(t)
    # the rest are admitted as memory is given back: release while draining
    seen, t0 = 0, time.time()
    while seen < 7:
        assert time.time() - t0 < 120, f"only {seen} of 7 completed"
        for c in srv.poll(wait_ms=50):
            check_completion(ctx, c, P.GM31, 100 + tickets.index(c.ticket), n, P.U32)
            srv.release(c.ticket)
            seen += 1
    assert srv.stats()["hbm_peak"] <= budget
    # a full queue rejects
    rcs = [srv.try_submit(P.GM19, k, n, P.U32)[0] for k in range(80)]
    assert P.EBUSY in rcs
    st = srv.stats()
    assert st["rejected"] >= 2
    srv.close()    # drops the waiting requests, frees the unreleased ones
