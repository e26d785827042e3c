"""Throughput benchmark on one MI355X.

Workload (many independent streams of every generator): for each of the 11
generators, 65536 streams with ids drawn uniformly from [0, 10^19) are
initialised by block splitting (stream id = default state jumped id * L
outputs) and each stream then generates 16384 32-bit words -- 2^30 words per
generator.  One step = stream initialisation + generation for all 11
generators.  Inputs (ids) and outputs stay in HBM.

Prints one JSON line: whole-step throughput in numbers/s, per-generator
figures, the roofline of the kernel that takes most of the step, and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                      # MI355X HBM3E
# VALU issue on gfx950 (256 CUs x 4 SIMDs, 2.4 GHz) comes in two rates: the
# simple 32-bit operations (add/sub, and/or/xor, three-input bitop3, right
# shifts, FP32 add/mul/fma) complete a wave64 instruction every two cycles,
# 32 lanes per SIMD per clock = 78.6 T lane-instructions/s -- the published
# fp32 vector peak, 157.3 TFLOP/s, counts this FMA rate as two flops; the
# others (left shifts, bit-field ops, 24-bit and 32-bit multiplies, min/max,
# conversions, every FP64 operation) every four cycles, 39.3 T -- the fp64
# vector peak, 78.6 TFLOP/s.  A probe of independent dependency chains
# measured 66-74 T and 35-39 T for the two groups.
VALU_FAST_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
VALU_SLOW_TOPS = VALU_FAST_TOPS / 2
# Word-XORs: one three-input XOR (v_bitop3_b32, truth table 0x96, a fast
# operation) adds two 32-bit words to a third, so the XOR-sum of the MT19937
# jump peaks at two word-XORs per lane-instruction at the fast rate.
XOR_PEAK_TOPS = 2 * VALU_FAST_TOPS
# VALU lane-instructions per 32-bit output word of the GM/GQ generation
# kernels (SQ_INSTS_VALU x 64 / words, counted at 65536 streams x 16384
# words); a mix of fast and slow operations, reported against the fast peak
GM_OPS_PER_WORD = {3: 266.1, 4: 330.1, 5: 330.1, 6: 153.6, 7: 428.1, 8: 338.1, 9: 150.6, 10: 105.5}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--streams", type=int, default=65536)
    ap.add_argument("--words", type=int, default=16384)
    ap.add_argument("--gens", type=str, default="all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dtype-sweep", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-jump", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the steps, one 1 GiB device-to-device copy (a plain copy kernel of known size, "
                         "the scale for hardware byte counters)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--batched-tasks", type=int, default=20000)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1307_5869_amd import prand as P
    from paper_1307_5869_amd import workloads as W

    if not os.path.exists(P.LIB_PATH):
        raise SystemExit("libprand.so is not built: python -m paper_1307_5869_amd.build")
    gens = list(range(P.NUM_GENERATORS)) if args.gens == "all" else [int(g) for g in args.gens.split(",")]
    S, N = args.streams, args.words
    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    stream = torch.cuda.current_stream()
    ids = {g: torch.from_numpy(W.stream_ids(S, g).view(np.int64)).to(dev) for g in gens}
    sb_max = max(P.state_bytes(g) for g in gens)
    states = torch.empty(S * sb_max, dtype=torch.uint8, device=dev)
    out = torch.empty(S * N, dtype=torch.int32, device=dev)
    # (gen, phase) -> list of (start, end) events
    ev = {}

    def step(record):
        for g in gens:
            e0 = torch.cuda.Event(enable_timing=True) if record else None
            e1 = torch.cuda.Event(enable_timing=True) if record else None
            e2 = torch.cuda.Event(enable_timing=True) if record else None
            if record:
                e0.record(stream)
            ctx.init_streams_dev(g, P.SEQ_DEFAULT, None, ids[g], S, states, stream)
            if record:
                e1.record(stream)
            ctx.generate_streams(g, states, S, N, P.U32, out, stream)
            if record:
                e2.record(stream)
                ev.setdefault((g, "init"), []).append((e0, e1))
                ev.setdefault((g, "gen"), []).append((e1, e2))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    numbers = len(gens) * S * N
    value = numbers * args.steps / wall

    def avg_ms(key):
        return float(np.mean([a.elapsed_time(b) for a, b in ev[key]]))

    per_gen = {}
    for g in gens:
        ti, tg = avg_ms((g, "init")), avg_ms((g, "gen"))
        per_gen[P.NAMES[g]] = {"init_ms": round(ti, 4), "gen_u32_ms": round(tg, 4),
                               "gen_u32_numbers_per_s": S * N / (tg * 1e-3),
                               "streams_init_per_s": S / (ti * 1e-3)}
    # dominant kernel of the step
    key = max(ev, key=avg_ms)
    g, phase = key
    t = avg_ms(key) * 1e-3
    if phase == "gen":
        sb = P.state_bytes(g)
        if g in (P.MT19937, P.MRG32K3A, P.LFSR113):
            traffic = S * N * 4 + 2 * S * sb     # outputs + state read/write
            roof = {"kernel": f"{P.NAMES[g]} generate", "bound": "hbm", "achieved": traffic / t / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            ops = S * N * GM_OPS_PER_WORD[g]     # VALU lane-instructions
            roof = {"kernel": f"{P.NAMES[g]} generate", "bound": "alu", "achieved": ops / t / 1e12,
                    "peak": VALU_FAST_TOPS, "unit": "T lane-instructions/s"}
    else:
        if g == P.MT19937:
            # XOR-sum: per stream one table polynomial per nonzero 16-bit digit
            # of the id's low 48 bits (its top 16 bits select a precomputed
            # start state), each costing (set coefficients ~ 19937/2) x 624
            # word XORs
            idv = W.stream_ids(S, g)
            apps = int(sum(sum(1 for k in range(3) if (int(x) >> (16 * k)) & 0xFFFF) for x in idv))
            ops = apps * (19937 // 2) * 624
            roof = {"kernel": "MT19937 jump", "bound": "alu", "achieved": ops / t / 1e12, "peak": XOR_PEAK_TOPS,
                    "unit": "T word-XOR/s"}
        else:
            sb = P.state_bytes(g)
            roof = {"kernel": f"{P.NAMES[g]} jump", "bound": "hbm", "achieved": 2 * S * sb / t / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["avg_ms"] = t * 1e3
    roof["traffic"] = recorded_traffic(roof["kernel"])

    extra = {}
    write_probe = None
    if not args.no_dtype_sweep:
        # context for the HBM-bound kernels: a plain device fill of the same
        # 4 GiB (torch's fill kernel), outside the timed region
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        out.fill_(1)
        a.record(stream)
        out.fill_(2)
        b.record(stream)
        b.synchronize()
        write_probe = {"bytes": out.numel() * 4, "ms": round(a.elapsed_time(b), 4),
                       "GBs": out.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9}
        # outside the timed region: every dtype for every generator, one
        # untimed launch and then five timed ones (the states advance from
        # launch to launch); median, fastest and slowest launch
        big = torch.empty(S * N * 2, dtype=torch.int32, device=dev)
        for g in gens:
            ctx.init_streams_dev(g, P.SEQ_DEFAULT, None, ids[g], S, states, stream)
            r = {}
            for dt, name in ((P.U32, "u32"), (P.F32, "f32"), (P.F64, "f64")):
                ctx.generate_streams(g, states, S, N, dt, big, stream)
                evs = []
                for _ in range(5):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    ctx.generate_streams(g, states, S, N, dt, big, stream)
                    b.record(stream)
                    evs.append((a, b))
                evs[-1][1].synchronize()
                t = sorted(a.elapsed_time(b) for a, b in evs)
                ms = t[len(t) // 2]
                es = 8 if dt == P.F64 else 4
                r[name] = {"ms": round(ms, 4), "ms_min": round(t[0], 4), "ms_max": round(t[-1], 4),
                           "numbers_per_s": S * N / (ms * 1e-3), "write_GBs": S * N * es / (ms * 1e-3) / 1e9,
                           "hbm_frac": S * N * es / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            extra[P.NAMES[g]] = r
        del big

    del out, states
    torch.cuda.empty_cache()
    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log("C2 step done; 4096-stream MRG32K3A workload")
    c1 = mrg_4096_streams(ctx, stream) if P.MRG32K3A in gens else None
    log("2^20-stream jump workload")
    c3 = None if args.no_jump else jump_2pow_k(ctx, stream, gens)
    log("batched workload")
    rates = {g: extra[P.NAMES[g]]["f32"]["numbers_per_s"] for g in gens} if extra and len(gens) == 11 else None
    batched = None if args.no_batched else batched_vs_plain(ctx, args.batched_tasks, stream, rates)
    log("batched done; serving loop")
    serving = None if args.no_serve else serve_trace(ctx, args.serve_rate, args.serve_seconds)
    log("serving done; CPU baseline")

    cpu = None if args.no_cpu_baseline else cpu_baseline(gens, S, N)
    simd = None if args.no_cpu_baseline else cpu_simd(ctx, gens)

    line = {
        "metric": "uniform numbers/sec per generator (bit-exact); batched vs plain; serve p99 ms",
        "value": value,
        "unit": "numbers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{len(gens)} generators x {S} streams (block-split, ids uniform in [0,1e19)) "
                               f"x {N} u32 words; step = stream init + generation",
                   "streams_per_generator": S, "words_per_stream": N, "generators": [P.NAMES[g] for g in gens],
                   "parallelism": "1 GPU"},
        "roofline": roof,
        "per_generator": per_gen,
        "dtype_sweep": extra,
        "mrg32k3a_4096_streams": c1,
        "jump_2pow_k": c3,
        "fill_probe": write_probe,
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
        "cpu_simd": simd,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def cpu_simd(ctx, gens):
    """The library's CPU SIMD generation (prand_simd_fill), one host thread
    per generator, u32: a state from block splitting (stream 1 of the
    default state), 2^24 words (MT19937, MRG32K3A, LFSR113) or 2^21 (GM/GQ)
    after a warm-up fill.  Context, not the baseline: the baseline is the
    oracle."""
    from paper_1307_5869_amd import prand as P

    res = {}
    isa = None
    for g in gens:
        st = ctx.init_stream(g, P.SEQ_DEFAULT, 1)
        s = P.SimdState(g, st)
        isa = "avx2" if s.vectorized else "scalar"
        n = 1 << (24 if g <= P.LFSR113 else 21)
        s.fill(P.U32, 4096)
        t = time.perf_counter()
        s.fill(P.U32, n)
        res[P.NAMES[g]] = n / (time.perf_counter() - t)
    return {"unit": "numbers/s", "threads": 1, "isa": isa, "per_generator": res, "host": host_cpu()}


def recorded_traffic(kernel):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summaries (FETCH_SIZE and WRITE_SIZE runs scaled by a copy kernel of known
    size), or None when none covers this kernel or its sources have changed
    since the counters were taken."""
    import glob
    import hashlib
    import re

    names = {"MT19937 jump": "mt_jump_kernel<1>"}
    want = names.get(kernel)
    if want is None:
        return None
    csrc = os.path.join(ROOT, "paper_1307_5869_amd", "csrc")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for m in re.finditer(r"traffic kernel=(\S+) bytes=(\d+) sources=(\S+) sha256_16=([0-9a-f]+)", open(path).read()):
            if m.group(1) != want:
                continue
            h = hashlib.sha256()
            for f in m.group(3).split("+"):
                h.update(open(os.path.join(csrc, f), "rb").read())
            if h.hexdigest()[:16] == m.group(4):
                return float(m.group(2))
    return None


def mrg_4096_streams(ctx, stream, reps=20):
    """4096 MRG32K3A streams from the all-12345 state, stream k skipped
    k * 2^76 ahead, then 4096 u32 outputs per stream and their float64
    conversion (16.7M numbers each): skip-ahead + both generation launches
    per repetition, states reset from the base outside the events."""
    import torch

    from paper_1307_5869_amd import prand as P

    dev = torch.device("cuda:0")
    gen, count, n = P.MRG32K3A, 4096, 4096
    base = ctx.seed(gen, 12345)
    d0 = torch.from_numpy(np.concatenate([base] * count)).to(dev)
    limbs = torch.from_numpy(np.stack([P.limbs(k * 2**76) for k in range(count)]).view(np.int64)).to(dev)
    d, d2 = torch.empty_like(d0), torch.empty_like(d0)
    u = torch.empty(count * n, dtype=torch.int32, device=dev)
    f = torch.empty(count * n, dtype=torch.float64, device=dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps + 2)]
    for r in range(reps + 2):
        d.copy_(d0)
        e = ev[r]
        e[0].record(stream)
        ctx.skipahead_dev(gen, d, count, limbs, 8, True, stream)
        d2.copy_(d)
        e[1].record(stream)
        ctx.generate_streams(gen, d, count, n, P.U32, u, stream)
        e[2].record(stream)
        ctx.generate_streams(gen, d2, count, n, P.F64, f, stream)
        e[3].record(stream)
    torch.cuda.synchronize()
    jump = float(np.mean([e[0].elapsed_time(e[1]) for e in ev[2:]]))
    gu = float(np.mean([e[1].elapsed_time(e[2]) for e in ev[2:]]))
    gf = float(np.mean([e[2].elapsed_time(e[3]) for e in ev[2:]]))
    total = jump + gu + gf
    written = count * n * (4 + 8)
    return {"workload": "MRG32K3A, 4096 streams from the all-12345 state, stream k skipped k*2^76, "
                        "4096 u32 + 4096 f64 per stream",
            "skipahead_ms": round(jump, 4), "gen_u32_ms": round(gu, 4), "gen_f64_ms": round(gf, 4),
            "total_ms": round(total, 4), "numbers_per_s": 2 * count * n / (total * 1e-3),
            "gen_write_GBs": written / ((gu + gf) * 1e-3) / 1e9,
            "gen_hbm_frac": written / ((gu + gf) * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "note": "16.7M outputs per launch take tens of microseconds, so launch latency is a large share"}


def jump_2pow_k(ctx, stream, gens):
    """2^20 streams per generator, each jumped 2^k ahead (k uniform in the
    generator's table range) by one per-stream skip-ahead launch: streams
    initialised per second."""
    import torch

    from paper_1307_5869_amd import prand as P
    from paper_1307_5869_amd import workloads as W

    dev = torch.device("cuda:0")
    S = 1 << 20
    res = {}
    for g in gens:
        base = ctx.seed(g, 4242 + g)
        states = torch.from_numpy(base.copy()).to(dev).repeat(S)
        ks = W.jump_exponents(S, g)
        limbs = np.zeros((S, 8), dtype=np.uint64)
        limbs[np.arange(S), ks // 64] = np.left_shift(np.uint64(1), (ks % 64).astype(np.uint64))
        t_limbs = torch.from_numpy(limbs.reshape(-1).view(np.int64)).to(dev)
        ctx.skipahead_dev(g, states, S, t_limbs, 8, True, stream)   # warm-up (and MT19937 tables)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.skipahead_dev(g, states, S, t_limbs, 8, True, stream)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b)
        lo, hi = W.JUMP_EXP_RANGE[g]
        res[P.NAMES[g]] = {"ms": round(ms, 3), "streams_per_s": S / (ms * 1e-3), "k_range": [lo, hi],
                           "state_bytes": P.state_bytes(g)}
        del states, t_limbs
    torch.cuda.empty_cache()
    return {"workload": "2^20 streams per generator, stream s jumped 2^k_s ahead, k_s uniform in the range",
            "per_generator": res}


def batched_vs_plain(ctx, ntasks, stream, plain_rates=None):
    """Many streams of mixed generators and uneven lengths (log-uniform in
    [1e3, 1e7]) in f32: one autotuned batched launch replayed from a HIP
    graph, against plain per-stream launches timed on a sample of the tasks."""
    import torch

    from paper_1307_5869_amd import prand as P
    from paper_1307_5869_amd import workloads as W

    dev = torch.device("cuda:0")
    gens, ids, lens = W.batched_tasks(count=ntasks)
    total = int(lens.sum())
    out = torch.empty(total, dtype=torch.float32, device=dev)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]])
    sb = [P.state_bytes(g) for g in range(P.NUM_GENERATORS)]
    sin = {}
    for g in range(P.NUM_GENERATORS):
        sel = np.nonzero(gens == g)[0]
        if sel.size == 0:
            continue
        st = torch.empty(sel.size * sb[g], dtype=torch.uint8, device=dev)
        t_ids = torch.from_numpy(ids[sel].view(np.int64)).to(dev)
        ctx.init_streams_dev(g, P.SEQ_DEFAULT, None, t_ids, sel.size, st, stream)
        sin[g] = (sel, st)
    sout = {g: torch.empty_like(v[1]) for g, v in sin.items()}
    tasks = [None] * ntasks
    for g, (sel, st) in sin.items():
        base_in, base_out = st.data_ptr(), sout[g].data_ptr()
        for j, k in enumerate(sel):
            tasks[k] = (g, P.F32, int(lens[k]), base_in + j * sb[g], base_out + j * sb[g],
                        out.data_ptr() + 4 * int(offs[k]))
    torch.cuda.synchronize()
    # tune on the whole mix (a small sample is dominated by its longest
    # single-wavefront MT19937 task whatever the shape), then run it
    t0 = time.perf_counter()
    best = P.autotune(ctx, tasks)
    tune_s = time.perf_counter() - t0
    b = P.Batch(ctx, tasks, best)
    b.launch(stream)
    torch.cuda.synchronize()
    reps = 2
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        b.launch(stream)
    z.record(stream)
    z.synchronize()
    ms = a.elapsed_time(z) / reps
    tiles = b.tiles()
    b.close()
    # plain per-generator launches on the same work: per generator, tasks
    # bucketed by length (lengths within a factor of two), one many-stream
    # launch per bucket generating the bucket's longest length for every
    # stream in it (padding outputs go to a scratch buffer)
    buckets = []
    for g, (sel, st) in sin.items():
        lg = lens[sel]
        key = np.floor(np.log2(lg)).astype(int)
        for kb in np.unique(key):
            idx = np.nonzero(key == kb)[0]
            gather = torch.from_numpy(np.concatenate([np.arange(j * sb[g], (j + 1) * sb[g]) for j in idx])).to(dev)
            buckets.append((g, len(idx), int(lg[idx].max()), int(lg[idx].sum()), st[gather].contiguous()))
    pad_out = torch.empty(max(c * nmax for _, c, nmax, _, _ in buckets), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    a.record(stream)
    for g, c, nmax, _, bst in buckets:
        ctx.generate_streams(g, bst, c, nmax, P.F32, pad_out, stream)
    z.record(stream)
    z.synchronize()
    bucket_ms = a.elapsed_time(z)
    bucket_padded = sum(c * nmax for _, c, nmax, _, _ in buckets)
    del buckets, pad_out
    # the same work at each generator's full-size many-stream f32 rate
    ideal_ms = None
    if plain_rates:
        ideal_ms = 1e3 * sum(int(lens[sel].sum()) / plain_rates[g] for g, (sel, _) in sin.items())
    # plain: one generate launch per stream (prand_generate_streams, count 1),
    # over a random order of the tasks until about 10 s of GPU time have been
    # spent; the output states are copies of the input states, advanced in place
    order = np.random.default_rng(7).permutation(ntasks)
    for g, (sel, st) in sin.items():
        sout[g].copy_(st)
    torch.cuda.synchronize()
    plain_ms, done, plain_numbers = 0.0, 0, 0
    while done < ntasks and plain_ms < 10e3:
        chunk = order[done:done + 25]
        a.record(stream)
        for k in chunk:
            g, _, n, _, pst, pout = tasks[k]
            ctx.generate_streams(g, pst, 1, n, P.F32, pout, stream)
        z.record(stream)
        z.synchronize()
        plain_ms += a.elapsed_time(z)
        done += len(chunk)
        plain_numbers += int(lens[chunk].sum())
    # plain, sectioned: one prand_generate call per task (the task's sections
    # jump to their starts and fill in parallel; the call copies the state in
    # and out and blocks), over the same random order until about 5 s
    host_states = {}
    for k in order[:2000]:
        g, _, n, pin, _, _ = tasks[k]
        sin_g, st_g = sin[g]
        j = int(np.nonzero(sin_g == k)[0][0])
        host_states[k] = st_g[j * sb[g]:(j + 1) * sb[g]].cpu().numpy().copy()
    torch.cuda.synchronize()
    sec_s, sec_done, sec_numbers = 0.0, 0, 0
    for k in order[:2000]:
        g, _, n, _, _, pout = tasks[k]
        t0 = time.perf_counter()
        ctx.generate(g, host_states[k], P.F32, pout, n, stream)
        sec_s += time.perf_counter() - t0
        sec_done += 1
        sec_numbers += n
        if sec_s > 5.0:
            break
    del out
    torch.cuda.empty_cache()
    return {"tasks": ntasks, "numbers": total, "dtype": "f32", "tiles": tiles,
            "plain_per_generator_ms": round(bucket_ms, 3), "plain_per_generator_padded_numbers": bucket_padded,
            "speedup_vs_plain_per_generator": bucket_ms / ms,
            "ideal_plain_ms": round(ideal_ms, 3) if ideal_ms else None,
            "batched_over_ideal_plain": ms / ideal_ms if ideal_ms else None,
            "plain_sectioned_tasks": sec_done, "plain_sectioned_numbers": sec_numbers,
            "plain_sectioned_s": round(sec_s, 3),
            "plain_sectioned_numbers_per_s": sec_numbers / sec_s,
            "speedup_vs_sectioned": (total / (ms * 1e-3)) / (sec_numbers / sec_s),
            "config": {"waves_per_block": best.waves_per_block, "reg_section": best.reg_section,
                       "gm_section": best.gm_section, "lds_chunk_words": best.lds_chunk_words,
                       "overlap": best.overlap,
                       "graph": bool(best.use_graph)},
            "autotune_s": round(tune_s, 2), "batched_ms": round(ms, 3),
            "batched_numbers_per_s": total / (ms * 1e-3),
            "one_launch_per_stream_sample_tasks": done, "one_launch_per_stream_sample_numbers": plain_numbers,
            "one_launch_per_stream_ms": round(plain_ms, 3),
            "one_launch_per_stream_numbers_per_s": plain_numbers / (plain_ms * 1e-3),
            "speedup_vs_one_launch_per_stream": (total / (ms * 1e-3)) / (plain_numbers / (plain_ms * 1e-3))}


def serve_trace(ctx, rate, seconds):
    """Poisson arrivals (rate/s for `seconds`), generator and dtype uniform,
    stream ids uniform in [0, 1e19), lengths log-uniform in [1e3, 1e8],
    submitted to the native serving loop at their arrival times; the client
    releases each output as soon as it is reported complete (outputs stay in
    HBM, no copy to the host)."""
    from paper_1307_5869_amd import prand as P
    from paper_1307_5869_amd import workloads as W

    t_arr, gens, ids, ns, dts = W.serving_requests(rate=rate, seconds=seconds)
    cfg = P.ServerConfig(hbm_budget=64 << 30)
    srv = P.Server(ctx, cfg)
    lat, tags, numbers, rejected = [], [], 0, 0
    first_t, last_t = None, 0.0
    t0 = srv.clock()
    next_log = 10.0

    def collect(wait_ms=0):
        nonlocal numbers, first_t, last_t
        for c in srv.poll(wait_ms=wait_ms):
            lat.append(c.t_done - (t0 + t_arr[c.tag]))   # from the scheduled arrival
            tags.append(c.tag)
            numbers += c.n
            first_t = c.t_submit if first_t is None else min(first_t, c.t_submit)
            last_t = max(last_t, c.t_done)
            srv.release(c.ticket)

    for k in range(len(t_arr)):
        while True:
            dt = t0 + t_arr[k] - srv.clock()
            if dt <= 0:
                break
            collect()
            if dt > 2e-4:
                time.sleep(min(dt, 1e-3))
        rc, _ = srv.try_submit(int(gens[k]), int(ids[k]), int(ns[k]), int(dts[k]), tag=k)
        if rc != P.OK:
            rejected += 1
        if t_arr[k] >= next_log:
            log(f"serving: {k + 1} submitted, {len(lat)} complete at t={t_arr[k]:.0f}s")
            next_log += 10.0
    deadline = time.time() + 120
    while len(lat) + rejected < len(t_arr) and time.time() < deadline:
        collect(wait_ms=50)
    st = srv.stats()
    srv.close()
    lat_ms = np.array(lat) * 1e3
    span = last_t - (first_t or 0.0)
    # where the tail comes from: percentiles per generator and per length decade
    tg = np.array(tags, dtype=np.int64)
    by_gen = {}
    for g in range(P.NUM_GENERATORS):
        v = lat_ms[gens[tg] == g] if lat else np.array([])
        if v.size:
            by_gen[P.NAMES[g]] = {"p50_ms": round(float(np.percentile(v, 50)), 3),
                                  "p99_ms": round(float(np.percentile(v, 99)), 3)}
    by_len = {}
    dec = np.floor(np.log10(np.maximum(ns[tg], 1))).astype(int) if lat else np.array([])
    for d in sorted(set(dec.tolist())):
        v = lat_ms[dec == d]
        by_len[f"1e{d}"] = {"requests": int(v.size), "p50_ms": round(float(np.percentile(v, 50)), 3),
                            "p99_ms": round(float(np.percentile(v, 99)), 3)}
    offered = float(ns.sum()) / seconds
    return {"requests": int(len(t_arr)), "completed": len(lat), "rejected": rejected, "rate_per_s": rate,
            "seconds": seconds, "offered_numbers_per_s": offered,
            "sustained_numbers_per_s": numbers / span if span > 0 else None,
            "p50_ms": float(np.percentile(lat_ms, 50)) if lat else None,
            "p99_ms": float(np.percentile(lat_ms, 99)) if lat else None,
            "max_ms": float(lat_ms.max()) if lat else None,
            "by_generator": by_gen, "by_length_decade": by_len,
            "hbm_budget": st["hbm_budget"], "hbm_peak": st["hbm_peak"], "iterations": st["iterations"],
            "gpu_busy_frac": st["gpu_busy_s"] / span if span > 0 else None,
            "workload": "Poisson arrivals, gen and dtype uniform, ids uniform in [0,1e19), n log-uniform [1e3,1e8]"}


def host_cpu():
    """(logical CPUs of the host, CPUs this process may run on, model name)"""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return os.cpu_count() or 1, usable, model


def cpu_baseline(gens, S, N, share=16):
    """The oracle (plain single-threaded C, untuned) on host threads over
    streams, per generator: block-splitting initialisation of a sample of the
    workload's streams, then generation of N words from those states (cycled
    over a larger sample).  The threads are the CPUs this process may use, at
    most `share` (a GPU's share of the host).  The whole workload's CPU time
    is estimated from the two rates."""
    from oracle import Oracle
    from paper_1307_5869_amd import prand as P
    from paper_1307_5869_amd import workloads as W

    O = Oracle()
    O.mt_charpoly()   # one-time polynomial set-up, not part of the timing
    nproc, usable, model = host_cpu()
    cores = max(1, min(share, usable))

    def run(fn, count):
        th = [threading.Thread(target=lambda c=c: [fn(k) for k in range(c, count, cores)]) for c in range(cores)]
        t0 = time.perf_counter()
        for t in th:
            t.start()
        for t in th:
            t.join()
        return time.perf_counter() - t0

    per_gen, total_s = {}, 0.0
    for g in gens:
        n_init = cores if g == P.MT19937 else (64 * cores if g == P.LFSR113 else 256 * cores)
        # about a second of generation per generator
        n_gen = cores * (1024 if g <= P.LFSR113 else (256 if g in (P.GM55, P.GQ58X3, P.GQ58X4) else 128))
        sid = W.stream_ids(n_init, g)
        sts = [None] * n_init
        t_init = run(lambda k: sts.__setitem__(k, O.init_stream(g, 0, int(sid[k]))), n_init)
        bufs = [np.empty(N, dtype=np.uint32) for _ in range(cores)]
        t_gen = run(lambda k: O.generate_into(g, sts[k % n_init], 0, bufs[k % cores]), n_gen)
        init_ps, gen_ps = n_init / t_init, n_gen * N / t_gen
        est = S / init_ps + S * N / gen_ps
        total_s += est
        per_gen[P.NAMES[g]] = {"init_streams_per_s": init_ps, "gen_u32_numbers_per_s": gen_ps,
                               "sample": f"init {n_init} streams, generate {n_gen} x {N} words",
                               "workload_s_est": round(est, 1)}
    value = len(gens) * S * N / total_s
    return {"value": value, "unit": "numbers/s", "cores": cores, "kind": "oracle",
            "host": {"nproc": nproc, "usable_cpus": usable, "model": model},
            "sample": f"per generator: block-splitting init of a sample of the workload's stream ids, then "
                      f"{N} u32 words from those states, on {cores} threads over streams; the whole "
                      f"{len(gens)} x {S}-stream workload's CPU time is estimated from the two rates",
            "per_generator": per_gen}


if __name__ == "__main__":
    main()
