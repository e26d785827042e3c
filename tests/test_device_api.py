"""The header-only per-thread API (include/prand_device.h).

CPU part: the header's functions compiled for the host run the same draw
loop as a user kernel, over states from the oracle; every value and the
advanced states must equal the oracle's plain generation, for all eleven
generators and every dtype, across MT19937 twist blocks and GQ58.3 blocks.

GPU part (marked gpu): a user kernel draws from one state per thread, in
device memory, seeded by the library on the device, and the result
is compared value by value with the oracle; the states it leaves are
continued by the library's many-stream call; a second kernel consumes the
numbers in registers and stores only their sums.
"""
import numpy as np
import pytest

import devapi_lib
from paper_1307_5869_amd import prand as P

NPDT = {0: np.uint32, 1: np.float32, 2: np.float64}


def host_draw(gen, dtype, states, n):
    lib = devapi_lib.load()
    blob = np.ascontiguousarray(np.concatenate(states))
    out = np.empty(len(states) * n, dtype=NPDT[dtype])
    assert lib.hostapi_draw(gen, dtype, blob.ctypes.data, len(states), n, out.ctypes.data) == 0
    sb = blob.size // len(states)
    return out.reshape(len(states), n), [blob[i * sb:(i + 1) * sb] for i in range(len(states))]


def test_blob_sizes_match_the_library():
    lib = devapi_lib.load()
    for g in range(11):
        assert lib.devapi_state_bytes(g) == P.state_bytes(g)


@pytest.mark.parametrize("gen", range(11))
@pytest.mark.parametrize("dtype", [0, 1, 2])
def test_host_build_equals_oracle(oracle, gen, dtype):
    # seeded states (GM/GQ not yet collapsed to the prime part), states from
    # block splitting, and a state part-way through an MT19937 / GQ58.3 block
    states = [oracle.seed(gen, s) for s in (1, 77, 2**40 + 3)]
    states += [oracle.init_stream(gen, 0, sid) for sid in (0, 5, 10**18 + 7)]
    mid = oracle.seed(gen, 9)
    oracle.generate(gen, mid, 13)
    states.append(mid)
    n = 1500 if gen == 0 else 700     # crosses MT19937 twists and GQ58.3 blocks
    got, after = host_draw(gen, dtype, [s.copy() for s in states], n)
    for i, s in enumerate(states):
        ref = oracle.generate(gen, s, n, dtype)
        np.testing.assert_array_equal(got[i], ref, err_msg=f"{P.NAMES[gen]} state {i}")
        assert np.array_equal(after[i], s), f"{P.NAMES[gen]} state {i} after"


@pytest.mark.parametrize("gen", [P.GQ58X3])
def test_host_build_gq58x3_every_word_offset(oracle, gen):
    """Single draws from each of the nine word offsets of a GQ58.3 block."""
    base = oracle.seed(gen, 31337)
    for off in range(9):
        st = base.copy()
        oracle.generate(gen, st, off)
        got, after = host_draw(gen, 0, [st.copy()], 1)
        assert got[0, 0] == oracle.generate(gen, st, 1)[0], off
        assert np.array_equal(after[0], st), off


# ------------------------------------------------------------------- GPU
@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.gpu
@pytest.mark.parametrize("gen", range(11))
def test_user_kernel_draws_match_oracle_and_continue(ctx, oracle, gen):
    import torch

    count = 256
    n1 = 1300 if gen == 0 else 600
    n2 = 1000
    seeds = np.arange(count, dtype=np.uint64) * np.uint64(7919) + np.uint64(3)
    seeds[-1] = np.uint64(2**63 + 11)    # the SplitMix64 branch of the register-state seeds
    states = torch.empty(count * P.state_bytes(gen), dtype=torch.uint8, device="cuda")
    ctx.seed_dev(gen, torch.from_numpy(seeds.view(np.int64)).cuda(), count, states)
    lib = devapi_lib.load()
    outs = {}
    for dtype, tdt in ((0, torch.int32), (1, torch.float32), (2, torch.float64)):
        st = states.clone()
        out = torch.empty(count * n1, dtype=tdt, device="cuda")
        assert lib.devapi_draw(gen, dtype, st.data_ptr(), count, n1, out.data_ptr(),
                               torch.cuda.current_stream().cuda_stream) == 0
        outs[dtype] = (out, st)
    # the library continues the states the user kernel left (u32 run)
    st_u32 = outs[0][1]
    cont = torch.empty(count * n2, dtype=torch.int32, device="cuda")
    ctx.generate_streams(gen, st_u32, count, n2, P.U32, cont)
    # a user kernel that keeps the numbers in registers: per-thread sums
    st = states.clone()
    sums = torch.empty(count, dtype=torch.float64, device="cuda")
    assert lib.devapi_sum(gen, st.data_ptr(), count, n1, sums.data_ptr(),
                          torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    got = {d: o.cpu().numpy().view(NPDT[d]).reshape(count, n1) for d, (o, _) in outs.items()}
    cont = cont.cpu().numpy().view(np.uint32).reshape(count, n2)
    sums = sums.cpu().numpy()
    for t in (0, 1, 2, 97, count - 1):
        base = oracle.seed(gen, int(seeds[t]))
        for d in (0, 1, 2):
            np.testing.assert_array_equal(got[d][t], oracle.generate(gen, base.copy(), n1, d),
                                          err_msg=f"{P.NAMES[gen]} thread {t} dtype {d}")
        o = base.copy()
        oracle.generate(gen, o, n1)
        np.testing.assert_array_equal(cont[t], oracle.generate(gen, o, n2), err_msg=f"{P.NAMES[gen]} continued {t}")
        dbl = oracle.generate(gen, base.copy(), n1, 2)
        assert sums[t] == np.cumsum(dbl)[-1], f"{P.NAMES[gen]} sum {t}"
    # every thread's u32 values (cheap on the oracle)
    for t in range(count):
        ref = oracle.generate(gen, oracle.seed(gen, int(seeds[t])), n1)
        assert np.array_equal(got[0][t], ref), f"{P.NAMES[gen]} thread {t}"
