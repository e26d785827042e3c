"""Many-stream generation of GM55, GQ58.3 and GQ58.4, whose kernel runs one
lane per section of a stream: sizes whose last section is shorter than one
GQ58.3 block (its final state is then the section's start state, written
over the input the other sections of the stream read), seeded states that
have not collapsed yet, block-split states, and GQ58.3 states inside a
block, in every dtype, states updated in place; outputs and final states
equal the oracle's."""
import numpy as np
import pytest
import torch

from paper_1307_5869_amd import prand as P

pytestmark = pytest.mark.gpu

TDT = {P.U32: torch.int32, P.F32: torch.float32, P.F64: torch.float64}
NPDT = {P.U32: np.uint32, P.F32: np.float32, P.F64: np.float64}
LANE_GENS = [P.GM55, P.GQ58X3, P.GQ58X4]


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def start_states(oracle, gen, count, kind):
    if kind == "seeded":   # exact (not yet collapsed) composite states
        return [oracle.seed(gen, 900 + 13 * i) for i in range(count)]
    sts = [oracle.init_stream(gen, 0, 10**18 + 97 * i) for i in range(count)]
    if kind == "offset":   # GQ58.3: 5 words into a block
        for st in sts:
            oracle.generate(gen, st, 5)
    return sts


# one stream of 5082 words runs 64 sections of 108 words, the last one 6 long
@pytest.mark.parametrize("count,n", [(1, 5082), (3, 5077), (2, 6913), (1, 2311), (4, 130)])
@pytest.mark.parametrize("kind", ["seeded", "split", "offset"])
@pytest.mark.parametrize("dtype", [P.U32, P.F32, P.F64])
@pytest.mark.parametrize("gen", LANE_GENS)
def test_lane_sections_match_oracle(ctx, oracle, gen, dtype, kind, count, n):
    states = start_states(oracle, gen, count, kind)
    d = torch.from_numpy(np.concatenate(states)).cuda()
    out = torch.empty(count * n, dtype=TDT[dtype], device="cuda")
    ctx.generate_streams(gen, d, count, n, dtype, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(NPDT[dtype]).reshape(count, n)
    sb = P.state_bytes(gen)
    got_st = d.cpu().numpy().reshape(count, sb)
    for i, st in enumerate(states):
        ref = oracle.generate(gen, st, n, dtype)
        np.testing.assert_array_equal(got[i], ref, err_msg=f"{P.NAMES[gen]} {kind} stream {i}")
        assert np.array_equal(got_st[i], st), f"{P.NAMES[gen]} {kind} state {i}"
