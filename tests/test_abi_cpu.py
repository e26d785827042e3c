"""CPU checks of the C ABI: the built library loads, exports every symbol the
header declares, and its host-only metadata (state sizes, block lengths,
Table 4 limits, error strings) and host-only seeding agree with the oracle and
the paper.  No GPU call is made here (no GPU in this environment)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1307_5869_amd import prand as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prand.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1307_5869_amd import prand
    if not os.path.exists(prand.LIB_PATH):
        from paper_1307_5869_amd import build
        build.build()
    return prand


def declared_functions():
    text = open(HEADER).read()
    # declarations start a line with their return type
    pat = r"^(?:int|size_t|double|uint32_t|const char\*)\s+(prand_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(pat, text, flags=re.M)))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ["prand_ctx_create", "prand_ctx_destroy", "prand_seed", "prand_skipahead", "prand_init_stream",
                 "prand_init_streams_dev", "prand_generate", "prand_generate_streams", "prand_skipahead_dev"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(so, name), name
    # and the binding knows every one of them
    assert set(declared_functions()) == set(lib._SIGNATURES)


def test_state_bytes_match_oracle(lib, oracle):
    for g in range(11):
        assert lib.state_bytes(g) == oracle.state_bytes(g)
    assert lib.state_bytes(11) == 0 and lib.state_bytes(-1) == 0


def test_block_lengths_match_oracle(lib, oracle):
    for g in range(11):
        for v in range(5):
            assert lib.block_log2(g, v) == oracle.block_log2(g, v), (g, v)
    assert lib.block_log2(11, 0) == lib.EINVAL
    assert lib.block_log2(0, 7) == lib.EINVAL


def test_independence_limits_are_table4(lib):
    gold = os.path.join(ROOT, "tests", "golden", "table4_streams.txt")
    names = ["mt19937", "mrg32k3a", "lfsr113", "gm19", "gm29", "gm31", "gm55", "gm61", "gq58x1", "gq58x3", "gq58x4"]
    var = {"init_sequence_": 1, "init_short_sequence_": 2, "init_medium_sequence_": 3, "init_long_sequence_": 4}
    for line in open(gold):
        if line.startswith("#") or not line.strip():
            continue
        fn, nseq, maxlen = line.split()
        gname, rest = fn.split("_", 1)
        a, b = lib.independence_limit(names.index(gname), var[rest])
        assert a == float(nseq) and b == float(maxlen)
    with pytest.raises(lib.PrandError):
        lib.independence_limit(0, 2)


def test_strerror(lib):
    for code in [0, -1, -2, -3, -4, -5, -6, -99]:
        assert isinstance(lib.strerror(code), str) and lib.strerror(code)


def test_null_arguments_rejected_without_device(lib):
    so = lib.load()
    assert so.prand_ctx_create(None, 0) == lib.EINVAL
    assert so.prand_ctx_destroy(None) == lib.OK
    # a context is required for every compute entry point
    assert so.prand_generate_streams(None, 0, None, 1, 1, 0, None, None) == lib.EINVAL
    assert so.prand_skipahead(None, 0, None, None, 0) == lib.EINVAL


def test_context_needs_gfx950(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.load().prand_ctx_create(ctypes.byref(h), 0) == lib.ENODEV


def test_mt_block_ladder_top_entry_matches_oracle(lib, oracle):
    """The whole-block jump table of batched MT19937 sections (sections of
    624 * 2^10 outputs, 22 entries): its last entry, used by sections whose
    number has bit 21 set, equals the oracle's x^(624 * 2^31) mod phi, and
    the table's x^(-1) times x is 1 mod phi.  Host code only."""
    so = ctypes.CDLL(lib.LIB_PATH)
    f = so.prand_internal_mt_block_poly
    f.restype = ctypes.c_int
    out, inv = (ctypes.c_uint32 * 624)(), (ctypes.c_uint32 * 624)()
    assert f(10, 21, out, inv) == 0
    as_int = lambda a: sum(int(a[w]) << (32 * w) for w in range(624))
    assert as_int(out) == oracle.mt_jump_poly(624 << 31)
    assert oracle.mt_reduce(as_int(inv) << 1, bitwise=False) == 1
    assert f(10, 3, out, inv) == 0
    assert as_int(out) == oracle.mt_jump_poly(624 << 13)


SEEDS = [0, 1, 127, 128, 12345, 2**31 - 1, 2**32 - 1, 2**32, 2**63 + 5, 2**64 - 1, 4294944443, 4294944442]


@pytest.mark.parametrize("gen", range(11))
def test_host_seeding_matches_oracle(oracle, gen):
    """prand_seed_host / prand_init_default_host: the library's seeding code
    run on the CPU, no context and no GPU, against the oracle (both
    branches of every generator's seeding: verbatim seeds and the SplitMix64
    expansion)."""
    for s in SEEDS:
        assert np.array_equal(P.seed_host(gen, s), oracle.seed(gen, s)), (P.NAMES[gen], s)
    assert np.array_equal(P.init_default_host(gen), oracle.init_default(gen)), P.NAMES[gen]


def test_host_seeding_errors(lib):
    lib = P.load()
    st = np.zeros(4096, dtype=np.uint8)
    assert lib.prand_seed_host(11, 1, st.ctypes.data) == P.EINVAL
    assert lib.prand_seed_host(-1, 1, st.ctypes.data) == P.EINVAL
    assert lib.prand_seed_host(0, 1, None) == P.EINVAL
    assert lib.prand_init_default_host(11, st.ctypes.data) == P.EINVAL
    assert lib.prand_init_default_host(3, None) == P.EINVAL
