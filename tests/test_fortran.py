"""Fortran bindings (include/prand.f90; the paper's "Fortran compatibility"):
test-side Fortran programs built with amdflang against libprand.so, run as
subprocesses, their output files compared with the oracle.

CPU: tests/fortran/simd_example.f90 -- a plain state from the oracle, made a
SIMD state and drawn from (single outputs, a u32 fill, an f64 fill, an error
code).  GPU: tests/fortran/gpu_array.f90 -- context, seeded state, host-array
fills in u32 and f64 (prand_generate_array), a skip-ahead."""
import os
import subprocess

import numpy as np
import pytest

from paper_1307_5869_amd import prand as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "fortran", "bin")


def program(name):
    exe = os.path.join(BIN, name)
    if not os.path.exists(exe):
        from paper_1307_5869_amd import build

        if not os.path.exists(P.LIB_PATH):
            build.build()
        build.build_fortran()
    return exe


def run(args, timeout=120):
    r = subprocess.run(args, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, f"{args[0]} exited {r.returncode}: {r.stdout} {r.stderr}"


@pytest.mark.parametrize("gen", [P.MT19937, P.MRG32K3A, P.LFSR113, P.GM19, P.GM55, P.GM61, P.GQ58X3, P.GQ58X4])
def test_fortran_simd_matches_oracle(oracle, gen, tmp_path):
    st = oracle.seed(gen, 4321 + gen)
    if gen in (P.MT19937, P.GQ58X3):
        oracle.generate(gen, st, 3)   # start inside a block
    fin, fout = tmp_path / "state.bin", tmp_path / "out.bin"
    st.tofile(fin)
    n = 5000
    run([program("simd_example"), str(gen), str(fin), str(n), str(fout)])
    got = np.fromfile(fout, dtype=np.uint32)
    ref = oracle.generate(gen, st, n + 3)
    np.testing.assert_array_equal(got, ref, err_msg=P.NAMES[gen])
    dbl = np.fromfile(str(fout) + ".f64", dtype=np.float64)
    np.testing.assert_array_equal(dbl, oracle.generate(gen, st, 5, P.F64), err_msg=P.NAMES[gen])


@pytest.mark.gpu
@pytest.mark.parametrize("gen", [P.MT19937, P.MRG32K3A, P.LFSR113, P.GM31, P.GQ58X3])
def test_fortran_gpu_array_matches_oracle(oracle, gen, tmp_path):
    seed, n, skip = 2**40 + 17 * gen, 70001, 10**9 + 7
    prefix = tmp_path / "run"
    run([program("gpu_array"), str(gen), str(seed), str(n), str(skip), str(prefix)], timeout=300)
    st = oracle.seed(gen, seed)
    np.testing.assert_array_equal(np.fromfile(str(prefix) + ".u32", dtype=np.uint32), oracle.generate(gen, st, n),
                                  err_msg=P.NAMES[gen])
    np.testing.assert_array_equal(np.fromfile(str(prefix) + ".f64", dtype=np.float64),
                                  oracle.generate(gen, st, n, P.F64), err_msg=P.NAMES[gen])
    oracle.skipahead(gen, st, skip)
    got = np.fromfile(str(prefix) + ".state", dtype=np.uint8)
    # a jumped MT19937 window is a canonical form of the same point: compare what follows
    np.testing.assert_array_equal(oracle.generate(gen, got.copy(), 2000), oracle.generate(gen, st.copy(), 2000),
                                  err_msg=P.NAMES[gen])
