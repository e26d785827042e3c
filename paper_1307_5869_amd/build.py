"""Build libprand.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to its own object in parallel; the objects link into
``paper_1307_5869_amd/libprand.so``.  Run ``python -m paper_1307_5869_amd.build``.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libprand.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # conversions and the exact FP64 reductions must not be contracted
    "-ffp-contract=off",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# pure host sources (no HIP): the host compiler, with the x86 carry-less multiply
HOST_CXX = os.environ.get("CXX", "g++")
HOST_SOURCES = {"mt_poly.cpp", "simd_host.cpp"}
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-mpclmul", "-msse4.1", "-pthread", "-I", CSRC, "-I", INCLUDE]
# the CPU SIMD realizations: AVX2/FMA only inside functions that carry the
# target attribute (chosen at run time); no contraction of the exact FP64
# reductions
HOST_SOURCE_FLAGS = {"simd_host.cpp": ["-O3", "-ffp-contract=off"]}


# per-source extra device flags: the MT19937 jump kernel scans jump
# coefficients with uniform branches joined by gotos; left unstructured they
# compile to one scalar compare and branch per coefficient.  Without hoisting
# of common code the test of the next bit, which both successors of a test
# make, stays a plain compare and branch in each (hoisted, it is carried as
# a lane mask and costs three more scalar instructions per group).
# Tail merging is off so that the repeated tests after each pair of
# coefficients (mt_pairs.inc) stay in place.
SOURCE_FLAGS = {"k_mt19937.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions",
                                  "-mllvm", "-simplifycfg-hoist-common=false",
                                  "-mllvm", "-enable-tail-merge=false"]}


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if os.path.basename(src) in HOST_SOURCES:
        cmd = [HOST_CXX] + HOST_FLAGS + HOST_SOURCE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    else:
        cmd = [HIPCC] + FLAGS + SOURCE_FLAGS.get(os.path.basename(src), []) + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    # -z defs: a symbol that no object defines fails the link instead of the load
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-Wl,-z,defs", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# test-side user kernels built on include/prand_device.h (not part of the
# library): tests/devapi/*.hip -> tests/devapi/lib<name>.so
TEST_KERNELS = os.path.join(ROOT, "tests", "devapi")


def build_test_kernels(verbose=False):
    built = []
    for f in sorted(os.listdir(TEST_KERNELS)):
        if not f.endswith(".hip"):
            continue
        src = os.path.join(TEST_KERNELS, f)
        lib = os.path.join(TEST_KERNELS, "lib" + f[:-4] + ".so")
        tmp = lib + ".tmp"
        cmd = [HIPCC] + FLAGS + ["-shared", "-x", "hip", src, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
        built.append(lib)
        if verbose:
            print("built", lib)
    return built


# Fortran: the binding module (include/prand.f90) and the test-side
# programs tests/fortran/*.f90 -> tests/fortran/bin/<name>, linked against
# libprand.so (found through an rpath relative to the program)
FC = os.environ.get("FC", "/opt/rocm/bin/amdflang")
FORTRAN_TESTS = os.path.join(ROOT, "tests", "fortran")


def build_fortran(verbose=False):
    mod_dir = os.path.join(BUILD, "fortran")
    bin_dir = os.path.join(FORTRAN_TESTS, "bin")
    os.makedirs(mod_dir, exist_ok=True)
    os.makedirs(bin_dir, exist_ok=True)
    mod_obj = os.path.join(mod_dir, "prand_mod.o")
    cmd = [FC, "-O2", "-J", mod_dir, "-c", os.path.join(INCLUDE, "prand.f90"), "-o", mod_obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"Fortran module failed:\n{r.stdout}\n{r.stderr}")
    built = []
    rpath = "-Wl,-rpath," + "$ORIGIN/" + os.path.relpath(HERE, bin_dir)
    for f in sorted(os.listdir(FORTRAN_TESTS)):
        if not f.endswith(".f90"):
            continue
        exe = os.path.join(bin_dir, f[:-4])
        cmd = [FC, "-O2", "-I", mod_dir, os.path.join(FORTRAN_TESTS, f), mod_obj, "-L", HERE, "-lprand", rpath,
               "-o", exe + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"Fortran build failed for {f}:\n{r.stdout}\n{r.stderr}")
        os.replace(exe + ".tmp", exe)
        built.append(exe)
        if verbose:
            print("built", exe)
    return built


if __name__ == "__main__":
    build(verbose=True)
    build_test_kernels(verbose=True)
    build_fortran(verbose=True)
    sys.exit(0)
