"""ctypes wrapper around the plain C oracle (test infrastructure only).

States are numpy ``uint8`` arrays holding the generator's POD state blob; the
layout is the one the public C ABI documents, so a state can be handed from
one side to the other.  Distances are Python ints (up to 512 bits).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SRC = os.path.join(HERE, "prand_oracle.c")
ORACLE_SO = os.path.join(HERE, "liboracle.so")

NLIMB = 8


def build_oracle(force=True):
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if not force and os.path.exists(ORACLE_SO):
        return ORACLE_SO
    tmp = ORACLE_SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-Wall", "-o", tmp, ORACLE_SRC])
    os.replace(tmp, ORACLE_SO)
    return ORACLE_SO


def to_limbs(n):
    if n < 0 or n >= 1 << (64 * NLIMB):
        raise ValueError("distance out of range")
    return (ctypes.c_uint64 * NLIMB)(*[(n >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(NLIMB)])


class Oracle:
    MT19937, MRG32K3A, LFSR113, GM19, GM29, GM31, GM55, GM61, GQ58X1, GQ58X3, GQ58X4 = range(11)
    NAMES = ["MT19937", "MRG32K3A", "LFSR113", "GM19", "GM29", "GM31", "GM55", "GM61",
             "GQ58.1", "GQ58.3", "GQ58.4"]
    U32, F32, F64 = 0, 1, 2
    DEFAULT, SEQ, SHORT, MEDIUM, LONG = range(5)
    PW = 312
    _DT = {0: np.uint32, 1: np.float32, 2: np.float64}

    def __init__(self, so_path=None):
        path = so_path or ORACLE_SO
        if not os.path.exists(path):
            build_oracle()
        lib = ctypes.CDLL(path)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        p64 = ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "or_state_bytes": (i32, [i32]),
            "or_default_seed": (u64, [i32]),
            "or_seed": (i32, [i32, u64, vp]),
            "or_init_default": (i32, [i32, vp]),
            "or_skipahead": (i32, [i32, vp, p64, i32]),
            "or_block_log2": (i32, [i32, i32]),
            "or_stream_distance": (i32, [i32, i32, u64, p64]),
            "or_init_stream": (i32, [i32, i32, vp, u64, vp]),
            "or_generate": (i32, [i32, vp, i32, vp, u64]),
            "or_mt_charpoly": (i32, [p64]),
            "or_mt_jump_poly": (i32, [p64, i32, p64]),
            "or_mt_reduce_bitwise": (i32, [p64]),
            "or_mt_reduce_words": (i32, [p64]),
            "or_mt_frobenius": (i32, [i32, p64]),
            "or_mt_poly_mulmod": (i32, [p64, p64, p64]),
            "or_mt_apply_poly": (i32, [vp, p64]),
            "or_mat3_pow": (i32, [p64, u64, p64, i32, p64]),
            "or_gm_generic_step": (i32, [u64, u64, u64, p64, p64]),
            "or_gm_generic_jump": (i32, [u64, u64, u64, p64, i32, p64, p64]),
            "or_lfsr_comp_step": (ctypes.c_uint32, [ctypes.c_uint32, i32, i32, i32]),
            "or_lfsr_comp_jump": (ctypes.c_uint32, [ctypes.c_uint32, i32, i32, i32, p64, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype, f.argtypes = res, args
        self.lib = lib

    # ---- helpers ----
    @staticmethod
    def _ptr(a):
        return ctypes.c_void_p(a.ctypes.data)

    def _check(self, rc, what):
        if rc < 0:
            raise RuntimeError(f"oracle {what} failed with {rc}")
        return rc

    # ---- states ----
    def state_bytes(self, gen):
        return self._check(self.lib.or_state_bytes(gen), "state_bytes")

    def new_state(self, gen):
        return np.zeros(self.state_bytes(gen), dtype=np.uint8)

    def default_seed(self, gen):
        return self.lib.or_default_seed(gen)

    def seed(self, gen, seed):
        st = self.new_state(gen)
        self._check(self.lib.or_seed(gen, seed, self._ptr(st)), "seed")
        return st

    def init_default(self, gen):
        st = self.new_state(gen)
        self._check(self.lib.or_init_default(gen, self._ptr(st)), "init_default")
        return st

    def skipahead(self, gen, st, distance):
        """Jump ``st`` (modified in place) ahead by ``distance`` outputs."""
        self._check(self.lib.or_skipahead(gen, self._ptr(st), to_limbs(distance), NLIMB), "skipahead")
        return st

    def block_log2(self, gen, variant=0):
        return self.lib.or_block_log2(gen, variant)

    def stream_distance(self, gen, variant, sid):
        out = (ctypes.c_uint64 * NLIMB)()
        self._check(self.lib.or_stream_distance(gen, variant, sid, out), "stream_distance")
        return sum(int(out[i]) << (64 * i) for i in range(NLIMB))

    def init_stream(self, gen, variant, sid, base=None):
        st = self.new_state(gen)
        bp = self._ptr(base) if base is not None else None
        self._check(self.lib.or_init_stream(gen, variant, bp, sid, self._ptr(st)), "init_stream")
        return st

    def generate(self, gen, st, n, dtype=0):
        """n outputs from ``st`` (advanced in place) as a numpy array."""
        out = np.empty(n, dtype=self._DT[dtype])
        self._check(self.lib.or_generate(gen, self._ptr(st), dtype, self._ptr(out), n), "generate")
        return out

    def generate_into(self, gen, st, dtype, out):
        """Same as generate, writing into a caller-provided contiguous array."""
        self._check(self.lib.or_generate(gen, self._ptr(st), dtype, self._ptr(out), out.size), "generate")
        return out

    # ---- building blocks for the pins ----
    def mt_charpoly(self):
        """Characteristic polynomial of the MT19937 transition as an int (bit i = x^i)."""
        buf = (ctypes.c_uint64 * self.PW)()
        deg = self._check(self.lib.or_mt_charpoly(buf), "mt_charpoly")
        return (1 << deg) | sum(int(buf[i]) << (64 * i) for i in range(self.PW))

    def mt_jump_poly(self, n):
        buf = (ctypes.c_uint64 * self.PW)()
        self._check(self.lib.or_mt_jump_poly(to_limbs(n), NLIMB, buf), "mt_jump_poly")
        return sum(int(buf[i]) << (64 * i) for i in range(self.PW))

    def mt_frobenius(self, n):
        """x^(2^n) mod phi as an int."""
        buf = (ctypes.c_uint64 * self.PW)()
        self._check(self.lib.or_mt_frobenius(n, buf), "mt_frobenius")
        return sum(int(buf[i]) << (64 * i) for i in range(self.PW))

    def _poly_words(self, poly):
        return (ctypes.c_uint64 * self.PW)(*[(poly >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(self.PW)])

    def mt_poly_mulmod(self, a, b):
        """a * b mod phi for reduced polynomials given as ints."""
        out = (ctypes.c_uint64 * self.PW)()
        self._check(self.lib.or_mt_poly_mulmod(self._poly_words(a), self._poly_words(b), out), "mt_poly_mulmod")
        return sum(int(out[i]) << (64 * i) for i in range(self.PW))

    def mt_apply_poly(self, st, g):
        """g(A) applied in place to an MT19937 state at a block boundary."""
        self._check(self.lib.or_mt_apply_poly(self._ptr(st), self._poly_words(g)), "mt_apply_poly")
        return st

    def mt_reduce(self, poly, bitwise):
        nw = 2 * self.PW + 2
        buf = (ctypes.c_uint64 * nw)(*[(poly >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(nw)])
        f = self.lib.or_mt_reduce_bitwise if bitwise else self.lib.or_mt_reduce_words
        self._check(f(buf), "mt_reduce")
        return sum(int(buf[i]) << (64 * i) for i in range(nw))

    def mat3_pow(self, M, m, n):
        a = (ctypes.c_uint64 * 9)(*[int(v) % m for row in M for v in row])
        out = (ctypes.c_uint64 * 9)()
        self._check(self.lib.or_mat3_pow(a, m, to_limbs(n), NLIMB, out), "mat3_pow")
        return [[int(out[3 * i + j]) for j in range(3)] for i in range(3)]

    def gm_generic_step(self, k, q, g, xc, xp):
        c, p = ctypes.c_uint64(xc), ctypes.c_uint64(xp)
        self._check(self.lib.or_gm_generic_step(k, q, g, ctypes.byref(c), ctypes.byref(p)), "gm_step")
        return c.value, p.value

    def gm_generic_jump(self, k, q, g, n, xc, xp):
        c, p = ctypes.c_uint64(xc), ctypes.c_uint64(xp)
        self._check(self.lib.or_gm_generic_jump(k, q, g, to_limbs(n), NLIMB, ctypes.byref(c),
                                                ctypes.byref(p)), "gm_jump")
        return c.value, p.value

    def lfsr_comp_step(self, z, p, q, s):
        return self.lib.or_lfsr_comp_step(z, p, q, s)

    def lfsr_comp_jump(self, z, p, q, s, n):
        return self.lib.or_lfsr_comp_jump(z, p, q, s, to_limbs(n), NLIMB)


# state layouts (the public ABI's POD blobs, restated for the tests)
def mt_words(st):
    """(mt[624], mti) of an MT19937 state blob."""
    w = st.view(np.uint32)
    return w[:624], int(w[624])


def gm_arrays(st):
    """(xp[32], xc[32], off) of a GM/GQ state blob."""
    w64 = st[:512].view(np.uint64)
    off = int(st[512:516].view(np.uint32)[0])
    return w64[:32], w64[32:64], off
