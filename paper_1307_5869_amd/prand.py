"""Thin ctypes binding of libprand.so (argument marshalling only).

Every ``prand_*`` function of ``include/prand.h`` is exposed under the same
name; :class:`Context` wraps them for torch tensors and numpy host states.
The library must have been built (``python -m paper_1307_5869_amd.build``);
there is no fallback of any kind.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprand.so")

MT19937, MRG32K3A, LFSR113, GM19, GM29, GM31, GM55, GM61, GQ58X1, GQ58X3, GQ58X4 = range(11)
NUM_GENERATORS = 11
NAMES = ["MT19937", "MRG32K3A", "LFSR113", "GM19", "GM29", "GM31", "GM55", "GM61", "GQ58.1", "GQ58.3", "GQ58.4"]
U32, F32, F64 = 0, 1, 2
SEQ_DEFAULT, SEQ, SEQ_SHORT, SEQ_MEDIUM, SEQ_LONG = range(5)
OK, EINVAL, EUNSUPPORTED, ERANGE, EHIP, ENOMEM, ENODEV, EBUSY, ENOTREADY = 0, -1, -2, -3, -4, -5, -6, -7, -8
NOALLOC_SCRATCH_BYTES = 4 << 20
MAX_LIMBS = 8

_u64, _u32, _i32, _vp, _sz = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
_SIGNATURES = {
    "prand_strerror": (ctypes.c_char_p, [_i32]),
    "prand_last_hip_error": (_i32, [_vp]),
    "prand_ctx_create": (_i32, [ctypes.POINTER(_vp), _i32]),
    "prand_ctx_destroy": (_i32, [_vp]),
    "prand_state_bytes": (_sz, [_i32]),
    "prand_block_log2": (_i32, [_i32, _i32]),
    "prand_independence_limit": (_i32, [_i32, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "prand_init_default": (_i32, [_vp, _i32, _vp]),
    "prand_seed": (_i32, [_vp, _i32, _u64, _vp]),
    "prand_seed_host": (_i32, [_i32, _u64, _vp]),
    "prand_init_default_host": (_i32, [_i32, _vp]),
    "prand_seed_dev": (_i32, [_vp, _i32, _vp, _u32, _vp, _vp]),
    "prand_skipahead": (_i32, [_vp, _i32, _vp, _vp, _i32]),
    "prand_skipahead_dev": (_i32, [_vp, _i32, _vp, _u32, _vp, _i32, _i32, _vp]),
    "prand_init_stream": (_i32, [_vp, _i32, _i32, _u64, _vp]),
    "prand_init_streams_dev": (_i32, [_vp, _i32, _i32, _vp, _vp, _u32, _vp, _vp]),
    "prand_generate": (_i32, [_vp, _i32, _vp, _i32, _vp, _u64, _vp]),
    "prand_generate_noalloc": (_i32, [_vp, _i32, _vp, _i32, _vp, _u64, _vp]),
    "prand_generate_array": (_i32, [_vp, _i32, _vp, _i32, _vp, _u64]),
    "prand_generate_streams": (_i32, [_vp, _i32, _vp, _u32, _u64, _i32, _vp, _vp]),
    "prand_batch_create": (_i32, [_vp, _vp, _u32, _vp, ctypes.POINTER(_vp)]),
    "prand_batch_launch": (_i32, [_vp, _vp]),
    "prand_batch_tiles": (_i32, [_vp, ctypes.POINTER(_u32)]),
    "prand_batch_destroy": (_i32, [_vp]),
    "prand_batch_autotune": (_i32, [_vp, _vp, _u32, _vp]),
    "prand_server_create": (_i32, [_vp, _vp, ctypes.POINTER(_vp)]),
    "prand_server_submit": (_i32, [_vp, _vp, ctypes.POINTER(_u64)]),
    "prand_server_poll": (_i32, [_vp, _vp, _u32, ctypes.POINTER(_u32), _i32]),
    "prand_server_release": (_i32, [_vp, _u64]),
    "prand_server_get_stats": (_i32, [_vp, _vp]),
    "prand_server_clock": (ctypes.c_double, [_vp]),
    "prand_server_destroy": (_i32, [_vp]),
    "prand_simd_state_bytes": (_sz, []),
    "prand_get_simd_state": (_i32, [_i32, _vp, _vp]),
    "prand_simd_next": (_u32, [_vp]),
    "prand_simd_fill": (_i32, [_vp, _i32, _vp, _u64]),
    "prand_simd_vectorized": (_i32, [_vp]),
}


class Task(ctypes.Structure):
    """struct prand_task"""
    _fields_ = [("gen", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_uint64),
                ("state_in", ctypes.c_void_p), ("state_out", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    """struct prand_batch_config (zeros select the defaults)"""
    _fields_ = [("waves_per_block", ctypes.c_uint32), ("reg_section", ctypes.c_uint32),
                ("gm_section", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("lds_chunk_words", ctypes.c_uint32), ("overlap", ctypes.c_uint32)]



class ServerConfig(ctypes.Structure):
    """struct prand_server_config (zeros select the defaults)"""
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("iter_numbers", ctypes.c_uint64), ("min_chunk", ctypes.c_uint64),
                ("mt_chunk", ctypes.c_uint64), ("mt_section", ctypes.c_uint64), ("max_active", ctypes.c_uint32), ("max_queue", ctypes.c_uint32),
                ("waves_per_block", ctypes.c_uint32), ("reg_section", ctypes.c_uint32),
                ("gm_section", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class Request(ctypes.Structure):
    """struct prand_request"""
    _fields_ = [("gen", ctypes.c_int32), ("variant", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("stream_id", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    """struct prand_completion"""
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("gen", ctypes.c_int32), ("dtype", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    """struct prand_server_stats"""
    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "admitted", "rejected", "completed", "released",
                                                "numbers", "iterations", "hbm_budget", "hbm_used", "hbm_peak")] + \
               [("waiting", ctypes.c_uint32), ("active", ctypes.c_uint32), ("gpu_busy_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


class PrandError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


def load():
    """Load libprand.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with python -m paper_1307_5869_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
        _lib = lib
    return _lib


def strerror(code):
    return load().prand_strerror(code).decode()


def _chk(rc, what):
    if rc != OK:
        raise PrandError(rc, what)


def limbs(n):
    """A non-negative int as 8 little-endian uint64 limbs."""
    if n < 0 or n >= 1 << (64 * MAX_LIMBS):
        raise ValueError("distance out of range")
    return np.array([(n >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(MAX_LIMBS)], dtype=np.uint64)


def _ptr(x):
    """Device or host address of a torch tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("host buffers must be contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("device buffers must be contiguous")
        return x.data_ptr()
    raise TypeError(f"cannot pass {type(x)}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def state_bytes(gen):
    return load().prand_state_bytes(gen)


def block_log2(gen, variant=SEQ_DEFAULT):
    return load().prand_block_log2(gen, variant)


def independence_limit(gen, variant=SEQ_DEFAULT):
    a, b = ctypes.c_double(), ctypes.c_double()
    _chk(load().prand_independence_limit(gen, variant, ctypes.byref(a), ctypes.byref(b)), "independence_limit")
    return a.value, b.value


def seed_host(gen, seed):
    """prand_seed_host: the seeded state, computed on the CPU (no context)."""
    st = np.zeros(state_bytes(gen), dtype=np.uint8)
    _chk(load().prand_seed_host(gen, seed, st.ctypes.data), "seed_host")
    return st


def init_default_host(gen):
    """prand_init_default_host: the default state, computed on the CPU."""
    st = np.zeros(state_bytes(gen), dtype=np.uint8)
    _chk(load().prand_init_default_host(gen, st.ctypes.data), "init_default_host")
    return st


class SimdState:
    """A CPU SIMD state (prand_get_simd_state) continuing a plain host state
    blob; next() and fill() are prand_simd_next / prand_simd_fill."""

    def __init__(self, gen, state):
        lib = load()
        self.blob = np.zeros(lib.prand_simd_state_bytes(), dtype=np.uint8)
        _chk(lib.prand_get_simd_state(gen, _ptr(np.ascontiguousarray(state)), _ptr(self.blob)), "get_simd_state")

    def next(self):
        return load().prand_simd_next(_ptr(self.blob))

    def fill(self, dtype, n):
        out = np.empty(n, dtype={U32: np.uint32, F32: np.float32, F64: np.float64}[dtype])
        _chk(load().prand_simd_fill(_ptr(self.blob), dtype, _ptr(out), n), "simd_fill")
        return out

    @property
    def vectorized(self):
        return bool(load().prand_simd_vectorized(_ptr(self.blob)))


class Context:
    """A libprand context on one HIP device."""

    def __init__(self, device=0):
        lib = load()
        h = _vp()
        _chk(lib.prand_ctx_create(ctypes.byref(h), device), "prand_ctx_create")
        self.handle = h
        self.device = device
        self.lib = lib

    def close(self):
        if self.handle:
            self.lib.prand_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        rc = getattr(self.lib, name)(self.handle, *args)
        if rc == EHIP:
            raise PrandError(rc, f"{name} (hipError {self.lib.prand_last_hip_error(self.handle)})")
        _chk(rc, name)

    # ---- host states (numpy uint8 blobs) ----
    def new_state(self, gen):
        return np.zeros(state_bytes(gen), dtype=np.uint8)

    def init_default(self, gen):
        st = self.new_state(gen)
        self._call("prand_init_default", gen, _ptr(st))
        return st

    def seed(self, gen, seed):
        st = self.new_state(gen)
        self._call("prand_seed", gen, seed, _ptr(st))
        return st

    def skipahead(self, gen, state, distance):
        d = limbs(distance)
        self._call("prand_skipahead", gen, _ptr(state), _ptr(d), MAX_LIMBS)
        return state

    def init_stream(self, gen, variant, sid):
        st = self.new_state(gen)
        self._call("prand_init_stream", gen, variant, sid, _ptr(st))
        return st

    def generate(self, gen, state, dtype, d_out, n, stream=None):
        self._call("prand_generate", gen, _ptr(state), dtype, _ptr(d_out), n, _stream(stream))
        return d_out

    def generate_array(self, gen, state, dtype, n):
        """n values from a host state into a new host (numpy) array."""
        out = np.empty(n, dtype={U32: np.uint32, F32: np.float32, F64: np.float64}[dtype])
        self._call("prand_generate_array", gen, _ptr(state), dtype, _ptr(out), n)
        return out

    def generate_noalloc(self, gen, state, dtype, d_out, n, stream=None):
        self._call("prand_generate_noalloc", gen, _ptr(state), dtype, _ptr(d_out), n, _stream(stream))
        return d_out

    # ---- device states (torch uint8 tensors of count * state_bytes) ----
    def seed_dev(self, gen, d_seeds, count, d_states, stream=None):
        self._call("prand_seed_dev", gen, _ptr(d_seeds), count, _ptr(d_states), _stream(stream))

    def skipahead_dev(self, gen, d_states, count, d_dist, nlimbs, per_stream, stream=None):
        self._call("prand_skipahead_dev", gen, _ptr(d_states), count, _ptr(d_dist), nlimbs, int(per_stream),
                   _stream(stream))

    def init_streams_dev(self, gen, variant, d_base, d_ids, count, d_states, stream=None):
        self._call("prand_init_streams_dev", gen, variant, _ptr(d_base), _ptr(d_ids), count, _ptr(d_states),
                   _stream(stream))

    def generate_streams(self, gen, d_states, count, n, dtype, d_out, stream=None):
        self._call("prand_generate_streams", gen, _ptr(d_states), count, n, dtype, _ptr(d_out), _stream(stream))


class Batch:
    """A planned batched launch (prand_batch_*).  `tasks`: iterable of
    (gen, dtype, n, state_in, state_out, out) with device buffers (torch
    tensors or addresses); the buffers must outlive the batch."""

    def __init__(self, ctx, tasks, config=None):
        self.ctx = ctx
        arr = (Task * max(1, len(tasks)))()
        for i, (gen, dtype, n, sin, sout, out) in enumerate(tasks):
            arr[i] = Task(gen, dtype, n, _ptr(sin), _ptr(sout), _ptr(out))
        self.ntasks = len(tasks)
        self._tasks = arr
        cfg = ctypes.byref(config) if config is not None else None
        h = _vp()
        rc = ctx.lib.prand_batch_create(ctx.handle, ctypes.cast(arr, _vp), len(tasks), cfg, ctypes.byref(h))
        _chk(rc, "prand_batch_create")
        self.handle = h

    def tiles(self):
        n = _u32()
        _chk(self.ctx.lib.prand_batch_tiles(self.handle, ctypes.byref(n)), "prand_batch_tiles")
        return n.value

    def launch(self, stream=None):
        _chk(self.ctx.lib.prand_batch_launch(self.handle, _stream(stream)), "prand_batch_launch")

    def close(self):
        if self.handle:
            self.ctx.lib.prand_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ctx, tasks):
    """prand_batch_autotune on the given tasks; returns a BatchConfig."""
    arr = (Task * max(1, len(tasks)))()
    for i, (gen, dtype, n, sin, sout, out) in enumerate(tasks):
        arr[i] = Task(gen, dtype, n, _ptr(sin), _ptr(sout), _ptr(out))
    best = BatchConfig()
    _chk(ctx.lib.prand_batch_autotune(ctx.handle, ctypes.cast(arr, _vp), len(tasks), ctypes.byref(best)),
         "prand_batch_autotune")
    return best


class Server:
    """A serving loop (prand_server_*) on a context's device."""

    def __init__(self, ctx, config=None):
        self.ctx = ctx
        h = _vp()
        cfg = ctypes.byref(config) if config is not None else None
        _chk(ctx.lib.prand_server_create(ctx.handle, cfg, ctypes.byref(h)), "prand_server_create")
        self.handle = h
        self._buf = (Completion * 1024)()

    def submit(self, gen, stream_id, n, dtype=U32, variant=SEQ_DEFAULT, tag=0):
        """Queue a request; returns its ticket (raises PrandError when rejected)."""
        req = Request(gen, variant, dtype, 0, stream_id, n, tag)
        t = _u64()
        _chk(self.ctx.lib.prand_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "prand_server_submit")
        return t.value

    def try_submit(self, gen, stream_id, n, dtype=U32, variant=SEQ_DEFAULT, tag=0):
        """As submit, but returns (rc, ticket) without raising."""
        req = Request(gen, variant, dtype, 0, stream_id, n, tag)
        t = _u64()
        rc = self.ctx.lib.prand_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t))
        return rc, t.value

    def poll(self, wait_ms=0, max_items=1024):
        """Completed requests (Completion structs copied out), oldest first."""
        n = _u32()
        m = min(max_items, len(self._buf))
        _chk(self.ctx.lib.prand_server_poll(self.handle, self._buf, m, ctypes.byref(n), int(wait_ms)),
             "prand_server_poll")
        out = []
        for i in range(n.value):
            c = Completion()
            ctypes.pointer(c)[0] = self._buf[i]
            out.append(c)
        return out

    def release(self, ticket):
        _chk(self.ctx.lib.prand_server_release(self.handle, ticket), "prand_server_release")

    def stats(self):
        st = ServerStats()
        _chk(self.ctx.lib.prand_server_get_stats(self.handle, ctypes.byref(st)), "prand_server_get_stats")
        return st.as_dict()

    def clock(self):
        return self.ctx.lib.prand_server_clock(self.handle)

    def close(self):
        if self.handle:
            self.ctx.lib.prand_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def __getattr__(name):
    # prand_* under their C names, for callers that want the raw ABI
    if name.startswith("prand_") and name in _SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)
