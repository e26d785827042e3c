"""Loader for the test-side user kernels of tests/devapi (built by
paper_1307_5869_amd.build.build_test_kernels, and here when missing)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "devapi", "libuser_kernel.so")

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            from paper_1307_5869_amd import build
            build.build_test_kernels()
        lib = ctypes.CDLL(LIB)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        lib.devapi_state_bytes.restype, lib.devapi_state_bytes.argtypes = ctypes.c_size_t, [i32]
        lib.devapi_draw.restype, lib.devapi_draw.argtypes = i32, [i32, i32, vp, u32, u64, vp, vp]
        lib.devapi_sum.restype, lib.devapi_sum.argtypes = i32, [i32, vp, u32, u64, vp, vp]
        lib.hostapi_draw.restype, lib.hostapi_draw.argtypes = i32, [i32, i32, vp, u32, u64, vp]
        _lib = lib
    return _lib
