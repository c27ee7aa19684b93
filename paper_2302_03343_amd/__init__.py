"""MI355X-native VEGAS hot path (HIP kernels behind the C ABI of libvgx.so).

`paper_2302_03343_amd.vgx` is the ctypes binding (same names as the C entry
points in include/vgx.h); `paper_2302_03343_amd.build` compiles the library.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libvgx.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vgx.h")


def lib_built():
    return os.path.exists(LIB_PATH)
