"""ctypes loader of the C generators (mspgen/gen.c), built with gcc on demand."""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libmspgen.so")
_lib = None


def build() -> str:
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
        L.gen_er_counts.argtypes = [i64, i64, ctypes.c_double, u64, vp]
        L.gen_er_fill.argtypes = [i64, i64, ctypes.c_double, u64, vp, vp]
        L.gen_er_rows_counts.argtypes = [i64, vp, i64, ctypes.c_double, u64, vp]
        L.gen_er_rows_fill.argtypes = [i64, vp, i64, ctypes.c_double, u64, vp, vp]
        L.gen_bfs_counts.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp]
        L.gen_bfs_counts.restype = ctypes.c_int
        L.gen_bfs_lists.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.gen_bfs_lists.restype = ctypes.c_int
        L.gen_lists_to_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
