"""ctypes loader for the oracle's serial C nests (test infrastructure only).

The shared object is built from ``oracle/nests.c`` with gcc at -O2 and
``-ffp-contract=off`` so that every FP32 expression is evaluated exactly in the
order written.  ``build()`` compiles it; ``lib()`` loads it (building first if
it is missing).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nests.c")
_SO = os.path.join(_HERE, "liboracle_nests.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force=True):
    """Compile nests.c into liboracle_nests.so (always, when force)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64

_SIGS = {
    "or_sm64_mix": (ctypes.c_uint64, [ctypes.c_uint64]),
    "or_sm64_nth": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
    "or_init_uniform": (None, [_f32p, _i64, ctypes.c_uint64, ctypes.c_uint32]),
    "or_gemm_f32": (None, [_f32p, _f32p, _f32p, _i64, _i64, _i64]),
    "or_gemm_f64": (None, [_f32p, _f32p, _f64p, _i64, _i64, _i64]),
    "or_gemm_bf16": (None, [_u16p, _u16p, _f32p, _i64, _i64, _i64]),
    "or_gemm_bf16_f64": (None, [_u16p, _u16p, _f64p, _i64, _i64, _i64]),
    "or_gemm_split_f64": (None, [_f32p, _f32p, _f64p, _i64, _i64, _i64, ctypes.c_int]),
    "or_e4m3_value": (ctypes.c_double, [ctypes.c_uint8]),
    "or_e4m3_rne": (ctypes.c_uint8, [ctypes.c_double]),
    "or_e4m3_scale": (ctypes.c_double, [ctypes.c_double]),
    "or_add_scaled": (None, [_f32p, _f32p, ctypes.c_float, _i64]),
    "or_avg2": (None, [_f32p, _f32p, _f32p, _i64]),
    "or_scale": (None, [_f32p, ctypes.c_float, _i64]),
    "or_copy": (None, [_f32p, _f32p, _i64]),
    "or_cast_bf16": (None, [_u16p, _f32p, _i64]),
    "or_transpose": (None, [_f32p, _f32p, _i64, _i64]),
    "or_sumsq": (None, [_f32p, _i64, _f64p]),
    "or_stencil19": (None, [_f32p, _f32p, _i64, _i64, _i64, _f64p]),
    "or_stencil19_f64": (None, [_f64p, _f64p, _i64, _i64, _i64, _f64p]),
    "or_copy_interior": (None, [_f32p, _f32p, _i64, _i64, _i64]),
    "or_copy_interior_f64": (None, [_f64p, _f64p, _i64, _i64, _i64]),
    "or_sin_field": (None, [ctypes.c_void_p, ctypes.c_void_p, _i64, _i64, _i64, ctypes.c_int32]),
    "or_rec_prefix": (None, [_f32p, _f32p, _i64, _i64]),
    "or_rec_decay": (None, [_f32p, _f32p, _i64, _i64]),
    "or_lcg_fill": (None, [_f32p, _i64, ctypes.c_uint32]),
    "or_lcg_states": (None, [_u32p, _i64, ctypes.c_uint32]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ----------------------------------------------------------------- wrappers
def sm64_mix(z):
    return lib().or_sm64_mix(z & 0xFFFFFFFFFFFFFFFF)


def sm64_nth(s, k):
    return lib().or_sm64_nth(s & 0xFFFFFFFFFFFFFFFF, k)


def init_uniform(n, seed, stream):
    x = np.empty(n, np.float32)
    lib().or_init_uniform(x, n, seed, stream)
    return x


def gemm_f32(A, B):
    M, Kd = A.shape
    N = B.shape[1]
    C = np.empty((M, N), np.float32)
    lib().or_gemm_f32(np.ascontiguousarray(A), np.ascontiguousarray(B), C, M, N, Kd)
    return C


def gemm_f64(A, B):
    M, Kd = A.shape
    N = B.shape[1]
    C = np.empty((M, N), np.float64)
    lib().or_gemm_f64(np.ascontiguousarray(A), np.ascontiguousarray(B), C, M, N, Kd)
    return C


def gemm_bf16(A16, B16):
    M, Kd = A16.shape
    N = B16.shape[1]
    C = np.empty((M, N), np.float32)
    lib().or_gemm_bf16(np.ascontiguousarray(A16), np.ascontiguousarray(B16), C, M, N, Kd)
    return C


def gemm_bf16_f64(A16, B16):
    M, Kd = A16.shape
    N = B16.shape[1]
    C = np.empty((M, N), np.float64)
    lib().or_gemm_bf16_f64(np.ascontiguousarray(A16), np.ascontiguousarray(B16), C, M, N, Kd)
    return C


SPLIT_VARIANTS = {"bf16x3": 1, "fp8x2": 2}


def gemm_split_f64(A, B, prec):
    """Split-precision product (hi/lo split, one refinement pass), FP64 sum."""
    M, Kd = A.shape
    N = B.shape[1]
    C = np.empty((M, N), np.float64)
    lib().or_gemm_split_f64(np.ascontiguousarray(A, np.float32), np.ascontiguousarray(B, np.float32), C, M, N, Kd,
                            SPLIT_VARIANTS[prec])
    return C


def e4m3_value(code):
    return lib().or_e4m3_value(int(code))


def e4m3_rne(x):
    return lib().or_e4m3_rne(float(x))


def e4m3_scale(amax):
    return lib().or_e4m3_scale(float(amax))


def add_scaled(C, A, alpha):
    lib().or_add_scaled(C.reshape(-1), np.ascontiguousarray(A).reshape(-1), alpha, C.size)


def avg2(S, X, Y):
    lib().or_avg2(S.reshape(-1), X.reshape(-1), Y.reshape(-1), S.size)


def scale(D, beta):
    lib().or_scale(D.reshape(-1), beta, D.size)


def copy(dst, src):
    lib().or_copy(dst.reshape(-1), src.reshape(-1), dst.size)


def cast_bf16(src):
    dst = np.empty(src.shape, np.uint16)
    lib().or_cast_bf16(dst.reshape(-1), np.ascontiguousarray(src).reshape(-1), src.size)
    return dst


def transpose(X):
    R, Cc = X.shape
    T = np.empty((Cc, R), np.float32)
    lib().or_transpose(np.ascontiguousarray(X), T, R, Cc)
    return T


def sumsq(x, s):
    lib().or_sumsq(np.ascontiguousarray(x).reshape(-1), x.size, s)


def stencil19(p, q, res_slot):
    I, J, K = p.shape
    lib().or_stencil19(p, q, I, J, K, res_slot)


def stencil19_f64(p, q, res_slot):
    I, J, K = p.shape
    lib().or_stencil19_f64(p, q, I, J, K, res_slot)


def copy_interior(p, q):
    I, J, K = p.shape
    if p.dtype == np.float64:
        lib().or_copy_interior_f64(p, q, I, J, K)
    else:
        lib().or_copy_interior(p, q, I, J, K)


def sin_field(I, J, K, m, want64=False):
    out32 = np.empty((I, J, K), np.float32)
    out64 = np.empty((I, J, K), np.float64) if want64 else None
    lib().or_sin_field(out32.ctypes.data, out64.ctypes.data if want64 else None, I, J, K, m)
    return (out32, out64) if want64 else out32


def rec_prefix(v, S):
    N, ld = S.shape
    lib().or_rec_prefix(v, np.ascontiguousarray(S).reshape(-1), v.shape[0], ld)


def rec_decay(w, p):
    I, J, K = p.shape
    lib().or_rec_decay(w, np.ascontiguousarray(p).reshape(-1), J, K)


def lcg_fill(L, seed32):
    lib().or_lcg_fill(L.reshape(-1), L.size, seed32 & 0xFFFFFFFF)


def lcg_states(n, seed32):
    out = np.empty(n, np.uint32)
    lib().or_lcg_states(out, n, seed32 & 0xFFFFFFFF)
    return out
