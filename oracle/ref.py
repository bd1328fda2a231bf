"""ctypes front end of the CPU oracle's plain definitions (ref.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the GPU path.
"""
import ctypes as C
import numpy as np

from .build import build

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        i32, i64, p = C.c_int32, C.c_int64, C.c_void_p
        L.oref_affine_xor.argtypes = [i32, i32, i32, i32, i64, i64, p]
        L.oref_affine_xor.restype = i64
        L.oref_fma_chain.argtypes = [p, i64, p, i32, p, i32, p, i64, i64, p]
        L.oref_fma_chain.restype = None
        L.oref_gather.argtypes = [p, i32, i64, i64, i64, p]
        L.oref_gather.restype = None
        L.oref_exact_sum.argtypes = [p, i64, p]
        L.oref_exact_sum.restype = C.c_double
        L.oref_fixed75_sum.argtypes = [p, i64, p, p]
        L.oref_fixed75_sum.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def affine_xor(a, b, c, d, lo, hi):
    """out[i - lo] and the int64 sum over [lo, hi) (Figure 1b pattern)."""
    out = np.empty(max(hi - lo, 0), np.int32)
    s = lib().oref_affine_xor(a, b, c, d, lo, hi, _ptr(out))
    return out, int(s)


def fma_chain(x, s_i32, s_f64, arr=None, i0=0):
    """y = fma chain of the shared scalars over x (Figure 5 pattern)."""
    x = np.ascontiguousarray(x, np.float32)
    si = np.ascontiguousarray(s_i32, np.int32)
    sf = np.ascontiguousarray(s_f64, np.float64)
    arr = np.ascontiguousarray(arr if arr is not None else np.zeros(0), np.int32)
    y = np.empty(x.size, np.float64)
    lib().oref_fma_chain(_ptr(x), x.size, _ptr(si), si.size, _ptr(sf), sf.size,
                         _ptr(arr), arr.size, i0, _ptr(y))
    return y


def gather(arrays, lo, hi):
    """out[i - lo] = sum_j arr_j[i mod len] + i (Figure 6 pattern)."""
    arrs = np.ascontiguousarray(np.concatenate(arrays), np.int32)
    out = np.empty(max(hi - lo, 0), np.int32)
    lib().oref_gather(_ptr(arrs), len(arrays), len(arrays[0]), lo, hi, _ptr(out))
    return out


def exact_sum(v):
    """Correctly rounded sum of a float64 array."""
    v = np.ascontiguousarray(v, np.float64)
    st = C.c_int32(0)
    r = lib().oref_exact_sum(_ptr(v), v.size, C.byref(st))
    if st.value:
        raise ValueError("non-finite input to exact_sum")
    return float(r)


def fixed75_sum(v):
    """Exact sum of values on the 2**-75 grid as a Python int (units of
    2**-75), or None when a value is off the grid."""
    v = np.ascontiguousarray(v, np.float64)
    lo, hi = C.c_uint64(0), C.c_int64(0)
    if lib().oref_fixed75_sum(_ptr(v), v.size, C.byref(lo), C.byref(hi)):
        return None
    return (hi.value << 64) | lo.value
