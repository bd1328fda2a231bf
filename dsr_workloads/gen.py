"""Counter-based random numbers (splitmix64) and their mappings to values.

splitmix64 is the generator of Steele, Lea and Flood ("Fast splittable
pseudorandom number generators", OOPSLA 2014) in the form popularised by
Vigna: the state advances by the golden-ratio increment GAMMA and each
output is the state passed through the mix64 finaliser.  Draw ``n`` of a
stream is the ``n``-th output (0-based) of a splitmix64 whose state starts at
``stream_base(seed, stream)``, so any draw can be computed directly from its
index.  All arithmetic is on numpy uint64 (wrapping mod 2**64).
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
STREAM_MUL = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def mix64(z):
    """splitmix64 finaliser on a numpy uint64 array (or scalar)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_base(seed, stream):
    """Starting state of stream ``stream`` under ``seed``."""
    with np.errstate(over="ignore"):
        v = np.uint64(seed & _MASK64) ^ (np.uint64(stream & _MASK64) * STREAM_MUL)
    return mix64(v)


def draws(seed, stream, start, count):
    """Raw uint64 draws ``start .. start+count-1`` of one stream."""
    base = stream_base(seed, stream)
    n = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(base + n * GAMMA)


def splitmix64_sequence(state, count):
    """The first ``count`` outputs of a sequential splitmix64 started at
    ``state`` (plain Python integers; used to cross-check ``draws``)."""
    out = []
    s = state & _MASK64
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & _MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out.append(z ^ (z >> 31))
    return out


def uniform_int(u, lo, hi):
    """Integers uniform on [lo, hi] (inclusive) from raw draws: the top 32
    bits scaled by the range width (Lemire's multiply-shift map)."""
    width = np.uint64(hi - lo + 1)
    top = np.asarray(u, dtype=np.uint64) >> np.uint64(32)
    with np.errstate(over="ignore"):
        r = (top * width) >> np.uint64(32)
    return (r.astype(np.int64) + lo)


def uniform_f32(u):
    """fp32 uniform on [-1, 1): 24 random bits on the 2**-23 grid (exact)."""
    top = (np.asarray(u, dtype=np.uint64) >> np.uint64(40)).astype(np.float64)
    return (top * 2.0 ** -23 - 1.0).astype(np.float32)


def uniform_f64(u):
    """fp64 uniform on [-1, 1): 53 random bits on the 2**-52 grid (exact)."""
    top = (np.asarray(u, dtype=np.uint64) >> np.uint64(11)).astype(np.float64)
    return top * 2.0 ** -52 - 1.0


def log_uniform_int(u, a, b):
    """Integers log-uniform on [a, b]: floor(a * (b/a)**v), v uniform on
    [0, 1).  Host-side only; callers hand the resulting table to both the
    oracle and the GPU path."""
    v = (np.asarray(u, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.floor(a * np.power(b / a, v)).astype(np.int64)
    return np.clip(r, a, b)


_fast = None


def _fastlib():
    global _fast
    if _fast is None:
        import ctypes
        from .build import build
        L = ctypes.CDLL(build())
        L.dsrgen_f32.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int]
        L.dsrgen_f32.restype = None
        _fast = L
    return _fast


def uniform_f32_draws(seed, stream, start, count, threads=None):
    """uniform_f32(draws(seed, stream, start, count)) computed by the C fast
    path (same definition, multithreaded); bit-identical to the numpy path."""
    import os
    out = np.empty(count, np.float32)
    if count:
        th = threads or min(16, os.cpu_count() or 1)
        _fastlib().dsrgen_f32(seed & _MASK64, stream & _MASK64, start, count,
                              out.ctypes.data, th)
    return out
