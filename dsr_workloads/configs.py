"""Input recipes for the five workloads of the data-sharing runtime.

Each recipe returns plain numpy arrays or small dataclasses: the master's
shared locals (scalars, arrays), the loop input x, loop lengths and frame
compositions.  Stream numbering: 0 = int32 scalars, 1 = fp64 scalars,
2 = x, 3 = loop lengths, 4 = frame sizes, 5 = arrival gaps, 16+j = array j;
per instance r of the batched and served workloads the field f lives on
stream (r+1)*256 + f.
"""
from dataclasses import dataclass
import numpy as np

from .gen import (draws, uniform_int, uniform_f32, uniform_f64,
                  log_uniform_int, uniform_f32_draws)

CFG2_KS = (1, 2, 4, 8, 16, 32, 64)
CFG3_AS = (1, 2, 3, 4)
CFG3_LENS = (16, 256, 4096, 16384)

I32_LO, I32_HI = -(1 << 20), (1 << 20)


@dataclass
class Cfg1:
    """Plain region: 4 shared int32 scalars a, b, c, d, loop over n."""
    a: int
    b: int
    c: int
    d: int
    n: int = 1024
    teams: int = 4
    wg: int = 256


def cfg1_inputs(seed=0, team=0):
    """a, b, c, d uniform on [-1000, 1000]: draws 4*team .. 4*team+3 of
    stream 0 (team 0 gives the default workload)."""
    v = uniform_int(draws(seed, 0, 4 * team, 4), -1000, 1000)
    return Cfg1(int(v[0]), int(v[1]), int(v[2]), int(v[3]))


@dataclass
class Cfg2:
    """Scalar sweep: K shared scalars (ceil(K/2) int32, floor(K/2) fp64)."""
    K: int
    s_i32: np.ndarray   # int32 [ceil(K/2)], applied first
    s_f64: np.ndarray   # float64 [floor(K/2)], applied after the int32 ones
    n: int
    teams: int = 512
    wg: int = 256


def cfg2_inputs(K, seed=1, n=1 << 24, with_x=True):
    """Scalars from streams 0 (int32 on [-2**20, 2**20]) and 1 (fp64 on
    [-1, 1)); prefix-stable, so a larger K extends a smaller one.  Returns
    (Cfg2, x) with x fp32[n] uniform on [-1, 1) from stream 2."""
    ni, nf = (K + 1) // 2, K // 2
    s_i = uniform_int(draws(seed, 0, 0, ni), I32_LO, I32_HI).astype(np.int32)
    s_f = uniform_f64(draws(seed, 1, 0, nf)) if nf else np.zeros(0, np.float64)
    x = uniform_f32_draws(seed, 2, 0, n) if with_x else None
    return Cfg2(K, s_i, s_f, n), x


def cfg2_x_chunk(seed, start, count):
    """A slice of the cfg2 loop input x (for bounded samples)."""
    return uniform_f32_draws(seed, 2, start, count)


@dataclass
class Cfg3:
    A: int
    length: int
    n: int = 1 << 26
    teams: int = 2048
    wg: int = 256


def cfg3_arrays(A, length, seed=2):
    """A shared int32 arrays of ``length`` elements, uniform on
    [0, 2**16): array j from stream 16+j."""
    return [uniform_int(draws(seed, 16 + j, 0, length), 0, (1 << 16) - 1)
            .astype(np.int32) for j in range(A)]


def frame_composition(F):
    """Split a frame payload of F bytes (multiple of 8, 8 <= F <= 32768)
    into shared locals: n_s = min(F/8, 32) scalar units made of
    floor(n_s/2) fp64 and 2*ceil(n_s/2) int32 scalars (8*n_s bytes), and
    the remaining bytes as one int32 array (possibly empty).
    Returns (n_i32, n_f64, arr_len)."""
    ns = max(1, min(F // 8, 32))
    nf = ns // 2
    ni = 2 * ((ns + 1) // 2)
    rest = F - 8 * ns
    return ni, nf, rest // 4


@dataclass
class Cfg4Instance:
    r: int
    L: int          # loop length (fp32 elements of x)
    F: int          # declared payload bytes
    s_i32: np.ndarray
    s_f64: np.ndarray
    arr: np.ndarray  # int32, may be empty


def cfg4_descriptors(n_inst=10000, seed=3):
    """Per-instance loop lengths L (log-uniform on [256, 2**20]) and frame
    payloads F (log-uniform on [8, 32768] bytes, rounded up to 8)."""
    L = log_uniform_int(draws(seed, 3, 0, n_inst), 256, 1 << 20)
    Fr = log_uniform_int(draws(seed, 4, 0, n_inst), 8, 32768)
    F = np.minimum(((Fr + 7) // 8) * 8, 32768)
    return L.astype(np.int64), F.astype(np.int64)


def _inst_stream(r, field):
    return (r + 1) * 256 + field


def cfg4_instance(r, L, F, seed=3):
    """Shared locals of instance r (its x is drawn by ``instance_x``)."""
    ni, nf, alen = frame_composition(int(F))
    s_i = uniform_int(draws(seed, _inst_stream(r, 0), 0, ni), I32_LO, I32_HI).astype(np.int32)
    s_f = uniform_f64(draws(seed, _inst_stream(r, 1), 0, nf)) if nf else np.zeros(0)
    arr = (uniform_int(draws(seed, _inst_stream(r, 16), 0, alen), 0, (1 << 16) - 1)
           .astype(np.int32) if alen else np.zeros(0, np.int32))
    return Cfg4Instance(int(r), int(L), int(F), s_i, s_f, arr)


def instance_x(r, L, seed=3, start=0, count=None):
    """fp32 loop input of instance r, uniform on [-1, 1)."""
    count = L - start if count is None else count
    return uniform_f32_draws(seed, _inst_stream(r, 2), start, count)


def poisson_schedule(rate, duration_s, seed=4):
    """Arrival times (seconds) of an open-loop Poisson process: gaps
    -ln(1-v)/rate from stream 5, until ``duration_s``."""
    n_guess = int(rate * duration_s * 1.2 + 64)
    u = draws(seed, 5, 0, n_guess)
    v = (u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    t = np.cumsum(-np.log1p(-v) / rate)
    return t[t < duration_s]
