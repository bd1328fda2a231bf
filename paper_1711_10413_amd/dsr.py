"""ctypes binding of libdsr.so: the C ABI of include/dsr.h, same names.

Argument marshalling only -- every step of a region runs in the HIP
kernels.  Device buffers are passed as integer addresses (for instance a
PyTorch tensor's ``data_ptr()``) and streams as integer handles
(``torch.cuda.current_stream().cuda_stream``).  Importing this module
fails loudly if the library has not been built.
"""
import ctypes as C
import os
import struct

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdsr.so")

DSR_OK = 0
DSR_E_INVAL = -1
DSR_E_NOMEM = -2
DSR_E_LDS = -3
DSR_E_UNDERFLOW = -4
DSR_E_ORDER = -5
DSR_E_LIVE = -6
DSR_E_STATE = -7
DSR_E_BUSY = -8
DSR_E_HIP = -9
DSR_E_RANGE = -10
ERROR_NAMES = {DSR_E_INVAL: "INVAL", DSR_E_NOMEM: "NOMEM", DSR_E_LDS: "LDS",
               DSR_E_UNDERFLOW: "UNDERFLOW", DSR_E_ORDER: "ORDER", DSR_E_LIVE: "LIVE",
               DSR_E_STATE: "STATE", DSR_E_BUSY: "BUSY", DSR_E_HIP: "HIP",
               DSR_E_RANGE: "RANGE"}

DSR_BODY_TERMINATE = 0
DSR_BODY_AFFINE_XOR = 1
DSR_BODY_FMA_CHAIN = 2
DSR_BODY_GATHER = 3
DSR_BODY_GATHER_NESTED = 4
DSR_BODY_FMA_CHAIN_REFS = 5
DSR_LIST_ONCHIP = 20

DSR_SCHED_STATIC = 0
DSR_SCHED_DYNAMIC_TAIL = 1

DSR_F_TRACE = 1
DSR_F_TIMING = 2
DSR_F_GLOBAL_LISTS = 4
DSR_F_NESTED_GLOBAL = 8
DSR_TRACE_WORDS = 256
NEST_SPACES = {4: "nlds", 5: "nhbm"}

# the exported C entry points (include/dsr.h)
EXPORTS = ("dsr_init", "dsr_destroy", "dsr_region_begin", "dsr_push", "dsr_publish",
           "dsr_pop", "dsr_launch", "dsr_region_sync", "dsr_region_reduction",
           "dsr_region_trace", "dsr_region_elapsed", "dsr_region_free", "dsr_strerror",
           "dsr_batch_create", "dsr_batch_tune", "dsr_batch_get_tune", "dsr_batch_launch",
           "dsr_batch_launch_each", "dsr_batch_sync", "dsr_batch_result", "dsr_batch_times",
           "dsr_batch_elapsed", "dsr_batch_free", "dsr_autotune", "dsr_batch_replay_serial",
           "dsr_serve_start", "dsr_serve_submit", "dsr_serve_poll", "dsr_serve_pending",
           "dsr_serve_replay", "dsr_serve_stop", "dsr_occupancy_model", "dsr_region_occupancy",
           "dsr_publish_list", "dsr_control_bytes", "dsr_serve_status", "dsr_launch_static",
           "dsr_static_bytes", "dsr_stream_ceiling", "dsr_autotune_plan",
           "dsr_serve_class_for", "dsr_region_freeze")


class dsr_ref(C.Structure):
    _fields_ = [("frame", C.c_int32), ("offset", C.c_uint32)]


class dsr_config(C.Structure):
    _fields_ = [("wg_size", C.c_uint32), ("lds_slab_bytes", C.c_uint32),
                ("overflow_threshold", C.c_uint32), ("master_joins", C.c_uint32),
                ("hbm_slab_bytes", C.c_uint64), ("max_teams", C.c_uint32),
                ("flags", C.c_uint32)]


class dsr_loop(C.Structure):
    _fields_ = [("n", C.c_uint64), ("chunk", C.c_uint64), ("in_", C.c_void_p),
                ("out", C.c_void_p), ("ni", C.c_uint32), ("nf", C.c_uint32),
                ("alen", C.c_uint32), ("arrays", C.c_uint32), ("len", C.c_uint32),
                ("schedule", C.c_uint32), ("tail_pct", C.c_uint32), ("block", C.c_uint32),
                ("depth", C.c_uint32), ("deref", C.c_uint32)]


class dsr_tune(C.Structure):
    _fields_ = [("wg_size", C.c_uint32), ("lds_slab_bytes", C.c_uint32),
                ("overflow_threshold", C.c_uint32), ("master_joins", C.c_uint32),
                ("grid", C.c_uint32), ("use_graph", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dsr_serve_cfg(C.Structure):
    _fields_ = [("tune", dsr_tune), ("slots", C.c_uint32), ("slot_bytes", C.c_uint32),
                ("max_teams", C.c_uint32), ("ring_items", C.c_uint32), ("idle_ms", C.c_uint32),
                ("budget_pct", C.c_uint32), ("n_classes", C.c_uint32), ("class_slab", C.c_uint32 * 4),
                ("class_grid", C.c_uint32 * 4)]


class dsr_done(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("n_red", C.c_int32),
                ("f64", C.c_double * 8), ("i64", C.c_int64 * 8), ("fixed", (C.c_uint64 * 3) * 8),
                ("device_us", C.c_double), ("lds_class", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        fx = []
        for i in range(self.n_red):
            w = self.fixed[i]
            fx.append(_fixed([w[0], w[1], w[2]]))
        return {"ticket": self.ticket, "status": self.status, "f64": list(self.f64[:self.n_red]),
                "i64": list(self.i64[:self.n_red]), "fixed": fx, "device_us": self.device_us,
                "lds_class": self.lds_class}


class dsr_result_rec(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_red", C.c_int32), ("f64", C.c_double * 8),
                ("i64", C.c_int64 * 8), ("fixed", (C.c_uint64 * 3) * 8)]

    def as_dict(self):
        fx = [_fixed([w[0], w[1], w[2]]) for w in list(self.fixed)[:self.n_red]]
        return {"status": self.status, "f64": list(self.f64[:self.n_red]),
                "i64": list(self.i64[:self.n_red]), "fixed": fx}


DSR_STATIC_SCRATCH_BYTES = 16 << 20
RESULT_REC_BYTES = C.sizeof(dsr_result_rec)


class dsr_serve_stat(C.Structure):
    _fields_ = [("grid", C.c_uint32), ("started", C.c_uint32), ("exited", C.c_uint32),
                ("closed", C.c_uint32), ("final_items", C.c_uint32), ("published", C.c_uint32),
                ("in_flight", C.c_uint32), ("classes", C.c_uint32), ("close_reason", C.c_uint32),
                ("close_block", C.c_uint32), ("close_item", C.c_uint32), ("close_seen", C.c_uint32),
                ("close_idle_us", C.c_double), ("relays", C.c_uint32), ("relay_misses", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dsr_hw_model(C.Structure):
    _fields_ = [("compute_units", C.c_uint32), ("regs_per_cu", C.c_uint32),
                ("reg_granule", C.c_uint32), ("max_teams_per_cu", C.c_uint32),
                ("max_threads_per_cu", C.c_uint32), ("shared_per_cu", C.c_uint32),
                ("shared_granule", C.c_uint32), ("simds_per_cu", C.c_uint32),
                ("wave_size", C.c_uint32)]


class dsr_occupancy_t(C.Structure):
    _fields_ = [("teams_per_cu", C.c_uint32), ("teams_by_registers", C.c_uint32),
                ("teams_by_shared", C.c_uint32), ("teams_by_threads", C.c_uint32),
                ("limiter", C.c_uint32), ("shared_per_team", C.c_uint32),
                ("shared_per_cu", C.c_uint64), ("regs_per_thread", C.c_uint32),
                ("hip_teams_per_cu", C.c_uint32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["limiter"] = ("teams", "registers", "shared", "threads")[self.limiter]
        return d


class DsrError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        self.name = ERROR_NAMES.get(code, str(code))
        super().__init__("%s: %s (%s)" % (where, strerror(code), self.name))


_lib = None


def lib():
    """The loaded library (raises if libdsr.so is missing)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own copy of the HIP runtime under the same soname
        # as ROCm's; load it first so that one runtime serves the process and
        # device pointers and streams from torch are valid here.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdsr.so is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, u32, i32 = C.c_void_p, C.c_uint32, C.c_int32
        sig = {
            "dsr_init": [C.POINTER(P), C.POINTER(dsr_config), C.c_int],
            "dsr_destroy": [P],
            "dsr_region_begin": [P, i32, C.POINTER(P)],
            "dsr_push": [P, u32, P, u32, u32, C.POINTER(i32)],
            "dsr_publish": [P, i32, i32, C.POINTER(dsr_loop)],
            "dsr_publish_list": [P, C.POINTER(dsr_ref), i32, i32, C.POINTER(dsr_loop)],
            "dsr_pop": [P, i32],
            "dsr_launch": [P, P],
            "dsr_launch_static": [P, P, P],
            "dsr_autotune_plan": [P, C.POINTER(dsr_tune), i32, C.POINTER(i32)],
            "dsr_serve_class_for": [C.POINTER(u32), i32, P],
            "dsr_stream_ceiling": [P, P, C.c_uint64, u32, u32, P],
            "dsr_region_sync": [P],
            "dsr_region_reduction": [P, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                     C.POINTER(C.c_uint64)],
            "dsr_region_trace": [P, i32, C.POINTER(u32), u32],
            "dsr_region_elapsed": [P, C.POINTER(C.c_float)],
            "dsr_region_free": [P],
            "dsr_region_freeze": [P],
            "dsr_batch_create": [P, C.POINTER(P), i32, C.POINTER(P)],
            "dsr_batch_tune": [P, C.POINTER(dsr_tune)],
            "dsr_batch_get_tune": [P, C.POINTER(dsr_tune)],
            "dsr_batch_launch": [P, P],
            "dsr_batch_launch_each": [P, P],
            "dsr_batch_sync": [P],
            "dsr_batch_result": [P, i32, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                 C.POINTER(C.c_uint64), C.POINTER(i32)],
            "dsr_batch_times": [P, C.POINTER(C.c_double), i32],
            "dsr_batch_elapsed": [P, C.POINTER(C.c_float)],
            "dsr_batch_free": [P],
            "dsr_autotune": [P, C.POINTER(dsr_tune), i32, i32, P, C.POINTER(dsr_tune),
                             C.POINTER(C.c_float)],
            "dsr_batch_replay_serial": [P, C.POINTER(i32), C.POINTER(C.c_double), i32,
                                        C.POINTER(C.c_double)],
            "dsr_serve_start": [P, C.POINTER(dsr_serve_cfg), C.POINTER(P)],
            "dsr_serve_submit": [P, P, C.POINTER(P), i32, C.POINTER(C.c_uint64)],
            "dsr_serve_poll": [P, C.POINTER(dsr_done), i32],
            "dsr_serve_pending": [P],
            "dsr_serve_replay": [P, C.POINTER(P), C.POINTER(i32), C.POINTER(C.c_double), i32,
                                 C.POINTER(P), i32, C.c_double, C.POINTER(C.c_double),
                                 C.POINTER(dsr_done)],
            "dsr_serve_stop": [P],
            "dsr_serve_status": [P, C.POINTER(dsr_serve_stat)],
            "dsr_occupancy_model": [C.POINTER(dsr_hw_model), u32, u32, u32,
                                    C.POINTER(dsr_occupancy_t)],
            "dsr_region_occupancy": [P, u32, C.POINTER(dsr_occupancy_t)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.dsr_strerror.argtypes = [C.c_int]
        L.dsr_strerror.restype = C.c_char_p
        L.dsr_control_bytes.argtypes = [u32]
        L.dsr_control_bytes.restype = u32
        L.dsr_static_bytes.argtypes = [P]
        L.dsr_static_bytes.restype = C.c_uint64
        _lib = L
    return _lib


def strerror(code):
    return lib().dsr_strerror(code).decode()


def _check(rc, where):
    if rc != DSR_OK:
        raise DsrError(rc, where)
    return rc


# ---- thin wrappers with the C names ---------------------------------------
def dsr_init(wg_size=256, lds_slab_bytes=65536, overflow_threshold=0, master_joins=0,
             hbm_slab_bytes=1 << 20, max_teams=4096, flags=0, device=0):
    cfg = dsr_config(wg_size, lds_slab_bytes, overflow_threshold, master_joins,
                     hbm_slab_bytes, max_teams, flags)
    ctx = C.c_void_p()
    _check(lib().dsr_init(C.byref(ctx), C.byref(cfg), device), "dsr_init")
    return ctx


def dsr_destroy(ctx):
    return _check(lib().dsr_destroy(ctx), "dsr_destroy")


def dsr_region_begin(ctx, teams):
    r = C.c_void_p()
    _check(lib().dsr_region_begin(ctx, teams, C.byref(r)), "dsr_region_begin")
    return r


def dsr_push(region, nbytes, init=b"", init_stride=0, init_bytes=None):
    """Push a frame of ``nbytes``.  Without ``init_stride`` the frame's first
    len(init) bytes come from ``init``; with it, ``init`` holds one image per
    team, ``init_stride`` bytes apart, of which ``init_bytes`` are copied."""
    init = bytes(init)
    buf = C.create_string_buffer(init, len(init)) if init else None
    if init_bytes is None:
        init_bytes = min(init_stride, nbytes) if init_stride else len(init)
    h = C.c_int32()
    _check(lib().dsr_push(region, nbytes, buf, init_bytes, init_stride, C.byref(h)), "dsr_push")
    return h.value


def dsr_publish(region, frame, body, n, inp=0, out=0, chunk=0, ni=0, nf=0, alen=0, arrays=0,
                length=0, schedule=0, tail_pct=0, block=0, depth=0):
    L = dsr_loop(n, chunk, inp or None, out or None, ni, nf, alen, arrays, length, schedule,
                 tail_pct, block, depth)
    return _check(lib().dsr_publish(region, frame, body, C.byref(L)), "dsr_publish")


def dsr_publish_list(region, refs, body, n, inp=0, out=0, chunk=0, ni=0, nf=0, alen=0,
                     schedule=0, tail_pct=0, block=0, deref=0):
    """refs: (frame, byte offset) per variable: the exact sum slot, the ni
    int32 scalars, the nf fp64 scalars, then the array if alen > 0.
    deref=1: the loop reads every scalar through its reference on each batch."""
    arr = (dsr_ref * max(1, len(refs)))(*[dsr_ref(int(f), int(o)) for f, o in refs])
    L = dsr_loop(n, chunk, inp or None, out or None, ni, nf, alen, 0, 0, schedule, tail_pct, block, 0, deref)
    return _check(lib().dsr_publish_list(region, arr, len(refs), body, C.byref(L)), "dsr_publish_list")


def dsr_control_bytes(wg_size):
    return lib().dsr_control_bytes(wg_size)


def dsr_pop(region, frame):
    return _check(lib().dsr_pop(region, frame), "dsr_pop")


def dsr_launch(region, stream=0):
    return _check(lib().dsr_launch(region, stream or None), "dsr_launch")


def dsr_launch_static(region, result_ptr, stream=0):
    """Launch without allocating: every device buffer in the library's fixed
    workspace; the result record (RESULT_REC_BYTES) goes to the device
    address `result_ptr`."""
    return _check(lib().dsr_launch_static(region, result_ptr, stream or None), "dsr_launch_static")


def dsr_stream_ceiling(x_ptr, y_ptr, n, grid, wg_size=256, stream=0):
    """The streaming ceiling kernel: y = double(x) over n elements."""
    return _check(lib().dsr_stream_ceiling(x_ptr or None, y_ptr or None, n, grid, wg_size, stream or None),
                  "dsr_stream_ceiling")


def dsr_static_bytes(region):
    return int(lib().dsr_static_bytes(region))


def result_rec(raw):
    """Decode a dsr_result_rec from its bytes (e.g. a copied-back tensor)."""
    rec = dsr_result_rec.from_buffer_copy(bytes(raw))
    return rec.as_dict()


def dsr_region_sync(region):
    """Device status of the last launch (0 or a negative DSR_E_* code)."""
    rc = lib().dsr_region_sync(region)
    if rc in (DSR_E_INVAL, DSR_E_STATE, DSR_E_HIP):
        raise DsrError(rc, "dsr_region_sync")
    return rc


def dsr_region_reduction(region, index):
    """(int64 sum, float sum, exact total as a Python int in 2**-75 units)."""
    i = C.c_int64()
    f = C.c_double()
    w = (C.c_uint64 * 3)()
    _check(lib().dsr_region_reduction(region, index, C.byref(i), C.byref(f), w),
           "dsr_region_reduction")
    v = w[0] | (w[1] << 64) | (w[2] << 128)
    if v >> 191:
        v -= 1 << 192
    return i.value, f.value, v


def dsr_region_trace(region, team):
    buf = (C.c_uint32 * DSR_TRACE_WORDS)()
    _check(lib().dsr_region_trace(region, team, buf, DSR_TRACE_WORDS), "dsr_region_trace")
    t = list(buf)
    k = t[0]
    return {"placements": [(("lds", "hbm")[t[1 + 3 * p]], t[2 + 3 * p], t[3 + 3 * p])
                           for p in range(min(k, 16))],
            "barriers": t[49:65], "inner_pushes": t[65:81],
            "error": C.c_int32(t[81]).value,
            "t_start": t[82] | (t[83] << 32), "t_end": t[84] | (t[85] << 32),
            "t_team": t[86], "t_program_end": t[87], "t_arrived": t[88],
            "t_partials_stored": t[92], "t_arrival_returned": t[93],
            "t_combine_start": t[94], "t_combine_end": t[95],
            "list": (("lds", "hbm", "none", "onchip")[t[89]], t[90], t[91]) if t[91] else None,
            "wave_loop": [(t[96 + 2 * w], t[97 + 2 * w]) for w in range(16)],
            "nested": [{"frame": _nest_place(t[128 + 8 * m]),
                        "groups": [_nest_place(t[129 + 8 * m + g]) for g in range(4)],
                        "pop_error": t[133 + 8 * m], "pushes": t[134 + 8 * m]} for m in range(16)]}


def _nest_place(w):
    """A nested frame's placement word: (space, offset) or None."""
    return (NEST_SPACES[w >> 24], w & 0xFFFFFF) if (w >> 24) in NEST_SPACES else None


def dsr_region_elapsed(region):
    ms = C.c_float()
    _check(lib().dsr_region_elapsed(region, C.byref(ms)), "dsr_region_elapsed")
    return ms.value


def dsr_region_free(region):
    return _check(lib().dsr_region_free(region), "dsr_region_free")


def dsr_region_freeze(region):
    """Upload the region's program and images without launching it."""
    return _check(lib().dsr_region_freeze(region), "dsr_region_freeze")


# ---- batched form -----------------------------------------------------------
def _fixed(w):
    v = w[0] | (w[1] << 64) | (w[2] << 128)
    return v - (1 << 192) if v >> 191 else v


def dsr_batch_create(ctx, regions):
    arr = (C.c_void_p * len(regions))(*[r.value if isinstance(r, C.c_void_p) else r for r in regions])
    b = C.c_void_p()
    _check(lib().dsr_batch_create(ctx, arr, len(regions), C.byref(b)), "dsr_batch_create")
    return b


def dsr_batch_tune(batch, wg_size=256, lds_slab_bytes=65536, overflow_threshold=0,
                   master_joins=0, grid=0, use_graph=0):
    t = dsr_tune(wg_size, lds_slab_bytes, overflow_threshold, master_joins, grid, use_graph)
    return _check(lib().dsr_batch_tune(batch, C.byref(t)), "dsr_batch_tune")


def dsr_batch_get_tune(batch):
    t = dsr_tune()
    _check(lib().dsr_batch_get_tune(batch, C.byref(t)), "dsr_batch_get_tune")
    return t.as_dict()


def dsr_batch_launch(batch, stream=0):
    return _check(lib().dsr_batch_launch(batch, stream or None), "dsr_batch_launch")


def dsr_batch_launch_each(batch, stream=0):
    return _check(lib().dsr_batch_launch_each(batch, stream or None), "dsr_batch_launch_each")


def dsr_batch_sync(batch):
    rc = lib().dsr_batch_sync(batch)
    if rc in (DSR_E_INVAL, DSR_E_STATE, DSR_E_HIP):
        raise DsrError(rc, "dsr_batch_sync")
    return rc


def dsr_batch_result(batch, r, index=0):
    """(int64 sum, float sum, exact total in 2**-75 units, status) of region r."""
    i = C.c_int64()
    f = C.c_double()
    w = (C.c_uint64 * 3)()
    st = C.c_int32()
    _check(lib().dsr_batch_result(batch, r, index, C.byref(i), C.byref(f), w, C.byref(st)),
           "dsr_batch_result")
    return i.value, f.value, _fixed(w), st.value


def dsr_batch_times(batch, n):
    us = (C.c_double * n)()
    _check(lib().dsr_batch_times(batch, us, n), "dsr_batch_times")
    return np.frombuffer(us, dtype=np.float64).copy()


def dsr_batch_elapsed(batch):
    ms = C.c_float()
    _check(lib().dsr_batch_elapsed(batch, C.byref(ms)), "dsr_batch_elapsed")
    return ms.value


def dsr_batch_free(batch):
    return _check(lib().dsr_batch_free(batch), "dsr_batch_free")


def dsr_autotune_plan(batch, max_n=64):
    """Model-seeded autotuner candidates (list of dicts)."""
    buf = (dsr_tune * max_n)()
    n = C.c_int32()
    _check(lib().dsr_autotune_plan(batch, buf, max_n, C.byref(n)), "dsr_autotune_plan")
    return [buf[k].as_dict() for k in range(min(n.value, max_n))]


def dsr_autotune(batch, candidates, reps=3, stream=0):
    """candidates: list of dicts of dsr_tune fields.  Returns (best dict,
    list of mean ms per candidate, negative when skipped)."""
    n = len(candidates)
    arr = (dsr_tune * n)(*[dsr_tune(**{k: c.get(k, 0) for k, _ in dsr_tune._fields_})
                           for c in candidates])
    best = dsr_tune()
    ms = (C.c_float * n)()
    _check(lib().dsr_autotune(batch, arr, n, reps, stream or None, C.byref(best), ms),
           "dsr_autotune")
    return best.as_dict(), list(ms)


def dsr_batch_replay_serial(batch, prog, arrival_s):
    """One launch + synchronisation per request; returns latencies (us)."""
    n = len(prog)
    p = np.ascontiguousarray(prog, np.int32)
    a = np.ascontiguousarray(arrival_s, np.float64)
    lat = np.zeros(n, np.float64)
    _check(lib().dsr_batch_replay_serial(batch, p.ctypes.data_as(C.POINTER(C.c_int32)),
                                         a.ctypes.data_as(C.POINTER(C.c_double)), n,
                                         lat.ctypes.data_as(C.POINTER(C.c_double))),
           "dsr_batch_replay_serial")
    return lat


# ---- served form ------------------------------------------------------------
def dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=65536, overflow_threshold=0, master_joins=0,
                    grid=0, slots=256, slot_bytes=40960, max_teams=64, ring_items=1 << 16,
                    idle_ms=10000, budget_pct=0, classes=None):
    """classes: list of (LDS slab bytes, grid or 0) per LDS class, or None."""
    cls = list(classes or [])
    slabs = (C.c_uint32 * 4)(*[c[0] for c in cls])
    grids = (C.c_uint32 * 4)(*[c[1] for c in cls])
    cfg = dsr_serve_cfg(dsr_tune(wg_size, lds_slab_bytes, overflow_threshold, master_joins, grid, 0),
                        slots, slot_bytes, max_teams, ring_items, idle_ms, budget_pct, len(cls), slabs, grids)
    srv = C.c_void_p()
    _check(lib().dsr_serve_start(ctx, C.byref(cfg), C.byref(srv)), "dsr_serve_start")
    return srv


def dsr_serve_class_for(slabs, region):
    """Index of the LDS class (of on-chip stack sizes `slabs`) the request
    with this program is admitted to."""
    arr = (C.c_uint32 * len(slabs))(*slabs)
    rc = lib().dsr_serve_class_for(arr, len(slabs), region)
    if rc < 0:
        raise DsrError(rc, "dsr_serve_class_for")
    return rc


def dsr_serve_submit(server, region, outs=None):
    """Returns the ticket, or raises DsrError (BUSY: retry after polling)."""
    tk = C.c_uint64()
    if outs:
        arr = (C.c_void_p * len(outs))(*outs)
        rc = lib().dsr_serve_submit(server, region, arr, len(outs), C.byref(tk))
    else:
        rc = lib().dsr_serve_submit(server, region, None, 0, C.byref(tk))
    _check(rc, "dsr_serve_submit")
    return tk.value


def dsr_serve_poll(server, max_n=256):
    buf = (dsr_done * max_n)()
    n = lib().dsr_serve_poll(server, buf, max_n)
    if n < 0:
        raise DsrError(n, "dsr_serve_poll")
    return [buf[i].as_dict() for i in range(n)]


def dsr_serve_pending(server):
    return lib().dsr_serve_pending(server)


def dsr_serve_replay(server, programs, prog, arrival_s, slot_outs=None, n_loops_max=1,
                     timeout_s=60.0):
    """Replay an arrival schedule; returns (latency_us array, list of done dicts)."""
    n = len(prog)
    progs = (C.c_void_p * len(programs))(*[r.value if isinstance(r, C.c_void_p) else r
                                           for r in programs])
    p = np.ascontiguousarray(prog, np.int32)
    a = np.ascontiguousarray(arrival_s, np.float64)
    lat = np.zeros(n, np.float64)
    done = (dsr_done * max(n, 1))()
    outs = (C.c_void_p * len(slot_outs))(*slot_outs) if slot_outs else None
    _check(lib().dsr_serve_replay(server, progs, p.ctypes.data_as(C.POINTER(C.c_int32)),
                                  a.ctypes.data_as(C.POINTER(C.c_double)), n, outs, n_loops_max,
                                  timeout_s, lat.ctypes.data_as(C.POINTER(C.c_double)), done),
           "dsr_serve_replay")
    return lat, [done[i].as_dict() for i in range(n)]


def dsr_serve_stop(server):
    return _check(lib().dsr_serve_stop(server), "dsr_serve_stop")


def dsr_serve_status(server):
    st = dsr_serve_stat()
    _check(lib().dsr_serve_status(server, C.byref(st)), "dsr_serve_status")
    return st.as_dict()


# ---- footprint and occupancy model --------------------------------------------
def dsr_occupancy(hw, threads_per_team, regs_per_thread, shared_per_team):
    o = dsr_occupancy_t()
    _check(lib().dsr_occupancy_model(C.byref(hw), threads_per_team, regs_per_thread,
                                     shared_per_team, C.byref(o)), "dsr_occupancy_model")
    return o.as_dict()


def dsr_region_occupancy(ctx, variant=0):
    o = dsr_occupancy_t()
    _check(lib().dsr_region_occupancy(ctx, variant, C.byref(o)), "dsr_region_occupancy")
    return o.as_dict()


# ---- frame images for the bodies' layouts (include/dsr.h) -----------------
def affine_xor_frame(a, b, c, d):
    """[0,8) int64 sum = 0; int32 a, b, c, d."""
    return struct.pack("<qiiii", 0, a, b, c, d)


def fma_chain_frame(s_i32, s_f64, arr=None):
    """[0,24) exact sum = 0; fp64 scalars; int32 scalars; array at the next
    16-byte boundary.  Returns (bytes, declared size)."""
    s_i32 = np.asarray(s_i32, np.int32)
    s_f64 = np.asarray(s_f64, np.float64)
    head = bytes(24) + s_f64.tobytes() + s_i32.tobytes()
    if arr is not None and len(arr):
        pad = (-len(head)) % 16
        head = head + bytes(pad) + np.asarray(arr, np.int32).tobytes()
    return head, len(head)


def gather_frame(arrays):
    return b"".join(np.asarray(a, np.int32).tobytes() for a in arrays)


def fma_chain_region(ctx, teams, s_i32, s_f64, arr, n, x_ptr, y_ptr, schedule=0):
    """A region whose masters share s_i32, s_f64 (and arr) in one frame and
    publish the fma-chain loop over x[0..n) -> y (convenience builder)."""
    img, size = fma_chain_frame(s_i32, s_f64, arr)
    r = dsr_region_begin(ctx, teams)
    f = dsr_push(r, size, img)
    dsr_publish(r, f, DSR_BODY_FMA_CHAIN, n, inp=x_ptr, out=y_ptr, ni=len(s_i32), nf=len(s_f64),
                alen=0 if arr is None else len(arr), schedule=schedule)
    dsr_pop(r, f)
    return r
