"""Contention-group simulator of implicit data sharing -- TEST INFRASTRUCTURE.

A plain, slow model of one OpenMP target region in generic mode:

* Each team is a contention group: one master and W workers (section 4,
  Figures 2 and 3).  The master alone runs the sequential code; workers wait
  until the master hands them an outlined body, run it, and join.
* The master's implicitly shared locals live in frames on a per-team stack
  (section 5.3.1, shared depot).  A frame goes to the on-chip stack when it
  fits (capacity ``lds_bytes``, frames no larger than ``threshold``) and
  otherwise to a per-team global-memory area (capacity ``hbm_bytes``): the
  global fallback of section 5.2 and the runtime-managed global stack of
  section 7.  A frame that fits neither is an out-of-memory error.
* Sharing is by reference (section 5.1): workers read shared locals through
  (space, offset) into the simulated bytes every time they use them.
* Reductions go into a shared variable held in the frame: each worker keeps
  a private partial, stores it in its own control slot, and after the join
  the master adds the partials, in worker order, into the frame's slot.
* Frames are popped in LIFO order and none may outlive the region.

Every step checks the invariants
  I1 each worker's view of a published frame equals the master's bytes at
     publish time,
  I2 frames pop in LIFO order,
  I3 no frame outlives its region (nor an inner frame its outer body),
  I4 stack bytes in use equal the sum of the live frames' rounded sizes,
  I5 stack pointers stay within capacity; out-of-memory happens exactly
     when a frame fits neither space,
and a race detector that records, per byte, the last writer and the phase
(barrier epoch) of the write, and flags a cross-thread access to a byte
written in the same phase, any access outside a live frame and any access
after a pop.

Loop bodies (their frame layouts are the bodies' contracts):
  affine_xor   [0,8) int64 sum slot; a, b, c, d int32 at 8, 12, 16, 20.
               out[i] = a*i + b - (c ^ i) + d (int32 wrap); sum += out[i].
  fma_chain    [0,24) exact sum slot: signed 192-bit integer, units of
               2**-75, little-endian 64-bit words; nf fp64 scalars at 24;
               ni int32 scalars after them; optional int32 array of alen
               elements at the next 16-byte boundary.
               y[i] = fma chain (int32 scalars first, then fp64) over x[i]
               starting from arr[i mod alen] (or +0.0); sum += y[i] exactly.
  gather       A int32 arrays of ``length`` elements back to back at 0.
               out[i] = sum_j arr_j[i mod length] + i.
  gather_nested  as gather, but each outer member pushes a 16-byte inner
               frame {lo, hi, stride, outer frame id} on its own sub-stack
               and hands it to its inner members (a second, nested parallel
               level), then pops it.
  fma_chain_refs the fma_chain loop published through a list of references
               (section 5.2): reference 0 is the 24-byte exact sum slot,
               then ni int32 scalars, nf fp64 scalars and, if alen > 0, the
               int32 array, each anywhere in a live frame.  Lists of up to
               20 references go to the team's on-chip list (160 bytes);
               longer ones to a list frame on the global-memory stack,
               pushed at the fork and popped at the join.  Workers read a
               reference, then the variable through it, on every use.

Sizes are rounded up to ``align`` (16) bytes; frame offsets are multiples
of it.  Fractions give correctly rounded fma (one rounding of the exact
a*b+c) independently of the C oracle.
"""
from dataclasses import dataclass, field
from fractions import Fraction
import hashlib
import random
import struct

import numpy as np

LDS, HBM, CTL = "lds", "hbm", "ctl"
REF_LIST_ENTRIES = 20             # references the on-chip list holds
REF_BYTES = 8                     # a reference: space (u32), offset (u32)
SLOT_F64_EXACT = 24
UNIT_EXP = 75                     # exact sums are integers in units of 2**-75
WINDOW_EXP = 32                   # |y| must be below 2**32
INT192 = 1 << 192


class SimError(Exception):
    """A runtime error; ``code`` is one of NOMEM, ORDER, UNDERFLOW, LIVE,
    STATE, INVAL, RANGE."""

    def __init__(self, code, msg=""):
        super().__init__("%s: %s" % (code, msg))
        self.code = code


class Violation(AssertionError):
    """An invariant or race-detector failure (a bug in the model or in the
    program under test, never an expected runtime error)."""


@dataclass
class Config:
    lds_bytes: int = 65536        # on-chip stack capacity per team
    hbm_bytes: int = 1 << 20      # global-memory stack capacity per team
    threshold: int = 1 << 30      # largest frame placed on chip
    workers: int = 3              # worker threads per team
    sub_bytes: int = 64           # per outer member sub-stack (nested level)
    inner: int = 4                # inner members per outer member
    align: int = 16
    schedule: str = "cyclic"      # iteration -> worker: block cyclic reverse random
    interleave: str = "canonical" # step order: canonical roundrobin random
    seed: int = 0


# ---- program ops ---------------------------------------------------------
@dataclass
class Push:
    nbytes: int
    init: object = b""            # bytes, or callable(team) -> bytes


@dataclass
class Publish:
    frame: int                    # index of the Push that made the frame
    body: str
    loop: dict = field(default_factory=dict)


@dataclass
class PublishList:
    refs: list                    # (push index, byte offset) per shared variable
    body: str
    loop: dict = field(default_factory=dict)


@dataclass
class Pop:
    frame: int


@dataclass
class FrameRec:
    fid: int
    space: str
    off: int
    size: int                     # rounded size
    nbytes: int                   # declared size
    owner: str                    # "team" or "outer<m>"


@dataclass
class TeamTrace:
    placements: list = field(default_factory=list)   # (space, off, size) per push
    sub_placements: list = field(default_factory=list)
    lists: list = field(default_factory=list)        # (space, off, entries) per list publish
    master_barriers: int = 0
    worker_barriers: list = field(default_factory=list)
    partials: list = field(default_factory=list)     # slot value after each join
    error: str = None


def round_up(n, a):
    return (n + a - 1) // a * a


def fma(a, b, c):
    """Correctly rounded fused multiply-add (one rounding of a*b + c)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def to_units(y):
    """y as an integer number of 2**-75 units, or None when y is off the
    2**-75 grid or |y| >= 2**32."""
    if y != y or y in (float("inf"), float("-inf")) or abs(y) >= 2.0 ** WINDOW_EXP:
        return None
    f = Fraction(y) * (1 << UNIT_EXP)
    return f.numerator if f.denominator == 1 else None


def units_to_float(u):
    """Correctly rounded double of u * 2**-75 (u a Python int)."""
    return float(Fraction(u, 1 << UNIT_EXP))


def int_to_le(v, nbytes):
    return (v % (1 << (8 * nbytes))).to_bytes(nbytes, "little")


def le_to_int(b):
    v = int.from_bytes(b, "little")
    return v - (1 << (8 * len(b))) if v >> (8 * len(b) - 1) else v


class Memory:
    """Byte store of one space with per-byte shadow (writer, phase, alive)."""

    def __init__(self, name, size):
        self.name = name
        self.data = bytearray(size)
        self.writer = [None] * size
        self.phase = [-1] * size


class Team:
    def __init__(self, tid, cfg, n_teams):
        self.tid = tid
        self.cfg = cfg
        self.n_teams = n_teams
        self.mem = {LDS: Memory(LDS, cfg.lds_bytes), HBM: Memory(HBM, cfg.hbm_bytes),
                    CTL: Memory(CTL, REF_LIST_ENTRIES * REF_BYTES)}
        self.sp = {LDS: 0, HBM: 0}
        self.frames = []           # live team-level frames, bottom .. top
        self.by_id = {}
        self.dead = set()
        self.phase = 0
        self.trace = TeamTrace(worker_barriers=[0] * cfg.workers)
        self.live_ranges = {LDS: [], HBM: []}   # (off, end) of live frames

    # -- invariants -------------------------------------------------------
    def check_stack(self):
        used = {LDS: 0, HBM: 0}
        for f in self.frames:
            used[f.space] += f.size
        for s in (LDS, HBM):
            if used[s] != self.sp[s]:
                raise Violation("I4: %s stack %d bytes, live frames %d" % (s, self.sp[s], used[s]))
        if self.sp[LDS] > self.cfg.lds_bytes or self.sp[HBM] > self.cfg.hbm_bytes:
            raise Violation("I5: stack pointer beyond capacity")

    # -- memory access through (space, offset) -----------------------------
    def _frame_covering(self, space, off, n):
        for f in self.frames:
            if f.space == space and f.off <= off and off + n <= f.off + f.size:
                return f
        return None

    def access(self, space, off, n, who, write, data=None, frames=None):
        pool = self.frames if frames is None else frames
        ok = any(f.space == space and f.off <= off and off + n <= f.off + f.size for f in pool)
        if not ok:
            raise Violation("race detector: %s access [%d,%d) of %s outside a live frame"
                            % (who, off, off + n, space))
        m = self.mem[space]
        for b in range(off, off + n):
            w, p = m.writer[b], m.phase[b]
            if w is not None and w != who and p == self.phase:
                raise Violation("race detector: %s %s byte %d of %s written by %s in phase %d"
                                % (who, "writes" if write else "reads", b, space, w, p))
        if write:
            m.data[off:off + n] = data
            for b in range(off, off + n):
                m.writer[b] = who
                m.phase[b] = self.phase
            return None
        return bytes(m.data[off:off + n])

    def read(self, f, off, n, who, frames=None):
        if f.fid in self.dead:
            raise Violation("race detector: %s reads frame %d after its pop" % (who, f.fid))
        if off < 0 or off + n > f.nbytes:
            raise Violation("race detector: %s reads [%d,%d) outside frame %d of %d bytes"
                            % (who, off, off + n, f.fid, f.nbytes))
        return self.access(f.space, f.off + off, n, who, False, frames=frames)

    def write(self, f, off, data, who, frames=None):
        if f.fid in self.dead:
            raise Violation("race detector: %s writes frame %d after its pop" % (who, f.fid))
        if off < 0 or off + len(data) > f.nbytes:
            raise Violation("race detector: %s writes outside frame %d" % (who, f.fid))
        self.access(f.space, f.off + off, len(data), who, True, data, frames=frames)

    def barrier(self, participants):
        self.phase += 1
        self.trace.master_barriers += 1
        for w in range(self.cfg.workers):
            self.trace.worker_barriers[w] += 1

    def frame_hash(self, f):
        return hashlib.sha256(bytes(self.mem[f.space].data[f.off:f.off + f.nbytes])).hexdigest()

    # -- stack operations (master only) -----------------------------------
    def push(self, fid, nbytes, global_only=False):
        if nbytes < 0:
            raise SimError("INVAL", "negative frame size")
        size = round_up(nbytes, self.cfg.align)
        c = self.cfg
        if not global_only and size <= c.threshold and self.sp[LDS] + size <= c.lds_bytes:
            space = LDS
        elif self.sp[HBM] + size <= c.hbm_bytes:
            space = HBM
        else:
            raise SimError("NOMEM", "frame of %d bytes fits neither stack" % size)
        f = FrameRec(fid, space, self.sp[space], size, nbytes, "team")
        self.sp[space] += size
        self.frames.append(f)
        self.by_id[fid] = f
        if not global_only:
            self.trace.placements.append((space, f.off, size))
        m = self.mem[space]
        for b in range(f.off, f.off + size):   # a new frame holds no one's data
            m.writer[b] = None
            m.phase[b] = -1
        self.check_stack()
        return f

    def pop(self, fid):
        if not self.frames:
            raise SimError("UNDERFLOW", "pop on an empty stack")
        f = self.by_id.get(fid)
        if f is None or f not in self.frames:
            raise SimError("STATE", "pop of a frame that is not live")
        if self.frames[-1] is not f:
            raise SimError("ORDER", "pop of frame %d, top is %d" % (fid, self.frames[-1].fid))
        self.frames.pop()
        self.sp[f.space] -= f.size
        self.dead.add(fid)
        self.check_stack()


# ---- iteration schedules -------------------------------------------------
def assign(items, n_workers, schedule, rng):
    """Split a list of iterations among workers."""
    items = list(items)
    if schedule == "block":
        per = -(-len(items) // n_workers) if items else 0
        return [items[w * per:(w + 1) * per] for w in range(n_workers)]
    if schedule == "cyclic":
        return [items[w::n_workers] for w in range(n_workers)]
    if schedule == "reverse":
        return [list(reversed(items[w::n_workers])) for w in reversed(range(n_workers))]
    if schedule == "random":
        out = [[] for _ in range(n_workers)]
        for it in items:
            out[rng.randrange(n_workers)].append(it)
        return out
    raise ValueError(schedule)


def interleave(queues, how, rng):
    """Yield (worker, iteration) in the chosen step order."""
    queues = [list(q) for q in queues]
    if how == "canonical":
        for w, q in enumerate(queues):
            for it in q:
                yield w, it
        return
    pos = [0] * len(queues)
    while True:
        live = [w for w in range(len(queues)) if pos[w] < len(queues[w])]
        if not live:
            return
        order = live if how == "roundrobin" else [rng.choice(live)]
        for w in order:
            yield w, queues[w][pos[w]]
            pos[w] += 1


def all_interleavings(queues):
    """Every interleaving of the workers' iteration sequences (tiny cases)."""
    n = [len(q) for q in queues]

    def rec(pos):
        if all(pos[w] == n[w] for w in range(len(n))):
            yield []
            return
        for w in range(len(n)):
            if pos[w] < n[w]:
                nxt = list(pos)
                nxt[w] += 1
                for rest in rec(nxt):
                    yield [(w, queues[w][pos[w]])] + rest
    yield from rec([0] * len(n))


# ---- loop bodies ---------------------------------------------------------
def team_range(loop, tid, n_teams):
    n = loop["n"]
    chunk = loop.get("chunk") or -(-n // n_teams)
    lo = min(n, tid * chunk)
    return lo, min(n, lo + chunk)


def _i32(b):
    return struct.unpack("<i", b)[0]


def _f64(b):
    return struct.unpack("<d", b)[0]


class Body:
    """One outlined parallel body: reads the frame through its references,
    writes its output element, returns its reduction contribution."""
    has_reduction = False
    slot_bytes = 0

    def iteration(self, team, f, who, i, loop):
        raise NotImplementedError


class AffineXor(Body):
    has_reduction = True
    slot_bytes = 8

    def iteration(self, team, f, who, i, loop):
        a = _i32(team.read(f, 8, 4, who))
        b = _i32(team.read(f, 12, 4, who))
        c = _i32(team.read(f, 16, 4, who))
        d = _i32(team.read(f, 20, 4, who))
        ui = i & 0xFFFFFFFF
        v = ((a & 0xFFFFFFFF) * ui + (b & 0xFFFFFFFF) - ((c & 0xFFFFFFFF) ^ ui)
             + (d & 0xFFFFFFFF)) & 0xFFFFFFFF
        o = v - (1 << 32) if v >> 31 else v
        loop["out"][i] = o
        return o


class FmaChain(Body):
    has_reduction = True
    slot_bytes = SLOT_F64_EXACT

    def iteration(self, team, f, who, i, loop):
        ni, nf, alen = loop["ni"], loop["nf"], loop.get("alen", 0)
        xi = float(loop["x"][i])
        acc = 0.0
        if alen:
            aoff = round_up(SLOT_F64_EXACT + 8 * nf + 4 * ni, 16)
            acc = float(_i32(team.read(f, aoff + 4 * (i % alen), 4, who)))
        for k in range(ni):
            acc = fma(float(_i32(team.read(f, SLOT_F64_EXACT + 8 * nf + 4 * k, 4, who))), xi, acc)
        for k in range(nf):
            acc = fma(_f64(team.read(f, SLOT_F64_EXACT + 8 * k, 8, who)), xi, acc)
        loop["y"][i] = acc
        u = to_units(acc)
        if u is None:
            raise SimError("RANGE", "y[%d] = %r is outside the exact-sum window" % (i, acc))
        return u


class Gather(Body):
    def iteration(self, team, f, who, i, loop, frames=None):
        A, length = loop["A"], loop["length"]
        s = i
        for j in range(A):
            s += _i32(team.read(f, 4 * (j * length + i % length), 4, who, frames=frames))
        loop["out"][i] = ((s + (1 << 31)) % (1 << 32)) - (1 << 31)
        return 0


class FmaChainRefs(Body):
    """fma_chain through references: every variable is reached by reading
    its reference from the list, then the variable (section 5.2)."""
    has_reduction = True
    slot_bytes = SLOT_F64_EXACT

    def iteration(self, team, lst, who, i, loop):
        ni, nf, alen = loop["ni"], loop["nf"], loop.get("alen", 0)
        xi = float(loop["x"][i])
        acc = 0.0
        if alen:
            sp, off = lst.ref(team, 1 + ni + nf, who)
            acc = float(_i32(team.access(sp, off + 4 * (i % alen), 4, who, False)))
        for k in range(ni):
            sp, off = lst.ref(team, 1 + k, who)
            acc = fma(float(_i32(team.access(sp, off, 4, who, False))), xi, acc)
        for k in range(nf):
            sp, off = lst.ref(team, 1 + ni + k, who)
            acc = fma(_f64(team.access(sp, off, 8, who, False)), xi, acc)
        loop["y"][i] = acc
        u = to_units(acc)
        if u is None:
            raise SimError("RANGE", "y[%d] = %r is outside the exact-sum window" % (i, acc))
        return u


BODIES = {"affine_xor": AffineXor(), "fma_chain": FmaChain(), "gather": Gather(),
          "gather_nested": Gather(), "fma_chain_refs": FmaChainRefs()}
SPACE_CODE = {LDS: 0, HBM: 1}
CODE_SPACE = {0: LDS, 1: HBM}


class RefList:
    """A published list of references: in the team's on-chip list area or
    in a list frame on the global-memory stack."""

    def __init__(self, frame):
        self.frame = frame

    def ref(self, team, k, who):
        b = team.access(self.frame.space, self.frame.off + REF_BYTES * k, REF_BYTES, who, False,
                        frames=[self.frame])
        code, off = struct.unpack("<II", b)
        if code not in CODE_SPACE:
            raise Violation("reference %d names no space" % k)
        return CODE_SPACE[code], off

    def view(self, team, n, sizes):
        """Bytes of the list and of every variable it references."""
        h = hashlib.sha256(bytes(team.mem[self.frame.space].data[self.frame.off:self.frame.off + REF_BYTES * n]))
        for k in range(n):
            code, off = struct.unpack_from("<II", team.mem[self.frame.space].data, self.frame.off + REF_BYTES * k)
            h.update(bytes(team.mem[CODE_SPACE[code]].data[off:off + sizes[k]]))
        return h.hexdigest()


# ---- the region ----------------------------------------------------------
def run_team(team, program, interleaving=None):
    """Run the master's program for one team; returns the team trace.  A
    runtime error stops the team's program and is recorded in the trace."""
    cfg = team.cfg
    rng = random.Random(cfg.seed * 1000003 + team.tid)
    pushed = []
    try:
        for op in program:
            if isinstance(op, Push):
                fid = len(pushed)
                f = team.push(fid, op.nbytes)
                pushed.append(f)
                init = op.init(team.tid) if callable(op.init) else op.init
                init = bytes(init)
                if len(init) > op.nbytes:
                    raise SimError("INVAL", "init bytes exceed the frame")
                if init:
                    team.write(f, 0, init, "master")
                if len(init) < op.nbytes:
                    team.write(f, len(init), bytes(op.nbytes - len(init)), "master")
            elif isinstance(op, Pop):
                if not team.frames:
                    raise SimError("UNDERFLOW", "pop on an empty stack")
                if op.frame >= len(pushed):
                    raise SimError("STATE", "pop of a frame never pushed")
                team.pop(op.frame)
            elif isinstance(op, Publish):
                if op.frame >= len(pushed) or pushed[op.frame] not in team.frames:
                    raise SimError("STATE", "publish of a frame that is not live")
                publish(team, pushed[op.frame], op, rng, interleaving)
            elif isinstance(op, PublishList):
                publish_list(team, pushed, op, rng, interleaving)
            else:
                raise SimError("INVAL", "unknown op %r" % (op,))
        if team.frames:
            raise SimError("LIVE", "%d frame(s) outlive the region" % len(team.frames))
    except SimError as e:
        team.trace.error = e.code
    # terminate: the master releases the workers one last time (Figure 3's
    # terminate branch), whether or not the program failed
    team.barrier("all")
    return team.trace


def publish(team, f, op, rng, interleaving):
    cfg = team.cfg
    body = BODIES[op.body]
    loop = op.loop
    master_view = team.frame_hash(f)
    team.barrier("all")                                   # fork: release workers
    for w in range(cfg.workers):                          # I1 at await
        if team.frame_hash(f) != master_view:
            raise Violation("I1: worker %d sees a frame different from the master's" % w)
    lo, hi = team_range(loop, team.tid, team.n_teams)
    partial = [0] * cfg.workers
    if op.body == "gather_nested":
        run_nested(team, f, loop, lo, hi, rng)
    else:
        queues = assign(range(lo, hi), cfg.workers, cfg.schedule, rng)
        steps = interleaving(queues) if interleaving else interleave(queues, cfg.interleave, rng)
        for w, i in steps:
            partial[w] += body.iteration(team, f, "w%d" % w, i, loop)
    # end of parallel: each worker stores its private partial in its own
    # control slot; the join barrier lets the master combine them
    team.barrier("all")
    if body.has_reduction:
        nb = body.slot_bytes
        cur = le_to_int(team.read(f, 0, nb, "master"))
        total = cur + sum(partial)
        if nb == 8:
            total = ((total + (1 << 63)) % (1 << 64)) - (1 << 63)
        team.write(f, 0, int_to_le(total, nb), "master")
        team.trace.partials.append(total)
    else:
        team.trace.partials.append(None)


def ref_sizes(body, loop):
    """Bytes of each referenced variable of a list-published body."""
    if body != "fma_chain_refs":
        raise SimError("INVAL", "body %r takes no reference list" % body)
    ni, nf, alen = loop["ni"], loop["nf"], loop.get("alen", 0)
    return [SLOT_F64_EXACT] + [4] * ni + [8] * nf + ([4 * alen] if alen else [])


def publish_list(team, pushed, op, rng, interleaving):
    """Fork through a list of references (section 5.2): up to 20 go to the
    team's on-chip list, more to a list frame on the global-memory stack
    that lives from the fork to the join."""
    cfg = team.cfg
    sizes = ref_sizes(op.body, op.loop)
    if len(op.refs) != len(sizes):
        raise SimError("INVAL", "%d references for %d variables" % (len(op.refs), len(sizes)))
    entries = []
    for (idx, off), nb in zip(op.refs, sizes):
        if idx >= len(pushed) or pushed[idx] not in team.frames:
            raise SimError("STATE", "reference into a frame that is not live")
        f = pushed[idx]
        if off < 0 or off + nb > f.nbytes:
            raise SimError("INVAL", "reference outside its frame")
        if off % (8 if nb in (8, SLOT_F64_EXACT) else 4):
            raise SimError("INVAL", "reference not naturally aligned")
        entries.append(struct.pack("<II", SPACE_CODE[f.space], f.off + off))
    n = len(entries)
    if n <= REF_LIST_ENTRIES:
        lf = FrameRec("list", CTL, 0, REF_LIST_ENTRIES * REF_BYTES, REF_BYTES * n, "team")
        m = team.mem[CTL]
        for b in range(REF_BYTES * n):
            m.writer[b] = None
            m.phase[b] = -1
        team.access(CTL, 0, REF_BYTES * n, "master", True, b"".join(entries), frames=[lf])
        global_list = None
    else:
        global_list = ("list", len(team.trace.lists))
        lf = team.push(global_list, REF_BYTES * n, global_only=True)
        team.write(lf, 0, b"".join(entries), "master")
    team.trace.lists.append((lf.space, lf.off, n))
    lst = RefList(lf)
    body = BODIES[op.body]
    loop = op.loop
    master_view = lst.view(team, n, sizes)
    team.barrier("all")                                   # fork: release workers
    for w in range(cfg.workers):                          # I1 at await
        if lst.view(team, n, sizes) != master_view:
            raise Violation("I1: worker %d sees a list or variable different from the master's" % w)
    lo, hi = team_range(loop, team.tid, team.n_teams)
    partial = [0] * cfg.workers
    queues = assign(range(lo, hi), cfg.workers, cfg.schedule, rng)
    steps = interleaving(queues) if interleaving else interleave(queues, cfg.interleave, rng)
    for w, i in steps:
        partial[w] += body.iteration(team, lst, "w%d" % w, i, loop)
    team.barrier("all")                                   # join
    sp, off = lst.ref(team, 0, "master")
    cur = le_to_int(team.access(sp, off, SLOT_F64_EXACT, "master", False))
    total = cur + sum(partial)
    team.access(sp, off, SLOT_F64_EXACT, "master", True, int_to_le(total, SLOT_F64_EXACT))
    team.trace.partials.append(total)
    if global_list is not None:
        team.pop(global_list)


def run_nested(team, outer_frame, loop, lo, hi, rng):
    """Second parallel level: the workers of the outer body are outer
    members; each pushes an inner frame on its own sub-stack, hands it to
    its inner members, and pops it after they finish."""
    cfg = team.cfg
    members = cfg.workers
    span = -(-(hi - lo) // members) if hi > lo else 0
    for m in range(members):
        mlo, mhi = min(hi, lo + m * span), min(hi, lo + (m + 1) * span)
        who = "w%d" % m
        sub = Memory("sub%d" % m, cfg.sub_bytes)
        size = round_up(16, cfg.align)
        if size > cfg.sub_bytes:
            raise SimError("NOMEM", "inner frame does not fit the sub-stack")
        team.trace.sub_placements.append(("sub%d" % m, 0, size))
        inner = struct.pack("<iiii", mlo, mhi, cfg.inner, outer_frame.fid)
        sub.data[0:16] = inner
        # inner members read the inner frame, then run their share
        for g in range(cfg.inner):
            vlo, vhi, stride, ref = struct.unpack("<iiii", bytes(sub.data[0:16]))
            if ref != outer_frame.fid:
                raise Violation("inner frame lost its outer reference")
            for i in range(vlo + g, vhi, stride):
                BODIES["gather"].iteration(team, outer_frame, who, i, loop)


def run_region(program, n_teams, cfg=None, interleaving=None):
    """Run ``program`` (list of Push/Publish/Pop) on ``n_teams`` teams.
    Returns (traces, reductions): reductions[p] is the p-th reducing
    publish's value combined over teams (int64 wrap for affine_xor, a
    correctly rounded float for fma_chain), or None if any team failed."""
    cfg = cfg or Config()
    traces = []
    for t in range(n_teams):
        traces.append(run_team(Team(t, cfg, n_teams), program, interleaving))
    pubs = [op for op in program if isinstance(op, (Publish, PublishList))]
    reductions = []
    if any(tr.error for tr in traces):
        return traces, None
    for p, op in enumerate(pubs):
        if not BODIES[op.body].has_reduction:
            reductions.append(None)
            continue
        vals = [tr.partials[p] for tr in traces]
        if op.body == "affine_xor":
            s = sum(vals)
            reductions.append(((s + (1 << 63)) % (1 << 64)) - (1 << 63))
        else:
            reductions.append(units_to_float(sum(vals)))
    return traces, reductions


# ---- helpers that build the frames of the standard bodies ----------------
def affine_xor_init(a, b, c, d):
    return struct.pack("<qiiii", 0, a, b, c, d)


def fma_chain_layout(ni, nf, alen):
    """(payload bytes, array offset) of an fma_chain frame."""
    base = SLOT_F64_EXACT + 8 * nf + 4 * ni
    if alen:
        aoff = round_up(base, 16)
        return aoff + 4 * alen, aoff
    return base, None


def fma_chain_init(s_i32, s_f64, arr=None):
    ni, nf = len(s_i32), len(s_f64)
    alen = 0 if arr is None else len(arr)
    size, aoff = fma_chain_layout(ni, nf, alen)
    b = bytearray(size)
    for k, v in enumerate(s_f64):
        struct.pack_into("<d", b, SLOT_F64_EXACT + 8 * k, float(v))
    for k, v in enumerate(s_i32):
        struct.pack_into("<i", b, SLOT_F64_EXACT + 8 * nf + 4 * k, int(v))
    if alen:
        b[aoff:aoff + 4 * alen] = np.asarray(arr, np.int32).tobytes()
    return bytes(b)


def gather_init(arrays):
    return b"".join(np.asarray(a, np.int32).tobytes() for a in arrays)
