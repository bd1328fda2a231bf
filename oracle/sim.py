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
  a private partial, and after the join the master adds the partials, in
  worker order, into the frame's slot.  The fp64 reduction is an exact
  rational sum, rounded once to nearest-even when the region's result is
  read: the plain definition of "sum += y[i]" with no rounding in between.
* Frames are popped in LIFO order and none may outlive the region.
* Nested parallelism (section 3.1.2; section 7's sharing at worker level):
  in a nested body each worker is the master of an inner team.  It pushes
  an inner frame on its own member stack, hands it to its inner members and
  pops it after they join; with three levels each inner member does the
  same again on its own lane-group stack.  A member stack lives on chip
  and overflows to the member's area of a global-memory stack when the
  on-chip part is exhausted (section 7), else the region fails with NOMEM.

Memory visibility.  Every thread has a private buffer of writes that the
others cannot see yet; a synchronisation of a scope (the team barrier, or
the barrier of one member's inner team) releases the buffered writes of
every thread in that scope.  A thread reads shared memory overlaid with its
own buffered writes.  So a worker that looked at a frame before the fork
barrier would see stale bytes, and invariant I1 below compares what each
worker actually sees with what its master wrote.

Every step checks the invariants
  I1 each worker's view of a published frame, taken at its await, equals
     the master's view of it at publish time (at every nesting level),
  I2 frames pop in LIFO order,
  I3 no frame outlives its region (nor an inner frame its outer body),
  I4 stack bytes in use equal the sum of the live frames' rounded sizes,
  I5 stack pointers stay within capacity; out-of-memory happens exactly
     when a frame fits neither space,
and a race detector that records, per byte, the last writer and the epochs
of the writer's scopes at the write, and flags a cross-thread access to a
byte unless a synchronisation of a scope holding both threads came after
the write, any access outside a live frame and any access after a pop.

Loop bodies (their frame layouts are the bodies' contracts):
  affine_xor   [0,8) int64 sum slot; a, b, c, d int32 at 8, 12, 16, 20.
               out[i] = a*i + b - (c ^ i) + d (int32 wrap); sum += out[i].
  fma_chain    [0,24) exact sum slot; nf fp64 scalars at 24; ni int32
               scalars after them; optional int32 array of alen elements at
               the next 16-byte boundary.  y[i] = fma chain (int32 scalars
               first, then fp64) over x[i] starting from arr[i mod alen]
               (or +0.0); sum += y[i] exactly.
  gather       A int32 arrays of ``length`` elements back to back at 0.
               out[i] = sum_j arr_j[i mod length] + i.
  gather_nested  as gather, run as ``depth`` (2 or 3) nested parallel
               levels.  Level 1: the workers split the team's range.  Each
               pushes a 16-byte inner frame {lo, hi, parent space, parent
               offset} on its member stack and hands it to its ``inner``
               members; these split [lo, hi) again.  At depth 3 each of them
               pushes a frame of the same shape, pointing at the inner
               frame, on its own lane-group stack for its ``inner`` members.
               The innermost members reach the team's frame by following
               the parent references, then gather.
  fma_chain_refs the fma_chain loop published through a list of references
               (section 5.2): reference 0 is the 24-byte exact sum slot,
               then ni int32 scalars, nf fp64 scalars and, if alen > 0, the
               int32 array, each anywhere in a live frame.  Lists of up to
               20 references go to the team's on-chip list (160 bytes);
               longer ones to a list frame on the global-memory stack,
               pushed at the fork and popped at the join.  Workers read a
               reference, then the variable through it, on every use.

Sizes are rounded up to ``align`` bytes (8 by default: section 5.3.1 aligns
the shared stack's variables to 8 bytes); frame offsets are multiples of
it.  Fractions give correctly rounded fma (one rounding of the exact a*b+c)
independently of the C oracle.
"""
from dataclasses import dataclass, field
from fractions import Fraction
import hashlib
import random
import struct

import numpy as np

LDS, HBM, CTL, NLDS, NHBM = "lds", "hbm", "ctl", "nlds", "nhbm"
REF_LIST_ENTRIES = 20             # references the on-chip list holds
REF_BYTES = 8                     # a reference: space (u32), offset (u32)
SLOT_F64_EXACT = 24
NEST_FRAME = 16                   # {lo, hi, parent space, parent offset}
UNIT_EXP = 75                     # the slot's bytes: a 192-bit integer of 2**-75 units
TEAM = "team"


class SimError(Exception):
    """A runtime error; ``code`` is one of NOMEM, ORDER, UNDERFLOW, LIVE,
    STATE, INVAL."""

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
    workers: int = 3              # worker threads per team (level-1 members)
    inner: int = 4                # inner members per member, at each nested level
    wave_lds: int = 64            # on-chip part of a level-1 member's stack
    wave_hbm: int = 256           # its global-memory part
    group_lds: int = 16           # on-chip part of a level-2 member's stack
    group_hbm: int = 64           # its global-memory part
    align: int = 8
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
    fid: object
    space: str
    off: int
    size: int                     # rounded size
    nbytes: int                   # declared size
    owner: str                    # "team" or the member that pushed it


@dataclass
class TeamTrace:
    placements: list = field(default_factory=list)   # (space, off, size) per push
    sub_placements: list = field(default_factory=list)  # (level, member, space, off, size)
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


def int_to_le(v, nbytes):
    return (v % (1 << (8 * nbytes))).to_bytes(nbytes, "little")


def le_to_int(b):
    v = int.from_bytes(b, "little")
    return v - (1 << (8 * len(b))) if v >> (8 * len(b) - 1) else v


def scopes_of(who):
    """The synchronisation scopes holding thread ``who``, outermost first:
    the team, then each member whose inner team it belongs to, then its own
    inner team (a member is the master of the team it forks)."""
    if who == "master":
        return [TEAM]
    parts = who.split(".")
    return [TEAM] + [".".join(parts[:k]) for k in range(1, len(parts) + 1)]


class Memory:
    """Byte store of one space with a per-byte shadow: the last writer and
    the epochs of its scopes at the write."""

    def __init__(self, name, size):
        self.name = name
        self.data = bytearray(size)
        self.shadow = [None] * size


class MemberStack:
    """A nested member's stack: an on-chip part and a global-memory part,
    each a LIFO bump region at a fixed base of the team's nested areas."""

    def __init__(self, team, owner, level, lds_base, lds_cap, hbm_base, hbm_cap):
        self.team, self.owner, self.level = team, owner, level
        self.base = {NLDS: lds_base, NHBM: hbm_base}
        self.cap = {NLDS: lds_cap, NHBM: hbm_cap}
        self.sp = {NLDS: 0, NHBM: 0}
        self.frames = []

    def check(self):
        used = {NLDS: 0, NHBM: 0}
        for f in self.frames:
            used[f.space] += f.size
        for s in (NLDS, NHBM):
            if used[s] != self.sp[s]:
                raise Violation("I4: %s stack of %s: %d bytes, live frames %d"
                                % (s, self.owner, self.sp[s], used[s]))
            if self.sp[s] > self.cap[s]:
                raise Violation("I5: %s stack of %s beyond capacity" % (s, self.owner))

    def push(self, nbytes):
        size = round_up(nbytes, self.team.cfg.align)
        if self.sp[NLDS] + size <= self.cap[NLDS]:
            space = NLDS
        elif self.sp[NHBM] + size <= self.cap[NHBM]:
            space = NHBM
        else:
            raise SimError("NOMEM", "nested frame of %d bytes fits neither stack of %s" % (size, self.owner))
        f = FrameRec(("nest", self.owner, len(self.team.trace.sub_placements)), space,
                     self.base[space] + self.sp[space], size, nbytes, self.owner)
        self.sp[space] += size
        self.frames.append(f)
        self.team.fresh(f)
        self.team.trace.sub_placements.append((self.level, self.owner, space, f.off, size))
        self.check()
        return f

    def pop(self, f):
        if not self.frames:
            raise SimError("UNDERFLOW", "pop on the empty stack of %s" % self.owner)
        if self.frames[-1] is not f:
            raise SimError("ORDER", "nested pop of a frame that is not the top")
        self.frames.pop()
        self.sp[f.space] -= f.size
        self.team.dead.add(f.fid)
        self.check()


class Team:
    def __init__(self, tid, cfg, n_teams):
        self.tid = tid
        self.cfg = cfg
        self.n_teams = n_teams
        m, g = cfg.workers, cfg.inner
        self.mem = {LDS: Memory(LDS, cfg.lds_bytes), HBM: Memory(HBM, cfg.hbm_bytes),
                    CTL: Memory(CTL, REF_LIST_ENTRIES * REF_BYTES),
                    NLDS: Memory(NLDS, m * cfg.wave_lds + m * g * cfg.group_lds),
                    NHBM: Memory(NHBM, m * cfg.wave_hbm + m * g * cfg.group_hbm)}
        self.sp = {LDS: 0, HBM: 0}
        self.frames = []           # live team-level frames, bottom .. top
        self.by_id = {}
        self.dead = set()
        self.epoch = {TEAM: 0}
        self.pending = {}          # thread -> {(space, byte): value} not yet released
        self.exact = {}            # (space, offset) -> exact value of an fp64 sum slot
        self.members = {}          # owner -> MemberStack
        self.trace = TeamTrace(worker_barriers=[0] * cfg.workers)

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

    def live_frames(self):
        out = list(self.frames)
        for ms in self.members.values():
            out += ms.frames
        return out

    # -- synchronisation --------------------------------------------------
    def sync(self, scope):
        """Release the buffered writes of every thread in ``scope`` and
        start a new epoch of it (a barrier of that scope)."""
        for who in list(self.pending):
            if scope == TEAM or who == scope or who.startswith(scope + "."):
                for (space, b), v in self.pending.pop(who).items():
                    self.mem[space].data[b] = v
        self.epoch[scope] = self.epoch.get(scope, 0) + 1

    def barrier(self, participants="all"):
        self.sync(TEAM)
        self.trace.master_barriers += 1
        for w in range(self.cfg.workers):
            self.trace.worker_barriers[w] += 1

    def ordered(self, rec, who):
        """Whether a write recorded as ``rec`` happens before an access by
        ``who``: same thread, or a later sync of a scope holding both."""
        writer, snap = rec
        if writer == who:
            return True
        for s in scopes_of(who):
            if s in snap and self.epoch.get(s, 0) > snap[s]:
                return True
        return False

    # -- memory access through (space, offset) -----------------------------
    def access(self, space, off, n, who, write, data=None, frames=None):
        pool = self.live_frames() if frames is None else frames
        ok = any(f.space == space and f.off <= off and off + n <= f.off + f.size for f in pool)
        if not ok:
            raise Violation("race detector: %s access [%d,%d) of %s outside a live frame"
                            % (who, off, off + n, space))
        m = self.mem[space]
        for b in range(off, off + n):
            rec = m.shadow[b]
            if rec is not None and not self.ordered(rec, who):
                raise Violation("race detector: %s %s byte %d of %s written by %s with no sync between"
                                % (who, "writes" if write else "reads", b, space, rec[0]))
        if write:
            buf = self.pending.setdefault(who, {})
            snap = {s: self.epoch.get(s, 0) for s in scopes_of(who)}
            for k in range(n):
                buf[(space, off + k)] = data[k]
                m.shadow[off + k] = (who, snap)
            return None
        return self.view(space, off, n, who)

    def view(self, space, off, n, who):
        """Bytes [off, off+n) of ``space`` as thread ``who`` sees them."""
        buf = self.pending.get(who, {})
        d = self.mem[space].data
        return bytes(buf.get((space, b), d[b]) for b in range(off, off + n))

    def frame_view(self, f, who):
        return hashlib.sha256(self.view(f.space, f.off, f.nbytes, who)).hexdigest()

    def fresh(self, f):
        """A newly pushed frame holds no one's data."""
        m = self.mem[f.space]
        for b in range(f.off, f.off + f.size):
            m.shadow[b] = None
        for k in [k for k in self.exact if k[0] == f.space and f.off <= k[1] < f.off + f.size]:
            del self.exact[k]

    def read(self, f, off, n, who, frames=None):
        if f.fid in self.dead:
            raise Violation("race detector: %s reads frame %r after its pop" % (who, f.fid))
        if off < 0 or off + n > f.nbytes:
            raise Violation("race detector: %s reads [%d,%d) outside frame %r of %d bytes"
                            % (who, off, off + n, f.fid, f.nbytes))
        return self.access(f.space, f.off + off, n, who, False, frames=frames)

    def write(self, f, off, data, who, frames=None):
        if f.fid in self.dead:
            raise Violation("race detector: %s writes frame %r after its pop" % (who, f.fid))
        if off < 0 or off + len(data) > f.nbytes:
            raise Violation("race detector: %s writes outside frame %r" % (who, f.fid))
        self.access(f.space, f.off + off, len(data), who, True, data, frames=frames)

    # -- exact fp64 sum slots ----------------------------------------------
    def read_exact(self, space, off, who):
        raw = self.access(space, off, SLOT_F64_EXACT, who, False)
        if (space, off) in self.exact:
            return self.exact[(space, off)]
        return Fraction(le_to_int(raw), 1 << UNIT_EXP)

    def write_exact(self, space, off, value, who):
        """The slot holds the exact value; its bytes hold the value's
        2**-75-unit encoding (truncated when it is off that grid)."""
        self.exact[(space, off)] = value
        units = (value.numerator << UNIT_EXP) // value.denominator
        self.access(space, off, SLOT_F64_EXACT, who, True, int_to_le(units, SLOT_F64_EXACT))

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
        self.fresh(f)
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

    # -- nested member stacks ------------------------------------------------
    def wave_stack(self, m):
        c = self.cfg
        key = "w%d" % m
        if key not in self.members:
            self.members[key] = MemberStack(self, key, 2, m * c.wave_lds, c.wave_lds, m * c.wave_hbm, c.wave_hbm)
        return self.members[key]

    def group_stack(self, m, g):
        c = self.cfg
        key = "w%d.g%d" % (m, g)
        if key not in self.members:
            k = m * c.inner + g
            self.members[key] = MemberStack(self, key, 3, c.workers * c.wave_lds + k * c.group_lds,
                                            c.group_lds, c.workers * c.wave_hbm + k * c.group_hbm,
                                            c.group_hbm)
        return self.members[key]


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


def split(lo, hi, parts, k):
    """Part k of [lo, hi) cut into ``parts`` contiguous pieces."""
    per = -(-(hi - lo) // parts) if hi > lo else 0
    return min(hi, lo + k * per), min(hi, lo + (k + 1) * per)


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
    reduction = None              # None, "i64" or "exact"
    slot_bytes = 0

    def iteration(self, team, f, who, i, loop):
        raise NotImplementedError


class AffineXor(Body):
    reduction = "i64"
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
    reduction = "exact"
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
        return exact(acc, i)


def exact(y, i):
    if y != y or y in (float("inf"), float("-inf")):
        raise SimError("INVAL", "y[%d] = %r has no exact sum" % (i, y))
    return Fraction(y)


def gather_at(team, space, off, who, i, loop):
    """out[i] from A arrays of ``length`` int32 at (space, off)."""
    A, length = loop["A"], loop["length"]
    s = i
    for j in range(A):
        s += _i32(team.access(space, off + 4 * (j * length + i % length), 4, who, False))
    loop["out"][i] = ((s + (1 << 31)) % (1 << 32)) - (1 << 31)
    return 0


class Gather(Body):
    def iteration(self, team, f, who, i, loop):
        if f.fid in team.dead:
            raise Violation("race detector: %s reads frame %r after its pop" % (who, f.fid))
        if 4 * loop["A"] * loop["length"] > f.nbytes:
            raise Violation("race detector: arrays beyond frame %r" % (f.fid,))
        return gather_at(team, f.space, f.off, who, i, loop)


class FmaChainRefs(Body):
    """fma_chain through references: every variable is reached by reading
    its reference from the list, then the variable (section 5.2)."""
    reduction = "exact"
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
        return exact(acc, i)


BODIES = {"affine_xor": AffineXor(), "fma_chain": FmaChain(), "gather": Gather(),
          "gather_nested": Gather(), "fma_chain_refs": FmaChainRefs()}
SPACE_CODE = {LDS: 0, HBM: 1, NLDS: 4, NHBM: 5}
CODE_SPACE = {v: k for k, v in SPACE_CODE.items()}


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

    def view(self, team, n, sizes, who):
        """Bytes of the list and of every variable it references, as
        thread ``who`` sees them."""
        lst = team.view(self.frame.space, self.frame.off, REF_BYTES * n, who)
        h = hashlib.sha256(lst)
        for k in range(n):
            code, off = struct.unpack_from("<II", lst, REF_BYTES * k)
            h.update(team.view(CODE_SPACE[code], off, sizes[k], who))
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


def check_views(team, who_list, expect, view):
    for w in who_list:
        if view(w) != expect:
            raise Violation("I1: %s sees a frame different from its master's" % w)


def combine(team, body, slot_space, slot_off, partial):
    """After the join: the master adds the workers' partials, in worker
    order, into the shared slot."""
    if body.reduction == "i64":
        cur = le_to_int(team.access(slot_space, slot_off, 8, "master", False))
        total = ((cur + sum(partial) + (1 << 63)) % (1 << 64)) - (1 << 63)
        team.access(slot_space, slot_off, 8, "master", True, int_to_le(total, 8))
    else:
        total = team.read_exact(slot_space, slot_off, "master") + sum(partial, Fraction(0))
        team.write_exact(slot_space, slot_off, total, "master")
    team.trace.partials.append(total)


def publish(team, f, op, rng, interleaving):
    cfg = team.cfg
    body = BODIES[op.body]
    loop = op.loop
    master_view = team.frame_view(f, "master")
    team.barrier("all")                                   # fork: release workers
    check_views(team, ["w%d" % w for w in range(cfg.workers)], master_view,
                lambda w: team.frame_view(f, w))          # I1 at await
    lo, hi = team_range(loop, team.tid, team.n_teams)
    partial = [0] * cfg.workers
    if op.body == "gather_nested":
        run_nested(team, f, loop, lo, hi)
    else:
        queues = assign(range(lo, hi), cfg.workers, cfg.schedule, rng)
        steps = interleaving(queues) if interleaving else interleave(queues, cfg.interleave, rng)
        for w, i in steps:
            partial[w] += body.iteration(team, f, "w%d" % w, i, loop)
    # end of parallel: each worker keeps its private partial; the join
    # barrier lets the master combine them
    team.barrier("all")
    if body.reduction:
        combine(team, body, f.space, f.off, partial)
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
        team.fresh(lf)
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
    master_view = lst.view(team, n, sizes, "master")
    team.barrier("all")                                   # fork: release workers
    check_views(team, ["w%d" % w for w in range(cfg.workers)], master_view,
                lambda w: lst.view(team, n, sizes, w))    # I1 at await
    lo, hi = team_range(loop, team.tid, team.n_teams)
    partial = [0] * cfg.workers
    queues = assign(range(lo, hi), cfg.workers, cfg.schedule, rng)
    steps = interleaving(queues) if interleaving else interleave(queues, cfg.interleave, rng)
    for w, i in steps:
        partial[w] += body.iteration(team, lst, "w%d" % w, i, loop)
    team.barrier("all")                                   # join
    sp, off = lst.ref(team, 0, "master")
    combine(team, body, sp, off, partial)
    if global_list is not None:
        team.pop(global_list)


def nested_fork(team, stack, who, lo, hi, parent):
    """Member ``who`` pushes the frame {lo, hi, parent ref} on its own
    stack and releases it to its inner members (their barrier)."""
    f = stack.push(NEST_FRAME)
    team.write(f, 0, struct.pack("<IIII", lo, hi, SPACE_CODE[parent.space], parent.off), who)
    view = team.frame_view(f, who)
    team.sync(who)
    return f, view


def read_nested(team, f, who):
    lo, hi, code, off = struct.unpack("<IIII", team.read(f, 0, NEST_FRAME, who))
    if code not in CODE_SPACE:
        raise Violation("nested frame names no space")
    return lo, hi, CODE_SPACE[code], off


def frame_at(team, space, off):
    """The live frame that starts at (space, off): what a reference names."""
    for f in team.live_frames():
        if f.space == space and f.off == off:
            return f
    raise Violation("reference to (%s, %d) names no live frame" % (space, off))


def run_nested(team, outer_frame, loop, lo, hi):
    """Nested levels below the team's fork (see gather_nested above): every
    member is the master of an inner team, shares a frame with it through
    its own stack, and pops the frame after the inner team joins."""
    cfg = team.cfg
    depth = loop.get("depth", 2)
    if depth not in (2, 3):
        raise SimError("INVAL", "nesting depth %r" % depth)
    for m in range(cfg.workers):
        who = "w%d" % m
        mlo, mhi = split(lo, hi, cfg.workers, m)
        ws = team.wave_stack(m)
        f2, v2 = nested_fork(team, ws, who, mlo, mhi, outer_frame)
        inner = ["%s.g%d" % (who, g) for g in range(cfg.inner)]
        check_views(team, inner, v2, lambda w: team.frame_view(f2, w))     # I1, level 2
        for g, gwho in enumerate(inner):
            vlo, vhi, psp, poff = read_nested(team, f2, gwho)
            glo, ghi = split(vlo, vhi, cfg.inner, g)
            if depth == 2:
                for i in range(glo, ghi):
                    gather_at(team, psp, poff, gwho, i, loop)
                continue
            gs = team.group_stack(m, g)
            f3, v3 = nested_fork(team, gs, gwho, glo, ghi, f2)
            leaves = ["%s.s%d" % (gwho, s) for s in range(cfg.inner)]
            check_views(team, leaves, v3, lambda w: team.frame_view(f3, w))  # I1, level 3
            for s, swho in enumerate(leaves):
                slo, shi, qsp, qoff = read_nested(team, f3, swho)
                _, _, osp, ooff = read_nested(team, frame_at(team, qsp, qoff), swho)
                a, b = split(slo, shi, cfg.inner, s)
                for i in range(a, b):
                    gather_at(team, osp, ooff, swho, i, loop)
            team.sync(gwho)                                # inner join
            gs.pop(f3)
        team.sync(who)                                     # inner join
        ws.pop(f2)
    for ms in team.members.values():                       # I3 for nested frames
        if ms.frames:
            raise Violation("I3: a nested frame of %s outlives its body" % ms.owner)


def run_region(program, n_teams, cfg=None, interleaving=None):
    """Run ``program`` (list of Push/Publish/Pop) on ``n_teams`` teams.
    Returns (traces, reductions): reductions[p] is the p-th reducing
    publish's value combined over teams (int64 wrap for affine_xor, the
    exact sum rounded once to nearest-even double for the fma chains), or
    None if any team failed."""
    cfg = cfg or Config()
    traces = []
    for t in range(n_teams):
        traces.append(run_team(Team(t, cfg, n_teams), program, interleaving))
    pubs = [op for op in program if isinstance(op, (Publish, PublishList))]
    reductions = []
    if any(tr.error for tr in traces):
        return traces, None
    for p, op in enumerate(pubs):
        kind = BODIES[op.body].reduction
        if not kind:
            reductions.append(None)
            continue
        vals = [tr.partials[p] for tr in traces]
        if kind == "i64":
            s = sum(vals)
            reductions.append(((s + (1 << 63)) % (1 << 64)) - (1 << 63))
        else:
            reductions.append(float(sum(vals, Fraction(0))))
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


# ---- served requests sized to their stacks (section 7) -------------------
# Section 7 proposes to size a team's shared memory to what the kernel needs
# instead of preallocating one size for every case.  A server that runs
# resident teams of a few LDS sizes ("classes") does this per request: the
# request goes to the smallest class whose on-chip stack holds every frame
# the request pushes; a request no class holds goes to the largest, where
# the frames that do not fit take the global-memory stack as usual.
def stack_peak(program, align=8):
    """Bytes a region's program holds on its stack at the most, every frame
    rounded up to `align`: the largest sum of the live frames' sizes over
    the program's pushes and pops (LIFO)."""
    live, cur, peak = [], 0, 0
    for op in program:
        if isinstance(op, Push):
            live.append(round_up(op.nbytes, align))
            cur += live[-1]
            peak = max(peak, cur)
        elif isinstance(op, Pop):
            cur -= live.pop()
    return peak


def lds_class(program, slabs, align=8):
    """Index in `slabs` (on-chip stack bytes per class, any order) of the
    class a request with this program is admitted to."""
    need = stack_peak(program, align)
    fits = [k for k, s in enumerate(slabs) if s >= need]
    if fits:
        return min(fits, key=lambda k: (slabs[k], k))
    return max(range(len(slabs)), key=lambda k: (slabs[k], -k))
