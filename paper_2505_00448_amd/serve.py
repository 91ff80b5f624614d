"""Continuous-batching query server for the interactive-explorer use case.

The paper motivates fast all-pairs association on the fly in an interactive
explorer over a cohort (NApy, Sections 1 and 6): a user picks a subset
of the samples and a subset of the variables and wants the correlation
matrices back at once.  Here that becomes a request loop on one GPU:

* the base matrix X (samples x variables) stays resident in device memory,
  and its columns are sorted once for Spearman (the sort-once structure of
  Section 3.5.3 reused across queries);
* a query is (row set, variable list, method) and returns r, p and n over
  X[rows][:, cols], exactly what the full call returns on that submatrix;
* queries are admitted as soon as a slot (one HIP stream each) is free and
  the query's device memory (workspace, outputs, index arrays) fits in the
  server's arena; queries that arrive while others run are admitted as
  slots and memory free up, so their kernels overlap on the device.  The
  oldest waiting query goes first; when its memory does not fit yet, a few
  younger ones that do fit may go ahead of it, a bounded number of times
  (after that it waits for memory alone), so small queries are not held up
  by a large one and a large one is not starved;
* every kernel of a query runs on its own slot's stream with a tiling fixed
  by the query's own shape, so a result does not depend on which other
  queries share the device at the time.

All arithmetic runs in libnapy's kernels; this module only moves indices,
carves memory and orders launches.
"""

from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

ALIGN = 256


def _round_up(x: int, a: int = ALIGN) -> int:
    return (int(x) + a - 1) // a * a


# ---------------------------------------------------------------------------
# host-side pieces (no GPU): arena allocator and admission scheduler
# ---------------------------------------------------------------------------

class Arena:
    """First-fit allocator over byte offsets [0, capacity) with 256-byte
    granularity; adjacent free ranges are merged on release."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity) // ALIGN * ALIGN
        self._free = [(0, self.capacity)]   # sorted (offset, size)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        size = _round_up(max(int(nbytes), 1))
        for i, (off, sz) in enumerate(self._free):
            if sz >= size:
                if sz == size:
                    del self._free[i]
                else:
                    self._free[i] = (off + size, sz - size)
                self.used += size
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        size = _round_up(max(int(nbytes), 1))
        lo, hi = 0, len(self._free)
        while lo < hi:
            mid = (lo + hi) // 2
            if self._free[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        i = lo
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] > off:
            raise ValueError(f"double release of arena offset {off}")
        if i < len(self._free) and off + size > self._free[i][0]:
            raise ValueError(f"double release of arena offset {off}")
        self._free.insert(i, (off, size))
        if i + 1 < len(self._free) and off + size == self._free[i + 1][0]:
            self._free[i] = (off, size + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == off:
            self._free[i - 1] = (self._free[i - 1][0], self._free[i - 1][1] + self._free[i][1])
            del self._free[i]
        self.used -= size

    def free_bytes(self) -> int:
        return sum(sz for _, sz in self._free)


@dataclass
class Request:
    qid: int
    method: str                 # "pearson" or "spearman"
    rows: np.ndarray            # int32, ascending, distinct sample indices
    cols: np.ndarray            # int32, distinct variable indices
    arrival: float = 0.0        # host monotonic seconds
    nbytes: int = -1            # device bytes, filled in at submission


@dataclass
class Completion:
    qid: int
    method: str
    n_rows: int
    n_cols: int
    arrival: float
    admitted: float
    done: float
    slot: int
    outputs: dict = field(default_factory=dict)   # device views, valid inside the callback only

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def pairs(self) -> int:
        return self.n_cols * (self.n_cols - 1) // 2


class Scheduler:
    """Continuous batching over `slots` independent slots and an arena of
    device memory.  The executor supplies

        nbytes(req) -> int          device bytes the query needs
        launch(req, slot, offset)   enqueue the query's work (non-blocking)
        is_done(slot) -> bool       the slot's last launch has completed
        outputs(req, slot, offset)  views of the finished outputs

    and optionally validate(req) (raises on a malformed request),
    retire(slot, completion) (bookkeeping when a query is retired) and
    released() (called after a retired query's callback, before its memory
    can be handed to another query).

    Admission: a request is admitted once a slot is free and its bytes fit in
    the arena.  The oldest waiting request (the head) goes first.  When the
    head's bytes do not fit, the first of the next `lookahead` requests whose
    bytes fit is admitted ahead of it, at most `max_overtakes` times per head;
    after that nothing overtakes it, so it is admitted as soon as memory for
    it frees up."""

    def __init__(self, executor, slots: int, capacity: int,
                 clock: Callable[[], float] = time.perf_counter,
                 lookahead: int = 8, max_overtakes: int = 16):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.ex = executor
        self.arena = Arena(capacity)
        self.clock = clock
        self.pending: deque = deque()
        self.free_slots = list(range(slots - 1, -1, -1))
        self.running = {}          # slot -> (req, offset, nbytes, t_admit)
        self.max_running = 0
        self.lookahead = max(0, int(lookahead))
        self.max_overtakes = max(0, int(max_overtakes))
        self.head_overtaken = 0    # times the current head has been overtaken
        self.overtakes = 0         # total admissions ahead of an older request

    def submit(self, req: Request) -> None:
        if hasattr(self.ex, "validate"):
            self.ex.validate(req)
        need = self.ex.nbytes(req)
        req.nbytes = need
        if _round_up(need) > self.arena.capacity:
            raise ValueError(f"query {req.qid} needs {need} bytes, more than the server's "
                             f"arena of {self.arena.capacity} bytes")
        self.pending.append(req)

    def idle(self) -> bool:
        return not self.pending and not self.running

    def step(self, on_done: Optional[Callable[[Completion], None]] = None) -> int:
        """Retire finished queries, then admit what fits.  Returns the number
        of queries retired."""
        retired = 0
        for slot in list(self.running):
            if self.ex.is_done(slot):
                req, off, nb, t_adm = self.running.pop(slot)
                t = self.clock()
                comp = Completion(req.qid, req.method, len(req.rows), len(req.cols),
                                  req.arrival, t_adm, t, slot)
                if hasattr(self.ex, "retire"):
                    self.ex.retire(slot, comp)
                if on_done is not None:
                    comp.outputs = self.ex.outputs(req, slot, off)
                    on_done(comp)
                    comp.outputs = {}
                    if hasattr(self.ex, "released"):
                        self.ex.released()
                self.arena.release(off, nb)
                self.free_slots.append(slot)
                retired += 1
        while self.pending and self.free_slots:
            pick, off, nb = self._choose()
            if pick is None:
                break
            req = self.pending[pick]
            del self.pending[pick]
            if pick == 0:
                self.head_overtaken = 0
            else:
                self.head_overtaken += 1
                self.overtakes += 1
            slot = self.free_slots.pop()
            t_adm = self.clock()
            self.ex.launch(req, slot, off)
            self.running[slot] = (req, off, nb, t_adm)
            self.max_running = max(self.max_running, len(self.running))
        return retired

    def _nbytes(self, req: Request) -> int:
        return req.nbytes if req.nbytes >= 0 else self.ex.nbytes(req)

    def _choose(self):
        """(index in pending, arena offset, bytes) of the request to admit
        next, or (None, None, None)."""
        nb = self._nbytes(self.pending[0])
        off = self.arena.alloc(nb)
        if off is not None:
            return 0, off, nb
        if self.head_overtaken >= self.max_overtakes:
            return None, None, None
        for k in range(1, min(len(self.pending), 1 + self.lookahead)):
            nb = self._nbytes(self.pending[k])
            off = self.arena.alloc(nb)
            if off is not None:
                return k, off, nb
        return None, None, None


# ---------------------------------------------------------------------------
# GPU executor and server
# ---------------------------------------------------------------------------

class _Carve:
    def __init__(self, base: int):
        self.off = base

    def take(self, nbytes: int) -> int:
        o = self.off
        self.off += _round_up(max(int(nbytes), 1))
        return o


class GpuExecutor:
    """Runs subset queries through libnapy on per-slot HIP streams, with all
    per-query memory carved from one device arena tensor."""

    def __init__(self, X, slots: int, capacity: int, precision: str = "bf16x3",
                 missing: Optional[float] = None, spearman: bool = True):
        import torch
        from . import _lib
        from .api import SpearmanBase, _prep_input
        self.torch = torch
        self.lib = _lib.load()
        self._lib = _lib
        self.X = _prep_input(X, 0, True)
        self.S, self.F = self.X.shape
        self.dev = self.X.device
        self.precision = precision
        self.missing = missing
        self.sbase = SpearmanBase(self.X, missing) if spearman else None
        self.arena = torch.empty(_round_up(capacity), dtype=torch.uint8, device=self.dev)
        self.base_ptr = self.arena.data_ptr()
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]
        self.events = [None] * slots
        self.t_events = [None] * slots
        # work the result callbacks queued on torch's current stream (device
        # copies of a finished query's outputs) must complete before the
        # arena memory they read is written by a later query
        self.fence = None
        self.spans = []
        self.staging = [torch.empty(self.S + self.F + 2, dtype=torch.int32).pin_memory()
                        for _ in range(slots)]
        self.opts_p = _lib.make_opts(precision, missing)
        self.opts_s = _lib.make_opts("fp32", missing)
        torch.cuda.synchronize(self.dev)

    # -- sizes --------------------------------------------------------------
    def _ws_bytes(self, req: Request) -> int:
        Sq, Fq = len(req.rows), len(req.cols)
        if req.method == "pearson":
            need = self.lib.napy_pearson_subset_workspace(Sq, Fq, ctypes.byref(self.opts_p))
        elif req.method == "spearman":
            if self.sbase is None:
                raise ValueError("this server was built without the Spearman base")
            need = self.lib.napy_spearman_subset_workspace(self.S, Sq, Fq, ctypes.byref(self.opts_s))
        else:
            raise ValueError(f"unknown method {req.method!r}")
        if need == 0:
            raise ValueError(f"query {req.qid}: shape Sq={Sq}, Fq={Fq} refused by the library")
        return int(need)

    def _layout(self, req: Request, off: int):
        Sq, Fq = len(req.rows), len(req.cols)
        c = _Carve(self.base_ptr + off)
        rows = c.take(4 * max(Sq, 1))
        cols = c.take(4 * Fq)
        r = c.take(8 * Fq * Fq)
        p = c.take(8 * Fq * Fq)
        n = c.take(4 * Fq * Fq)
        ws_bytes = self._ws_bytes(req)
        ws = c.take(ws_bytes)
        return rows, cols, r, p, n, ws, ws_bytes, c.off - (self.base_ptr + off)

    def nbytes(self, req: Request) -> int:
        if len(req.cols) < 1 or len(req.cols) > self.F or len(req.rows) > self.S:
            raise ValueError(f"query {req.qid}: {len(req.rows)} rows x {len(req.cols)} cols "
                             f"does not fit the base {self.S} x {self.F}")
        return self._layout(req, 0)[-1]

    # -- launch / poll ------------------------------------------------------
    def validate(self, req: Request) -> None:
        rows = np.asarray(req.rows)
        cols = np.asarray(req.cols)
        if rows.dtype != np.int32 or cols.dtype != np.int32 or rows.ndim != 1 or cols.ndim != 1:
            raise ValueError(f"query {req.qid}: rows and cols must be 1-D int32 arrays")
        if len(rows) and (rows[0] < 0 or rows[-1] >= self.S or np.any(np.diff(rows) <= 0)):
            raise ValueError(f"query {req.qid}: rows must be ascending, distinct and in [0, {self.S})")
        if len(cols) == 0 or cols.min() < 0 or cols.max() >= self.F or len(np.unique(cols)) != len(cols):
            raise ValueError(f"query {req.qid}: cols must be non-empty, distinct and in [0, {self.F})")

    def released(self) -> None:
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.dev))
        self.fence = ev

    def launch(self, req: Request, slot: int, off: int) -> None:
        torch = self.torch
        Sq, Fq = len(req.rows), len(req.cols)
        rows, cols, r, p, n, ws, ws_bytes, _ = self._layout(req, off)
        s = self.streams[slot]
        if self.fence is not None:
            s.wait_event(self.fence)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        stg = self.staging[slot]
        stg_np = stg.numpy()
        stg_np[:Sq] = req.rows
        stg_np[Sq:Sq + Fq] = req.cols
        # one async copy of both index arrays; rows and cols sit back to back
        # in the staging buffer but at 256-byte aligned places in the arena
        dst_rows = self._view_i32(rows, Sq)
        dst_cols = self._view_i32(cols, Fq)
        with torch.cuda.stream(s):
            if Sq:
                dst_rows.copy_(stg[:Sq], non_blocking=True)
            dst_cols.copy_(stg[Sq:Sq + Fq], non_blocking=True)
        sh = ctypes.c_void_p(s.cuda_stream)
        V = ctypes.c_void_p
        if req.method == "pearson":
            st = self.lib.napy_pearson_subset(V(self.X.data_ptr()), self.S, self.F, self.X.stride(0),
                                              V(rows), Sq, V(cols), Fq, V(r), V(p), V(n), Fq,
                                              V(ws), ws_bytes, ctypes.byref(self.opts_p), sh)
        else:
            st = self.lib.napy_spearman_subset(V(self.sbase.buf.data_ptr()), self.S, self.F,
                                               V(rows), Sq, V(cols), Fq, V(r), V(p), V(n), Fq,
                                               V(ws), ws_bytes, ctypes.byref(self.opts_s), sh)
        self._lib.check(st, f"query {req.qid} ({req.method})")
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        self.events[slot] = ev
        self.t_events[slot] = ev0

    def retire(self, slot: int, comp: "Completion") -> None:
        self.spans.append((self.t_events[slot], self.events[slot]))

    def busy_ms(self, ref) -> float:
        """Length of the union of the device intervals [start, end] of the
        retired queries, measured with their HIP events."""
        iv = sorted((ref.elapsed_time(a), ref.elapsed_time(b)) for a, b in self.spans)
        total, cur_lo, cur_hi = 0.0, None, None
        for lo, hi in iv:
            if cur_hi is None or lo > cur_hi:
                if cur_hi is not None:
                    total += cur_hi - cur_lo
                cur_lo, cur_hi = lo, hi
            else:
                cur_hi = max(cur_hi, hi)
        if cur_hi is not None:
            total += cur_hi - cur_lo
        return total

    def is_done(self, slot: int) -> bool:
        ev = self.events[slot]
        return ev is None or ev.query()

    def _view_i32(self, addr: int, count: int):
        off = addr - self.base_ptr
        return self.arena[off:off + 4 * max(count, 0)].view(self.torch.int32)

    def outputs(self, req: Request, slot: int, off: int) -> dict:
        torch = self.torch
        Fq = len(req.cols)
        _, _, r, p, n, _, _, _ = self._layout(req, off)
        o = lambda a: a - self.base_ptr
        R = self.arena[o(r):o(r) + 8 * Fq * Fq].view(torch.float64).view(Fq, Fq)
        P = self.arena[o(p):o(p) + 8 * Fq * Fq].view(torch.float64).view(Fq, Fq)
        N = self.arena[o(n):o(n) + 4 * Fq * Fq].view(torch.int32).view(Fq, Fq)
        return {"r": R, "p": P, "n": N}


class Server:
    """Resident base matrix + continuous-batching request loop.

    >>> srv = Server(X, slots=4, capacity=4 << 30)
    >>> stats = srv.serve(requests, on_done=callback)   # requests carry arrival offsets

    Results are handed to `on_done(completion)` as device views into the
    arena, valid only during the callback: copy what must be kept (a device
    copy queued on torch's current stream is fine; later queries wait for
    that stream's work before they reuse the memory).  The memory is released
    when the callback returns."""

    def __init__(self, X, slots: int = 4, capacity: int = 4 << 30, precision: str = "bf16x3",
                 missing: Optional[float] = None, spearman: bool = True):
        self.ex = GpuExecutor(X, slots, capacity, precision, missing, spearman)
        self.slots = slots
        self.capacity = capacity

    def serve(self, requests, on_done: Optional[Callable[[Completion], None]] = None,
              realtime: bool = True) -> dict:
        """Replay `requests` (Request.arrival = seconds after the start).
        With realtime=True a request is submitted when its arrival time has
        passed on the host clock; with False all are submitted at once (a
        burst).  Latency is measured from the arrival time to the moment the
        host sees the query's completion event."""
        torch = self.ex.torch
        sched = Scheduler(self.ex, self.slots, self.capacity)
        reqs = sorted(requests, key=lambda q: q.arrival)
        comps = []

        def record(c: Completion):
            comps.append(c)
            if on_done is not None:
                on_done(c)

        torch.cuda.synchronize(self.ex.dev)
        self.ex.spans = []
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(torch.cuda.current_stream(self.ex.dev))
        t0 = time.perf_counter()
        i = 0
        while i < len(reqs) or not sched.idle():
            now = time.perf_counter()
            while i < len(reqs) and (not realtime or t0 + reqs[i].arrival <= now):
                q = reqs[i]
                q = Request(q.qid, q.method, q.rows, q.cols, t0 + q.arrival if realtime else now)
                sched.submit(q)
                i += 1
            sched.step(record)
            if sched.running and not sched.pending and i < len(reqs):
                nxt = t0 + reqs[i].arrival
                if nxt - time.perf_counter() > 2e-4:
                    time.sleep(5e-5)
            elif not sched.running and i < len(reqs) and realtime:
                wait = t0 + reqs[i].arrival - time.perf_counter()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        wall = time.perf_counter() - t0
        torch.cuda.synchronize(self.ex.dev)
        out = summarize(comps, wall, sched)
        out["overtakes"] = sched.overtakes
        if self.ex.spans:
            busy = self.ex.busy_ms(ref)
            out["device_busy_ms"] = busy
            out["device_busy_frac"] = busy / (wall * 1e3)
        return out


def summarize(comps, wall: float, sched: Optional[Scheduler] = None) -> dict:
    lat = np.array([c.latency for c in comps]) if comps else np.zeros(1)
    pairs = sum(c.pairs for c in comps)
    out = {
        "queries": len(comps),
        "wall_s": wall,
        "pairs": pairs,
        "pairs_per_s": pairs / wall if wall > 0 else float("nan"),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "max_ms": float(lat.max() * 1e3),
    }
    if sched is not None:
        out["max_concurrent"] = sched.max_running
        out["arena_peak_bytes"] = sched.arena.peak
    return out
