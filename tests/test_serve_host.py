"""Host logic of the continuous-batching server (no GPU): the arena
allocator and the admission scheduler, driven by a fake executor whose
queries finish when the test says so."""

import numpy as np
import pytest

from paper_2505_00448_amd.serve import Arena, Request, Scheduler, summarize


def test_arena_first_fit_merge_and_double_release():
    a = Arena(4096)
    x = a.alloc(1000)      # rounds to 1024
    y = a.alloc(256)
    z = a.alloc(2000)      # rounds to 2048
    assert (x, y, z) == (0, 1024, 1280)
    assert a.alloc(1024) is None           # 768 left
    a.release(y, 256)                      # hole of 256 at 1024, tail of 768 at 3328
    w = a.alloc(300)                       # rounds to 512: only the tail fits
    assert w == 3328
    v = a.alloc(200)                       # first fit: the hole
    assert v == 1024
    a.release(v, 200)
    a.release(x, 1000)
    a.release(z, 2000)                     # merges 0..3328 into one range
    assert a.alloc(3328) == 0
    a.release(w, 300)
    with pytest.raises(ValueError):
        a.release(w, 300)
    assert a.used == 3328


def test_arena_random_stress_never_overlaps():
    rng = np.random.default_rng(7)
    a = Arena(1 << 20)
    live = {}
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            a.release(off, live.pop(off))
        else:
            nb = int(rng.integers(1, 40000))
            off = a.alloc(nb)
            if off is not None:
                live[off] = nb
        iv = sorted((o, o + (nb + 255) // 256 * 256) for o, nb in live.items())
        assert all(iv[i][1] <= iv[i + 1][0] for i in range(len(iv) - 1))
        assert all(0 <= lo and hi <= a.capacity for lo, hi in iv)
        assert a.used + a.free_bytes() == a.capacity
    for off, nb in list(live.items()):
        a.release(off, nb)
    assert a._free == [(0, a.capacity)]


class FakeExecutor:
    def __init__(self, sizes):
        self.sizes = sizes
        self.launched = []
        self.finished = set()
        self.slot_q = {}

    def nbytes(self, req):
        return self.sizes[req.qid]

    def launch(self, req, slot, off):
        self.launched.append((req.qid, slot, off))
        self.slot_q[slot] = req.qid

    def is_done(self, slot):
        return self.slot_q[slot] in self.finished

    def outputs(self, req, slot, off):
        return {"qid": req.qid}


def _req(i):
    return Request(i, "pearson", np.arange(4, dtype=np.int32), np.arange(3, dtype=np.int32), float(i))


def test_scheduler_admits_by_slots_and_memory_in_order():
    sizes = {0: 3000, 1: 3000, 2: 5000, 3: 100, 4: 100}
    ex = FakeExecutor(sizes)
    t = [0.0]
    sch = Scheduler(ex, slots=2, capacity=8192, clock=lambda: t[0], max_overtakes=0)
    for i in range(5):
        sch.submit(_req(i))
    sch.step()
    assert [q for q, _, _ in ex.launched] == [0, 1]        # two slots
    ex.finished.add(0)
    done = []
    sch.step(done.append)
    assert [c.qid for c in done] == [0]
    # query 2 (5000 B) does not fit beside query 1 (3072 B) in 8192 B:
    # it waits, and with overtaking switched off the small queries behind it
    # wait too
    assert [q for q, _, _ in ex.launched] == [0, 1]
    ex.finished.add(1)
    sch.step(done.append)
    assert [q for q, _, _ in ex.launched] == [0, 1, 2, 3]
    assert sch.max_running == 2
    ex.finished.update({2, 3})
    sch.step(done.append)
    assert [q for q, _, _ in ex.launched][-1] == 4
    ex.finished.add(4)
    sch.step(done.append)
    assert sch.idle()
    assert sorted(c.qid for c in done) == [0, 1, 2, 3, 4]
    assert sch.arena.used == 0


def test_scheduler_bounded_overtaking():
    """When the head's memory does not fit, younger queries that fit go
    ahead of it, at most max_overtakes times; then the head is admitted
    first as soon as its memory frees up."""
    sizes = {0: 6000, 1: 6000, 2: 100, 3: 100, 4: 100, 5: 100}
    ex = FakeExecutor(sizes)
    sch = Scheduler(ex, slots=4, capacity=8192, max_overtakes=2)
    for i in range(6):
        sch.submit(_req(i))
    sch.step()
    # 0 runs; 1 does not fit beside it; 2 and 3 overtake it (the bound)
    assert [q for q, _, _ in ex.launched] == [0, 2, 3]
    assert sch.overtakes == 2
    ex.finished.update({2, 3})
    done = []
    sch.step(done.append)
    # slots are free but 1 still does not fit and may not be overtaken again
    assert [q for q, _, _ in ex.launched] == [0, 2, 3]
    ex.finished.add(0)
    sch.step(done.append)
    # 1 first, then the rest in order (they fit beside it)
    assert [q for q, _, _ in ex.launched] == [0, 2, 3, 1, 4, 5]
    ex.finished.update({1, 4, 5})
    sch.step(done.append)
    assert sch.idle() and sch.arena.used == 0


def test_scheduler_calls_released_after_callback():
    ex = FakeExecutor({0: 100})
    order = []
    ex.released = lambda: order.append("released")
    sch = Scheduler(ex, slots=1, capacity=1 << 20)
    sch.submit(_req(0))
    sch.step()
    ex.finished.add(0)
    sch.step(lambda c: order.append("callback"))
    assert order == ["callback", "released"]


def test_scheduler_admits_while_others_run():
    """A query that arrives while another runs starts before that one ends."""
    ex = FakeExecutor({0: 100, 1: 100})
    sch = Scheduler(ex, slots=2, capacity=1 << 20)
    sch.submit(_req(0))
    sch.step()
    sch.submit(_req(1))
    sch.step()
    assert [q for q, _, _ in ex.launched] == [0, 1]
    assert not ex.finished and len(sch.running) == 2


def test_scheduler_rejects_oversized_query():
    ex = FakeExecutor({0: 1 << 30})
    sch = Scheduler(ex, slots=1, capacity=1 << 20)
    with pytest.raises(ValueError):
        sch.submit(_req(0))


def test_summarize_percentiles():
    from paper_2505_00448_amd.serve import Completion
    comps = [Completion(i, "pearson", 10, 5, 0.0, 0.0, (i + 1) * 1e-3, 0) for i in range(100)]
    s = summarize(comps, 1.0)
    assert s["queries"] == 100 and s["pairs"] == 1000
    assert abs(s["p50_ms"] - 50.5) < 1e-9 and abs(s["p99_ms"] - 99.01) < 1e-9
