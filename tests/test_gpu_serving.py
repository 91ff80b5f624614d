"""GPU tests of the continuous-batching server: every query's result is the
same, bit for bit, whether it runs alone or overlapped with others, and it
matches the oracle on that query's submatrix."""

import numpy as np
import pytest

import synth
from oracle import oracle as orc
from parity_util import assert_counts_equal, assert_p_close, assert_r_close

pytestmark = pytest.mark.gpu


def _requests(S, F, count, seed):
    from paper_2505_00448_amd.serve import Request
    qs = synth.serving_queries(count, S, F, rate=2000.0, seed=seed, vmin=2, vmax=F)
    reqs = [Request(i, q.method, q.rows, q.cols, q.arrival_s) for i, q in enumerate(qs)]
    rng = np.random.default_rng(seed + 1)
    k = len(reqs)
    few = np.sort(rng.choice(S, size=3, replace=False)).astype(np.int32)
    one_col = np.array([int(rng.integers(F))], dtype=np.int32)
    two_col = rng.choice(F, size=2, replace=False).astype(np.int32)
    empty = np.zeros(0, dtype=np.int32)
    every = np.arange(S, dtype=np.int32)
    for j, (m, rows, cols) in enumerate([
            ("pearson", few, two_col), ("spearman", few, two_col),
            ("pearson", every, one_col), ("spearman", every, one_col),
            ("pearson", empty, two_col), ("spearman", empty, two_col),
            ("spearman", every, np.arange(F, dtype=np.int32)[::-1].copy())]):
        reqs.append(Request(k + j, m, rows, cols, reqs[-1].arrival + 1e-4 * (j + 1)))
    return reqs


def _grab(store):
    def cb(c):
        store[c.qid] = {k: v.detach().cpu().numpy().copy() for k, v in c.outputs.items()}
    return cb


def _bits(a):
    return a.view(np.int64) if a.dtype == np.float64 else a


def test_serving_alone_vs_mix_bit_identical(gpu_device):
    import torch
    from paper_2505_00448_amd.serve import Server
    S, F = 3000, 240
    X = synth.cfg_serving_base(S=S, F=F)
    Xd = torch.from_numpy(X).to(gpu_device)
    reqs = _requests(S, F, 30, seed=101)
    print(f"[serving] {len(reqs)} queries on a {S}x{F} base", flush=True)

    alone = {}
    srv1 = Server(Xd, slots=1, capacity=512 << 20)
    for q in reqs:
        srv1.serve([q], on_done=_grab(alone), realtime=False)
    big = max(srv1.ex.nbytes(q) for q in reqs)

    # 4 slots but an arena of ~2.5 of the largest query: admission is bound by
    # slots for small queries and by memory for large ones
    mix = {}
    srv = Server(Xd, slots=4, capacity=int(2.5 * big))
    stats = srv.serve(reqs, on_done=_grab(mix), realtime=False)
    assert stats["queries"] == len(reqs)
    assert stats["max_concurrent"] >= 2, stats
    assert stats["arena_peak_bytes"] <= int(2.5 * big)
    for q in reqs:
        for k in ("r", "p", "n"):
            a, b = alone[q.qid][k], mix[q.qid][k]
            assert a.shape == (len(q.cols), len(q.cols))
            assert np.array_equal(_bits(a), _bits(b)), (q.qid, q.method, k)

    # oracle on a seeded sample of the queries (and every edge query)
    rng = np.random.default_rng(5)
    pick = set(rng.choice(30, size=6, replace=False).tolist()) | set(range(30, len(reqs)))
    for q in reqs:
        if q.qid not in pick:
            continue
        sub = X[np.ix_(q.rows, q.cols)]
        if q.method == "pearson":
            ro, po, no = orc.pearson(sub)
            tol = 1e-6
        else:
            ro, po, no = orc.spearman(sub)
            tol = 1e-12
        got = mix[q.qid]
        where = f"query {q.qid} ({q.method}, {len(q.rows)}x{len(q.cols)})"
        assert_counts_equal(got["n"], no, where)
        worst = assert_r_close(got["r"], ro, tol, where)
        assert_p_close(got["p"], po, ro, no, max(worst, 1e-15), where)


def test_serving_large_base_alone_vs_mix(gpu_device):
    """A 20,000 x 500 resident base (30% MCAR) and queries of up to 18,000
    rows and all 500 variables: each result bit-identical alone and in the
    mix; two small queries also against the oracle."""
    import torch
    from paper_2505_00448_amd.serve import Request, Server
    S, F = 20000, 500
    X = synth.cfg_serving_base(S=S, F=F)
    Xd = torch.from_numpy(X).to(gpu_device)
    rng = np.random.default_rng(2024)
    reqs = []
    for i in range(12):
        nr = int(rng.integers(1000, 18001)) if i < 10 else int(rng.integers(200, 2001))
        nc = int(rng.integers(50, F + 1)) if i < 10 else int(rng.integers(5, 40))
        rows = np.sort(rng.choice(S, size=nr, replace=False)).astype(np.int32)
        cols = rng.choice(F, size=nc, replace=False).astype(np.int32)
        reqs.append(Request(i, "spearman" if i % 2 else "pearson", rows, cols, 1e-4 * i))
    print(f"[serving] large base: {len(reqs)} queries", flush=True)
    alone = {}
    srv1 = Server(Xd, slots=1, capacity=2 << 30)
    for q in reqs:
        srv1.serve([q], on_done=_grab(alone), realtime=False)
    big = max(srv1.ex.nbytes(q) for q in reqs)
    mix = {}
    srv = Server(Xd, slots=4, capacity=int(2.5 * big))
    stats = srv.serve(reqs, on_done=_grab(mix), realtime=False)
    assert stats["queries"] == len(reqs) and stats["max_concurrent"] >= 2, stats
    for q in reqs:
        for k in ("r", "p", "n"):
            assert np.array_equal(_bits(alone[q.qid][k]), _bits(mix[q.qid][k])), (q.qid, q.method, k)
    for q in reqs[10:]:
        sub = X[np.ix_(q.rows, q.cols)]
        ro, po, no = (orc.pearson if q.method == "pearson" else orc.spearman)(sub)
        tol = 1e-6 if q.method == "pearson" else 1e-12
        got = mix[q.qid]
        where = f"query {q.qid} ({q.method}, {len(q.rows)}x{len(q.cols)})"
        assert_counts_equal(got["n"], no, where)
        worst = assert_r_close(got["r"], ro, tol, where)
        assert_p_close(got["p"], po, ro, no, max(worst, 1e-15), where)


def test_serving_device_copies_in_callback(gpu_device):
    """A callback that keeps its results as device copies queued on torch's
    current stream (no host wait): the arena memory is reused by later
    queries only after those copies, so every kept result still equals the
    result of the query run alone."""
    import torch
    from paper_2505_00448_amd.serve import Server
    S, F = 3000, 240
    X = synth.cfg_serving_base(S=S, F=F)
    Xd = torch.from_numpy(X).to(gpu_device)
    reqs = _requests(S, F, 24, seed=303)
    alone = {}
    srv1 = Server(Xd, slots=1, capacity=512 << 20)
    for q in reqs:
        srv1.serve([q], on_done=_grab(alone), realtime=False)
    big = max(srv1.ex.nbytes(q) for q in reqs)
    kept = {}

    def keep(c):
        kept[c.qid] = {k: v.clone() for k, v in c.outputs.items()}

    srv = Server(Xd, slots=4, capacity=int(2.5 * big))
    stats = srv.serve(reqs, on_done=keep, realtime=False)
    torch.cuda.synchronize(gpu_device)
    assert stats["queries"] == len(reqs)
    for q in reqs:
        for k in ("r", "p", "n"):
            a = alone[q.qid][k]
            b = kept[q.qid][k].cpu().numpy()
            assert np.array_equal(_bits(a), _bits(b)), (q.qid, q.method, k)


def test_serving_realtime_stream(gpu_device):
    """Real-time replay of a short Poisson stream: every query completes,
    latencies are positive and queries overlap on the device."""
    import torch
    from paper_2505_00448_amd.serve import Server
    S, F = 4000, 400
    X = synth.cfg_serving_base(S=S, F=F)
    Xd = torch.from_numpy(X).to(gpu_device)
    reqs = _requests(S, F, 60, seed=202)[:60]
    srv = Server(Xd, slots=4, capacity=1 << 30)
    seen = []
    stats = srv.serve(reqs, on_done=lambda c: seen.append((c.qid, c.latency, c.admitted - c.arrival)))
    print(f"[serving] {stats}", flush=True)
    assert sorted(q for q, _, _ in seen) == list(range(60))
    assert all(lat > 0 and wait >= 0 for _, lat, wait in seen)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    assert 0 < stats["device_busy_frac"] <= 1.0 + 1e-6


def test_serving_rejects_bad_queries(gpu_device):
    import torch
    from paper_2505_00448_amd.serve import Request, Server
    X = synth.cfg_serving_base(S=500, F=40)
    srv = Server(torch.from_numpy(X).to(gpu_device), slots=2, capacity=64 << 20)
    ok_rows = np.arange(10, dtype=np.int32)
    bad = [
        Request(0, "pearson", np.array([3, 2], dtype=np.int32), np.arange(3, dtype=np.int32)),
        Request(1, "pearson", np.array([0, 500], dtype=np.int32), np.arange(3, dtype=np.int32)),
        Request(2, "spearman", ok_rows, np.array([1, 1], dtype=np.int32)),
        Request(3, "spearman", ok_rows, np.array([40], dtype=np.int32)),
        Request(4, "kendall", ok_rows, np.arange(3, dtype=np.int32)),
        Request(5, "pearson", ok_rows.astype(np.int64), np.arange(3, dtype=np.int32)),
    ]
    for q in bad:
        with pytest.raises(ValueError):
            srv.serve([q], realtime=False)
