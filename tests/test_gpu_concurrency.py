"""Concurrent calls: napy_pearson and napy_spearman issued from two host
threads, each on its own stream with its own workspace, return exactly what
the same calls return one after the other.  The library holds no state
shared between calls (a kernel's dynamic-LDS attribute is set once per
device under an atomic flag), and every kernel is deterministic, so the
comparison is bit for bit."""

import threading

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_pearson_and_spearman_on_two_streams(gpu_device):
    import torch

    import paper_2505_00448_amd as napy

    # a scaled-down headline matrix: factor model, integer columns, MCAR and
    # one block of columns missing on a shared half of the samples
    X = synth.cfg_gpu_headline(S=3000, F=160)
    Xd = torch.from_numpy(X).to(gpu_device)
    print(f"concurrency: S={X.shape[0]} F={X.shape[1]}", flush=True)

    ref_p = napy.pearson(Xd, precision="bf16x3")
    ref_s = napy.spearman(Xd)
    torch.cuda.synchronize(gpu_device)

    rounds = 3
    got = {"pearson": [], "spearman": []}
    errors = []

    def worker(kind):
        try:
            st = torch.cuda.Stream(gpu_device)  # default priority
            with torch.cuda.stream(st):
                for _ in range(rounds):
                    if kind == "pearson":
                        out = napy.pearson(Xd, precision="bf16x3")
                    else:
                        out = napy.spearman(Xd)
                    got[kind].append(out)
            st.synchronize()
        except Exception as e:  # reported in the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(k,)) for k in ("pearson", "spearman")]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a worker did not finish"
    assert not errors, errors
    torch.cuda.synchronize(gpu_device)

    for kind, ref in (("pearson", ref_p), ("spearman", ref_s)):
        assert len(got[kind]) == rounds
        for out in got[kind]:
            for key in ref:
                a = ref[key].cpu().numpy()
                b = out[key].cpu().numpy()
                assert np.array_equal(a, b, equal_nan=True), (kind, key)
