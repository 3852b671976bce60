"""Serving loop: admission control (CPU) and continuous batching (GPU).

GPU bar: every request's covering, kept flags, masks and query answers are
bit-identical when served in the mix (concurrent slots, overlapping on the
device) and when served alone, and equal the CPU oracle's.
"""
import hashlib
import json
import os
import random
import threading
import time

import numpy as np
import pytest

from conftest import gpu_available
from paper_2202_06111_amd import workloads as W


def test_admission_never_exceeds_budget_and_defers():
    from paper_2202_06111_amd.serve import Admission
    adm = Admission(n_slots=3, budget_bytes=100)
    rng = random.Random(0)
    peak = [0]
    lock = threading.Lock()
    live = [0]

    def job(need):
        slot = adm.admit(need)
        with lock:
            live[0] += 1
            peak[0] = max(peak[0], live[0])
            assert adm.in_use <= 100
        time.sleep(rng.random() * 0.003)
        with lock:
            live[0] -= 1
        adm.release(slot, need)

    threads = [threading.Thread(target=job, args=(rng.randint(10, 60),)) for _ in range(60)]
    # one request larger than the whole budget: admitted alone, never rejected
    threads.append(threading.Thread(target=job, args=(1000,)))
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert adm.max_in_use <= 100 and adm.in_use == 0
    assert peak[0] <= 3
    assert adm.deferred > 0


def test_memory_estimate_grows_with_grid():
    from paper_2202_06111_amd.serve import estimate_bytes
    reqs = W.serving_stream(40, 10.0, seed=3, n_queries=4)
    by_side = {}
    for r in reqs:
        by_side[r.workload.grid.n0[0]] = estimate_bytes(r.workload)
    sides = sorted(by_side)
    assert all(by_side[a] < by_side[b] for a, b in zip(sides, sides[1:]))


def _digests():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "digests_fullsize.json")
    with open(path) as f:
        return json.load(f)["serving_stream"]


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")
def test_results_identical_alone_and_in_the_mix():
    """The seeded test stream (24 requests, grids 32^2 .. 256^2, 4000 queries
    each): every request's covering, kept flags, masks and query answers are
    identical when served in the mix (4 slots, batches overlapping on the
    device) and alone, and equal the CPU oracle's (digests written by
    tests/golden/make_digests.py from oracle/ only)."""
    from paper_2202_06111_amd import serve
    want = _digests()
    st = want["stream"]
    reqs = W.serving_stream(st["n_requests"], st["rate_per_s"], seed=st["seed"],
                            n_queries=st["n_queries"])
    assert 256 in {r.workload.grid.n0[0] for r in reqs}
    srv = serve.Server(n_slots=4, mem_budget_bytes=1 << 34, export_results=True)
    try:
        mix = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    alone = serve.serve_alone(reqs, export_results=True)
    # overlap really happened: some request started before an earlier one finished
    res = sorted(mix["results"], key=lambda r: r.start_s)
    assert any(b.start_s < a.done_s for a, b in zip(res, res[1:]))
    assert max(r.slot for r in mix["results"]) > 0
    by_rid = {w["rid"]: w for w in want["requests"]}
    for a, b in zip(sorted(mix["results"], key=lambda r: r.rid), alone):
        assert a.rid == b.rid and a.n_cells == b.n_cells and a.n_kept == b.n_kept
        for x, y in zip(a.export, b.export):
            np.testing.assert_array_equal(x, y, err_msg=f"request {a.rid}")
        np.testing.assert_array_equal(a.member, b.member)
        np.testing.assert_array_equal(a.admissible, b.admissible)
        w = by_rid[a.rid]
        lv, ix, kept, mask = b.export
        an = reqs[a.rid].workload.analysis
        assert (lv.shape[0], int(kept.sum())) == (w["covering"]["n_cells"], w[an]["n_kept"])
        assert _sha(lv) == w["covering"]["level"] and _sha(ix) == w["covering"]["idx"]
        assert _sha(kept) == w[an]["kept"] and _sha(mask) == w[an]["mask"], a.rid
        assert _sha(b.member) == w["member"] and _sha(b.admissible) == w["admissible"], a.rid


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")
def test_low_budget_defers_without_failing():
    from paper_2202_06111_amd import serve
    reqs = W.serving_stream(6, 1e6, seed=12, n_queries=100, sides=(32,))
    srv = serve.Server(n_slots=4, mem_budget_bytes=1)
    try:
        out = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    assert out["deferred"] > 0 and out["max_bytes_in_use"] <= 1
    assert len(out["results"]) == 6
