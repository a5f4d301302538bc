"""CPU tests of the serving loop's scheduling core with the fake executor
(simulated work durations; no GPU): FIFO admission, admission by device
footprint, queue-full and over-budget errors, cancellation of queued and
running requests, and an injected executor failure that fails one request
while the others complete."""
import os
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_06340_amd", "libhsd_testhooks.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd_testhooks.so not built")

from hsd_inputs import icosphere  # noqa: E402


def _mesh(level, scale=1.0):
    v, f = icosphere(level)
    return v * scale, f


def _expected(v1, v2=None):
    e = float(np.sum(np.asarray(v1) ** 2))
    if v2 is not None:
        e -= float(np.sum(np.asarray(v2) ** 2))
    return e


def test_all_requests_complete_with_their_own_results():
    import paper_2304_06340_amd as hsd
    with hsd.Server.fake(slots=3, pairs_per_s=5e8) as srv:
        reqs = []
        for i in range(12):
            v, f = _mesh(i % 3, 1.0 + 0.01 * i)
            if i % 4 == 3:
                v2, f2 = _mesh(1, 0.9)
                reqs.append((srv.submit(v, f, verts2=v2, tris2=f2, tag=i), _expected(v, v2)))
            else:
                reqs.append((srv.submit(v, f, tag=i), _expected(v)))
        for tk, exp in reqs:
            t = srv.wait(tk, 30.0)
            assert t.status == 0
            assert t.result.d2 == pytest.approx(exp, rel=1e-14)
            assert t.arrival_s <= t.admitted_s <= t.finished_s
            srv.release(tk)


def test_admission_respects_footprint_budget_and_fifo():
    import paper_2304_06340_amd as hsd
    v, f = _mesh(2)
    foot = len(f) * 80 + v.size * 8 + 1024   # the fake executor's footprint formula
    # budget for exactly one request at a time, even with 4 slots
    with hsd.Server.fake(slots=4, budget_bytes=int(foot * 1.5), pairs_per_s=2e7,
                         chunk_pairs=100_000) as srv:
        tks = [srv.submit(v, f) for _ in range(4)]
        res = [srv.wait(t, 30.0) for t in tks]
        assert all(r.status == 0 for r in res)
        for a, b in zip(res[:-1], res[1:]):
            assert b.admitted_s >= a.finished_s - 1e-3      # strictly one at a time
            assert b.admitted_s >= a.admitted_s            # FIFO
    with hsd.Server.fake(slots=4, budget_bytes=int(foot * 4.5), pairs_per_s=2e7,
                         chunk_pairs=100_000) as srv:
        tks = [srv.submit(v, f) for _ in range(4)]
        res = [srv.wait(t, 30.0) for t in tks]
        # all four admitted before the first finished: their work overlaps
        assert max(r.admitted_s for r in res) < min(r.finished_s for r in res)


def test_queue_full_and_over_budget():
    import paper_2304_06340_amd as hsd
    v, f = _mesh(1)
    with hsd.Server.fake(slots=1, queue_capacity=2, pairs_per_s=1e6, chunk_pairs=10_000) as srv:
        tks = [srv.submit(v, f)]
        time.sleep(0.05)                 # first one admitted, queue empty
        tks += [srv.submit(v, f), srv.submit(v, f)]
        with pytest.raises(hsd.HsdError) as e:
            srv.submit(v, f)
        assert e.value.status == -4      # EAGAIN
        for t in tks:
            srv.cancel(t)
    big_v, big_f = _mesh(4)
    with hsd.Server.fake(slots=1, budget_bytes=10_000) as srv:
        with pytest.raises(hsd.HsdError) as e:
            srv.submit(big_v, big_f)
        assert e.value.status == -2      # ENOMEM: can never be admitted


def test_cancel_queued_and_running_and_bad_input():
    import paper_2304_06340_amd as hsd
    v, f = _mesh(2)
    with hsd.Server.fake(slots=1, pairs_per_s=1e6, chunk_pairs=20_000) as srv:
        running = srv.submit(v, f)
        queued = srv.submit(v, f)
        time.sleep(0.05)
        srv.cancel(queued)
        srv.cancel(running)
        assert srv.wait(queued, 10.0).status == -5
        assert srv.wait(running, 10.0).status == -5
        with pytest.raises(hsd.HsdError) as e:
            srv.submit(v, np.array([[0, 1, len(v)]]))
        assert e.value.status == -1
        bad = v.copy()
        bad[0, 0] = np.inf
        with pytest.raises(hsd.HsdError):
            srv.submit(bad, f)
        with pytest.raises(hsd.HsdError) as e:
            srv.poll(123456)
        assert e.value.status == -6


def test_injected_failure_fails_only_that_request():
    import paper_2304_06340_amd as hsd
    v, f = _mesh(1)
    with hsd.Server.fake(slots=2, pairs_per_s=1e8) as srv:
        ok1 = srv.submit(v, f)
        bad = srv.submit(v, f, tag=-13)
        ok2 = srv.submit(v, f)
        assert srv.wait(bad, 10.0).status == -3
        assert srv.wait(ok1, 10.0).status == 0
        assert srv.wait(ok2, 10.0).status == 0
