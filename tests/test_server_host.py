"""Host-only tests of the serving loop's admission and completion logic
(dry-run mode: no device work, outputs untouched)."""
import threading
import time

import pytest

import paper_2603_03935_amd as disc

FAKE = 1 << 20


def req(m=10, h=480, w=640, patch=16, c=1024, dtype=disc.DISC_BF16, e=768):
    gh, gw = -(-h // patch), -(-w // patch)
    t = disc.Tokens(FAKE, dtype, gh, gw, c, patch, FAKE if dtype == disc.DISC_F8E4M3 else None)
    mk = disc.Masks(FAKE, m, h, w)
    o = disc.Out(FAKE, m, e, None, None)
    return t, mk, o


@pytest.fixture(scope="module", autouse=True)
def lib():
    disc.load()


def make(**kw):
    base = dict(dry_run=1, lanes=2, max_frames=4, max_masks=200, mem_budget=8 << 30)
    base.update(kw)
    return disc.Server(**base)


def test_all_requests_complete_in_order():
    with make() as s:
        tickets = [s.submit(*req(m=5 + i)) for i in range(40)]
        s.drain()
        for t in tickets:
            done, res = s.poll(t)
            assert done and res == 0
        st = s.stats()
        assert st["submitted"] == 40 and st["completed"] == 40 and st["failed"] == 0 and st["rejected"] == 0
        assert st["lanes"] == 2 and st["batches"] >= 10  # at most 4 frames per batch


def test_slot_limit_serialises():
    with make(max_slots=1, lanes=3, dry_run=200) as s:
        for _ in range(12):
            s.submit(*req())
        s.drain()
        st = s.stats()
        assert st["completed"] == 12 and st["batches"] == 12 and st["mean_batch_frames"] == 1.0


def test_continuous_batching_packs_waiting_requests():
    """While one batch runs, arrivals queue up and the next free lane takes
    them together (up to the frame capacity)."""
    with make(lanes=1, max_frames=8, dry_run=20000) as s:
        first = s.submit(*req())
        time.sleep(0.005)
        rest = [s.submit(*req()) for _ in range(8)]
        s.drain()
        st = s.stats()
        assert st["completed"] == 9
        assert st["batches"] == 2, st  # [first], [the 8 that arrived meanwhile]


def test_capacity_rejections():
    with make() as s:
        for kw in (dict(m=201), dict(h=721, w=640), dict(w=1300, h=480), dict(patch=8), dict(c=768),
                   dict(dtype=disc.DISC_F32)):
            with pytest.raises(disc.DiscError) as ei:
                s.submit(*req(**kw))
            assert ei.value.status == 7, kw  # DISC_ERR_ADMISSION
        assert s.stats()["rejected"] == 6


def test_malformed_request_is_rejected_before_queueing():
    with make() as s:
        t, m, o = req()
        t.gh = 29  # grid does not cover the frame
        with pytest.raises(disc.DiscError) as ei:
            s.submit(t, m, o)
        assert ei.value.status == 2
        t, m, o = req()
        o.m = 3
        with pytest.raises(disc.DiscError) as ei:
            s.submit(t, m, o)
        assert ei.value.status == 2
        st = s.stats()
        assert st["submitted"] == 0


def test_memory_budget():
    with pytest.raises(disc.DiscError) as ei:
        make(mem_budget=1)
    assert ei.value.status == 5  # DISC_ERR_OUT_OF_MEMORY
    with make(mem_budget=8 << 30, lanes=1) as s1:
        per_lane = s1.stats()["lane_workspace_bytes"]
    with make(mem_budget=int(per_lane * 2.5), lanes=8) as s:
        assert s.stats()["lanes"] == 2


def test_fault_injection_fails_only_that_batch():
    with make(lanes=1, max_frames=1, fault_batch=2) as s:
        tickets = [s.submit(*req()) for _ in range(5)]
        s.drain()
        results = [s.poll(t)[1] for t in tickets]
        assert results == [0, 0, 6, 0, 0]
        st = s.stats()
        assert st["completed"] == 4 and st["failed"] == 1


def test_admission_timeout():
    with make(lanes=1, max_frames=1, dry_run=30000, admission_timeout_ms=10.0) as s:
        tickets = [s.submit(*req()) for _ in range(3)]
        s.drain()
        results = [s.poll(t)[1] for t in tickets]
        assert results[0] == 0 and results[1:] == [7, 7]


def test_concurrent_submitters_and_wait():
    with make(lanes=3, dry_run=300) as s:
        got = []
        lock = threading.Lock()

        def producer(k):
            for _ in range(25):
                t = s.submit(*req(m=1 + k))
                with lock:
                    got.append(t)

        th = [threading.Thread(target=producer, args=(k,)) for k in range(8)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for t in got:
            assert s.wait(t) == 0
        st = s.stats()
        assert st["completed"] == 200 and len(set(got)) == 200
        assert st["p99_ms"] >= st["p50_ms"] >= 0.0


def test_zero_mask_request_completes_immediately():
    with make() as s:
        t = s.submit(*req(m=0))
        assert s.poll(t) == (True, 0)


def test_reported_tickets_are_forgotten_and_stats_reset():
    """A ticket whose completion was reported is dropped (the server does not
    grow with the requests served); reset_stats restarts counts and latency
    samples, so a warm-up can be left out of p50/p99."""
    with make(lanes=1, dry_run=2000) as s:
        warm = [s.submit(*req()) for _ in range(3)]
        for t in warm:
            assert s.wait(t) == 0
        with pytest.raises(disc.DiscError):
            s.poll(warm[0])
        s.reset_stats()
        st = s.stats()
        assert st["submitted"] == 0 and st["completed"] == 0 and st["p99_ms"] == 0.0
        tickets = [s.submit(*req()) for _ in range(5)]
        s.drain()
        assert all(s.poll(t) == (True, 0) for t in tickets)
        st = s.stats()
        assert st["submitted"] == 5 and st["completed"] == 5 and st["p50_ms"] > 0.0
