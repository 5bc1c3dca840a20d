"""Host logic of the labelling server, on its simulated device (no GPU).

The scheduler, arena and admission code are the ones the GPU server runs;
only batch execution is replaced by a timer (fixed_ns + ns_per_site * sites).
"""
from __future__ import annotations

import time

import pytest

from paper_1405_1931_amd import _lib
from paper_1405_1931_amd.serve import Server

MS = 1_000_000  # ns


def test_all_requests_complete_in_batches_and_free_their_memory():
    shapes = [(8 + i % 5, 16 + i % 7, 30 + i % 11) for i in range(60)]
    with Server(1 << 30, slots=2, max_batch=16, simulate=(2 * MS, 0.0)) as s:
        tickets = [s.submit_shape(sh, periodic=i % 8) for i, sh in enumerate(shapes)]
        s.drain(30)
        st = s.stats()
        assert st["submitted"] == 60 and st["completed"] == 60 and st["failed"] == 0
        assert st["pending"] == 0 and st["running"] == 0
        assert st["batches"] < 60, "requests waiting together must share a batch"
        assert st["latency_samples"] == 60
        assert 0 < st["latency_p50_ns"] <= st["latency_p99_ns"] <= st["latency_max_ns"]
        assert st["sites_completed"] == sum(a * b * c for a, b, c in shapes)
        # outputs stay resident until released, then the arena is empty again
        assert st["arena_in_use"] > 0
        for t in tickets:
            labels, k, sizes, lat = s.result(t)
            assert k == 0 and lat > 0
            s.release(t)
        assert s.stats()["arena_in_use"] == 0
        assert s.stats()["arena_peak"] <= s.stats()["arena_bytes"]


def test_admission_by_footprint_bounds_arena_use():
    shape = (40, 40, 40)
    with Server(1 << 30, simulate=(0, 0.0)) as probe:
        fp = probe.footprint(shape)
    arena = int(2.5 * fp)  # room for two requests at a time, not three
    with Server(arena, slots=4, max_batch=64, simulate=(3 * MS, 0.0)) as s:
        tickets = []
        for _ in range(10):
            t = s.submit_shape(shape)
            tickets.append(t)
        # finished requests keep their outputs: release them as they complete
        done = set()
        deadline = time.time() + 30
        while len(done) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in done and s.poll(t):
                    s.release(t)
                    done.add(t)
            time.sleep(0.0005)
        st = s.stats()
        assert st["completed"] == 10
        assert st["arena_peak"] <= arena
        assert st["mean_batch_jobs"] <= 2.0
        assert st["arena_in_use"] == 0


def test_request_larger_than_the_arena_is_refused():
    with Server(1 << 20, simulate=(0, 0.0)) as s:
        with pytest.raises(_lib.HkError) as e:
            s.submit_shape((64, 64, 64))
        assert e.value.status == _lib.HK_ERR_TOO_LARGE
        assert s.stats()["submitted"] == 0


def test_arrivals_during_a_run_join_the_next_batch():
    """Continuous batching: with one slot busy, requests that arrive wait and
    then go out together as soon as the slot frees."""
    with Server(1 << 30, slots=1, max_batch=64, simulate=(40 * MS, 0.0)) as s:
        a = s.submit_shape((16, 16, 16))
        time.sleep(0.008)
        assert not s.poll(a)
        late = [s.submit_shape((16, 16, 16 + i)) for i in range(5)]
        assert s.stats()["running"] == 1 and s.stats()["pending"] == 5
        s.drain(30)
        st = s.stats()
        assert st["batches"] == 2
        assert st["completed"] == 6
        lat_a = s.result(a)[3]
        for t in late:
            assert s.result(t)[3] > 40 * MS  # waited for the slot, then ran
        assert lat_a >= 40 * MS


def test_max_batch_caps_each_batch():
    with Server(1 << 30, slots=1, max_batch=3, simulate=(5 * MS, 0.0)) as s:
        for i in range(10):
            s.submit_shape((8, 8, 8 + i))
        s.drain(30)
        st = s.stats()
        assert st["completed"] == 10
        assert st["batches"] >= 4
        assert st["mean_batch_jobs"] <= 3.0


def test_waiting_request_can_be_withdrawn_running_one_cannot():
    with Server(1 << 30, slots=1, max_batch=1, simulate=(50 * MS, 0.0)) as s:
        a = s.submit_shape((8, 8, 8))
        time.sleep(0.005)
        b = s.submit_shape((8, 8, 8))
        with pytest.raises(_lib.HkError):
            s.release(a)  # running
        s.release(b)  # waiting: withdrawn
        with pytest.raises(_lib.HkError):
            s.poll(b)
        s.wait(a, 30)
        s.release(a)
        st = s.stats()
        assert st["completed"] == 1 and st["arena_in_use"] == 0


def test_wait_times_out_and_latency_counts_from_arrival():
    with Server(1 << 30, slots=1, max_batch=8, simulate=(30 * MS, 0.0)) as s:
        t0 = s.now_ns()
        t = s.submit_shape((8, 8, 8), arrival_ns=t0 - 10 * MS)  # arrived 10 ms before submission
        with pytest.raises(_lib.HkError) as e:
            s.wait(t, 0.001)
        assert e.value.status == _lib.HK_ERR_TIMEOUT
        s.wait(t, 30)
        assert s.result(t)[3] >= 40 * MS


def test_time_scales_with_sites():
    """The simulated batch time grows with its sites, so a large request
    finishes after a small one submitted at the same time on another slot."""
    with Server(1 << 32, slots=2, max_batch=1, simulate=(1 * MS, 200.0)) as s:
        big = s.submit_shape((64, 64, 64))      # 262144 sites * 200 ns = 52 ms
        small = s.submit_shape((8, 8, 8))       # 0.1 ms
        s.wait(small, 30)
        assert not s.poll(big)
        s.wait(big, 30)
        assert s.result(big)[3] > s.result(small)[3]


def test_invalid_arguments():
    with pytest.raises(_lib.HkError):
        Server(0, simulate=(0, 0.0))
    with pytest.raises(_lib.HkError):
        Server(1 << 20, slots=0, simulate=(0, 0.0))
    with Server(1 << 30, simulate=(0, 0.0)) as s:
        with pytest.raises(_lib.HkError):
            s.submit_shape((0, 4, 4))
        with pytest.raises(ValueError):
            s.submit_shape((4, 4, 4), periodic=9)
        with pytest.raises(_lib.HkError):
            s.poll(12345)


def test_future_arrivals_are_held_until_due():
    """A trace submitted ahead of time is admitted at its arrival times."""
    with Server(1 << 30, slots=2, max_batch=64, simulate=(1 * MS, 0.0)) as s:
        t0 = s.now_ns() + 30 * MS
        ts = [s.submit_shape((8, 8, 8), arrival_ns=t0 + i * 10 * MS) for i in range(4)]
        time.sleep(0.01)
        st = s.stats()
        assert st["running"] == 0 and st["pending"] == 4 and st["batches"] == 0
        s.drain(30)
        st = s.stats()
        assert st["completed"] == 4 and st["batches"] == 4  # 10 ms apart: one batch each
        for t in ts:
            lat = s.result(t)[3]
            assert 1 * MS <= lat < 9 * MS


def _held(s, n, shape=(20, 20, 20), ahead_ns=50 * MS):
    """n requests arriving together ahead of now (so they wait, and a
    failure can be planted on them first); returns the tickets."""
    at = s.now_ns() + ahead_ns
    return [s.submit_shape(shape, arrival_ns=at) for _ in range(n)]


def test_device_check_fails_only_its_own_request():
    """Each request of a batch has its own device-check word: the planted
    check fails that request alone, the others of the same batch complete."""
    with Server(1 << 30, slots=1, max_batch=16, simulate=(1 * MS, 0.0)) as s:
        tickets = _held(s, 8)
        s.sim_fail(tickets[3], _lib.HK_ERR_DEVICE)
        s.drain(30)
        st = s.stats()
        assert st["batches"] == 1, "the eight requests run as one batch"
        assert st["completed"] == 7 and st["failed"] == 1
        for j, t in enumerate(tickets):
            if j == 3:
                with pytest.raises(_lib.HkError) as e:
                    s.result(t)
                assert e.value.status == _lib.HK_ERR_DEVICE
                with pytest.raises(_lib.HkError) as e:
                    s.wait(t, 1.0)
                assert e.value.status == _lib.HK_ERR_DEVICE
                assert s._lib.hk_server_poll(s._h, t) == _lib.HK_ERR_DEVICE
            else:
                assert s.poll(t)
                _, k, _, lat = s.result(t)
                assert k == 0 and lat > 0
            s.release(t)
        assert s.stats()["arena_in_use"] == 0


def test_batch_error_fails_that_batch_and_no_other():
    """An error of a batch itself (as a failed launch or an asynchronous error
    reported by its completion event) fails every request of that batch, and
    the next batch runs normally."""
    with Server(1 << 30, slots=1, max_batch=4, simulate=(1 * MS, 0.0)) as s:
        tickets = _held(s, 8)
        s.sim_fail(tickets[1], _lib.HK_ERR_HIP)
        s.drain(30)
        st = s.stats()
        assert st["batches"] == 2 and st["failed"] == 4 and st["completed"] == 4
        for j, t in enumerate(tickets):
            if j < 4:
                with pytest.raises(_lib.HkError) as e:
                    s.wait(t, 1.0)
                assert e.value.status == _lib.HK_ERR_HIP
            else:
                s.wait(t, 1.0)
            s.release(t)
        # failed requests gave their outputs back when their batch failed
        assert s.stats()["arena_in_use"] == 0


def test_wait_times_out_on_a_held_request_and_reports_a_failure_at_the_deadline():
    with Server(1 << 30, slots=1, max_batch=4, simulate=(0, 0.0)) as s:
        held = s.submit_shape((10, 10, 10), arrival_ns=s.now_ns() + 10_000 * MS)
        with pytest.raises(_lib.HkError) as e:
            s.wait(held, 0.01)
        assert e.value.status == _lib.HK_ERR_TIMEOUT
        s.release(held)  # withdrawn while waiting
        # a failure that lands while the caller waits is reported as the
        # failure, not as a time-out
        t = _held(s, 1, ahead_ns=20 * MS)[0]
        s.sim_fail(t, _lib.HK_ERR_DEVICE)
        with pytest.raises(_lib.HkError) as e:
            s.wait(t, 5.0)
        assert e.value.status == _lib.HK_ERR_DEVICE
        s.release(t)


def test_sim_fail_is_refused_for_unknown_or_started_requests():
    with Server(1 << 30, slots=1, max_batch=4, simulate=(0, 0.0)) as s:
        t = s.submit_shape((8, 8, 8))
        s.drain(10)
        with pytest.raises(_lib.HkError):
            s.sim_fail(t, _lib.HK_ERR_DEVICE)  # already done
        with pytest.raises(_lib.HkError):
            s.sim_fail(12345, _lib.HK_ERR_DEVICE)
        s.release(t)
