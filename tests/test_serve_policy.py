"""Serving policy on the host: the real server thread, admission, batching and
chunking code driven through the C ABI with the simulated backend (virtual
memory, synthetic batch durations), so no GPU is touched."""
import time

import pytest

import paper_1011_3583_amd as rr

MiB = 1 << 20


def _job(dims, perm, esize, src=0x7f0000000000, dst=None):
    return rr.make_jobs([(dst or 0, src, dims, perm, esize)])[0]


def _wait(srv, tickets, timeout=20.0):
    left = set(tickets)
    res = {}
    t0 = time.time()
    while left and time.time() - t0 < timeout:
        for t in srv.completions():
            if t in left:
                res[t] = srv.poll(t)
                left.discard(t)
        time.sleep(0.0005)
    assert not left, f"{len(left)} tickets never completed"
    return res


def test_budget_is_never_exceeded_and_outputs_are_released():
    budget = 64 * MiB
    with rr.Server(budget, max_inflight=3, max_batch_jobs=16, chunk_bytes=0, simulated=True,
                   sim_bytes_per_us=20_000.0) as srv:
        tickets = [srv.submit(0, 0x7f0000000000 + i * 16 * MiB, (1024, 1024), (1, 0), 4)  # 4 MiB outputs
                   for i in range(60)]
        done = []
        t0 = time.time()
        while len(done) < len(tickets) and time.time() - t0 < 20:
            for t in srv.completions():
                r = srv.poll(t)
                assert r.status == 0
                done.append(t)
                srv.release(t)
            st = srv.stats()
            assert st["budget_used"] <= budget
            time.sleep(0.0005)
        assert len(done) == len(tickets)
        st = srv.stats()
        assert st["budget_peak"] <= budget and st["budget_used"] == 0
        assert st["completed"] == 60 and st["batches"] >= 4


def test_large_job_runs_whole_beside_small_jobs():
    """Several slots: a large job is launched whole, alone, and the small jobs'
    batches run beside it (the simulated device shares its bandwidth)."""
    with rr.Server(8 << 30, max_inflight=2, max_batch_jobs=64, chunk_bytes=16 * MiB, simulated=True,
                   sim_bytes_per_us=2_000.0) as srv:
        big = srv.submit(0, 0x7e0000000000, (8192, 8192), (1, 0), 4)           # 256 MiB
        time.sleep(0.002)
        small = [srv.submit(0, 0x7f0000000000 + i * MiB, (64, 64), (1, 0), 4) for i in range(20)]
        res = _wait(srv, [big] + small)
        assert res[big].chunks == 1
        assert all(res[t].chunks == 1 for t in small)
        # every small job finished before the large one
        assert max(res[t].t_done_ns for t in small) < res[big].t_done_ns
        assert all(res[t].status == 0 for t in [big] + small)


def test_large_jobs_leave_a_slot_for_small_ones():
    """Large jobs hold at most max_inflight - 1 slots: with two slots the second
    large job waits for the first, and a small job arriving meanwhile runs."""
    with rr.Server(8 << 30, max_inflight=2, max_batch_jobs=64, chunk_bytes=16 * MiB, simulated=True,
                   sim_bytes_per_us=4_000.0) as srv:
        big = [srv.submit(0, 0x7e0000000000 + i * (1 << 30), (4096, 8192), (1, 0), 4) for i in range(2)]
        time.sleep(0.002)
        small = srv.submit(0, 0x7f0000000000, (64, 64), (1, 0), 4)
        res = _wait(srv, big + [small])
        assert all(r.status == 0 and r.chunks == 1 for r in res.values())
        assert res[small].t_done_ns < res[big[0]].t_done_ns
        assert res[big[1]].t_launch_ns >= res[big[0]].t_done_ns


def test_large_job_is_cut_into_pieces_with_one_slot():
    """One slot: a batch blocks the device, so the large job goes in pieces and
    the small jobs ride in the batches beside them."""
    with rr.Server(8 << 30, max_inflight=1, max_batch_jobs=64, chunk_bytes=16 * MiB, simulated=True,
                   sim_bytes_per_us=2_000.0) as srv:
        big = srv.submit(0, 0x7e0000000000, (8192, 8192), (1, 0), 4)           # 256 MiB
        time.sleep(0.002)
        small = [srv.submit(0, 0x7f0000000000 + i * MiB, (64, 64), (1, 0), 4) for i in range(20)]
        res = _wait(srv, [big] + small)
        assert res[big].chunks >= 3    # pieces grow while it is alone, shrink when the small jobs arrive
        assert all(res[t].chunks == 1 for t in small)
        assert max(res[t].t_done_ns for t in small) < res[big].t_done_ns
        assert all(res[t].status == 0 for t in [big] + small)


def test_failed_batch_fails_its_jobs_and_serving_continues():
    with rr.Server(1 << 30, max_inflight=1, max_batch_jobs=8, chunk_bytes=0, simulated=True,
                   sim_bytes_per_us=50_000.0) as srv:
        srv.fail_next_batch()
        first = [srv.submit(0, 0x7f0000000000 + i * MiB, (128, 128), (1, 0), 4) for i in range(4)]
        res = _wait(srv, first)
        codes = [res[t].status for t in first]
        nfail = codes.count(rr.STATUS_CODE["RR_ERR_HIP"])
        # the batch formed next held the first job(s) submitted; those failed, the rest ran
        assert nfail >= 1 and codes == [rr.STATUS_CODE["RR_ERR_HIP"]] * nfail + [0] * (4 - nfail)
        later = [srv.submit(0, 0x7f0000000000 + i * MiB, (128, 128), (1, 0), 4) for i in range(4)]
        res2 = _wait(srv, later)
        assert all(r.status == 0 for r in res2.values())
        st = srv.stats()
        assert st["failed"] == nfail and st["completed"] == 8 - nfail


def test_submit_errors():
    with rr.Server(16 * MiB, max_inflight=1, max_batch_jobs=4, queue_capacity=3, simulated=True,
                   sim_bytes_per_us=2000.0) as srv:
        st, _ = srv.submit_raw(_job((4096, 4096), (1, 0), 4))          # 64 MiB output > budget
        assert st == rr.STATUS_CODE["RR_ERR_NO_MEMORY"]
        st, _ = srv.submit_raw(_job((4, 4), (0, 0), 4))                 # not a permutation
        assert st == rr.STATUS_CODE["RR_ERR_INVALID_ARG"]
        st, _ = srv.submit_raw(_job((4, 4), (1, 0), 4, src=0x1000, dst=0x1008))
        assert st == rr.STATUS_CODE["RR_ERR_ALIAS"]
        # a very slow device: the queue fills up
        codes = [srv.submit_raw(_job((256, 256), (1, 0), 4, src=0x7f0000000000 + i * MiB))[0]
                 for i in range(40)]
        assert rr.STATUS_CODE["RR_ERR_BUSY"] in codes
        st, t = srv.submit_raw(_job((0, 5), (1, 0), 4))                 # empty job completes at once
        assert st == 0 and srv.poll(t).status == 0


def test_destroy_drains_in_flight_work():
    srv = rr.Server(1 << 30, max_inflight=2, max_batch_jobs=4, chunk_bytes=MiB, simulated=True,
                    sim_bytes_per_us=5_000.0)
    tickets = [srv.submit(0, 0x7f0000000000 + i * 32 * MiB, (2048, 1024), (1, 0), 4) for i in range(6)]
    srv.close()
    assert len(tickets) == 6


def test_resident_allocations_count_against_budget():
    with rr.Server(100 * MiB, simulated=True, sim_bytes_per_us=1e5) as srv:
        a = srv.alloc(60 * MiB)
        with pytest.raises(rr.RRError):
            srv.alloc(60 * MiB)
        srv.free(a)
        b = srv.alloc(60 * MiB)
        assert srv.stats()["budget_used"] == 60 * MiB
        srv.free(b)


def test_direct_mode_launches_one_job_at_a_time():
    with rr.Server(1 << 30, max_inflight=2, max_batch_jobs=64, chunk_bytes=MiB, simulated=True,
                   sim_bytes_per_us=20_000.0, direct=True) as srv:
        tickets = [srv.submit(0, 0x7f0000000000 + i * 16 * MiB, (2048, 1024), (1, 0), 4) for i in range(10)]
        res = _wait(srv, tickets)
        assert all(r.status == 0 and r.chunks == 1 for r in res.values())
        assert srv.stats()["batches"] == 10


def test_device_refusal_within_budget_fails_the_job_and_destroy_returns():
    """The simulated device has 32 MiB although the budget allows 1 GiB: with
    nothing in flight, a job whose output cannot be allocated completes with
    RR_ERR_NO_MEMORY instead of waiting forever, and the server keeps serving
    jobs that fit."""
    srv = rr.Server(1 << 30, max_inflight=2, max_batch_jobs=8, chunk_bytes=0, simulated=True,
                    sim_bytes_per_us=50_000.0, sim_device_bytes=32 * MiB)
    try:
        big = srv.submit(0, 0x7e0000000000, (4096, 4096), (1, 0), 4)          # 64 MiB output
        res = _wait(srv, [big])
        assert res[big].status == rr.STATUS_CODE["RR_ERR_NO_MEMORY"]
        small = srv.submit(0, 0x7f0000000000, (1024, 1024), (1, 0), 4)       # 4 MiB output
        assert _wait(srv, [small])[small].status == 0
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 1 and st["reserved"] <= 32 * MiB
    finally:
        srv.close()   # returns: nothing is left waiting


def test_reserved_memory_stays_within_budget_and_free_slabs_are_given_back():
    """Slabs count against the budget.  Ten 50 MiB outputs fill two 256 MiB slabs;
    once they are released, a 500 MiB job does not fit any slab and the budget has
    no room for a new one until the two empty slabs are given back."""
    budget = 600 * MiB
    with rr.Server(budget, max_inflight=4, max_batch_jobs=16, chunk_bytes=0, simulated=True,
                   sim_bytes_per_us=200_000.0) as srv:
        small = [srv.submit(0, 0x7f0000000000 + i * 64 * MiB, (3200, 4096), (1, 0), 4) for i in range(10)]
        res = _wait(srv, small)
        assert all(r.status == 0 for r in res.values())
        assert srv.stats()["reserved"] <= budget
        for t in small:
            srv.release(t)
        big = srv.submit(0, 0x7e0000000000, (32000, 4096), (1, 0), 4)          # 500 MiB output
        r = _wait(srv, [big])[big]
        assert r.status == 0
        st = srv.stats()
        assert st["reserved"] <= budget and st["budget_peak"] <= budget
        srv.release(big)


def test_destroy_fails_jobs_still_waiting_for_memory():
    """Outputs never released hold the budget: at shutdown the job waiting for
    memory completes with RR_ERR_NO_MEMORY and destroy returns."""
    srv = rr.Server(100 * MiB, max_inflight=1, max_batch_jobs=4, chunk_bytes=0, simulated=True,
                    sim_bytes_per_us=100_000.0)
    first = srv.submit(0, 0x7f0000000000, (3840, 4096), (1, 0), 4)            # 60 MiB, kept
    assert _wait(srv, [first])[first].status == 0
    waiting = srv.submit(0, 0x7e0000000000, (3840, 4096), (1, 0), 4)          # no room while first is held
    time.sleep(0.01)
    assert srv.poll(waiting) is None   # still waiting for memory
    t0 = time.time()
    srv.close()                        # fails it and returns
    assert time.time() - t0 < 5


def test_lone_job_on_idle_server_is_launched_at_submit():
    """With nothing queued and a slot free, the submitting thread admits and
    launches the job itself: its launch time follows its submission directly."""
    with rr.Server(1 << 30, max_inflight=2, max_batch_jobs=8, chunk_bytes=64 * MiB, simulated=True,
                   sim_bytes_per_us=100_000.0, tick_us=1000) as srv:
        time.sleep(0.01)   # the server thread is idle
        t = srv.submit(0, 0x7f0000000000, (512, 512), (1, 0), 4)
        r = _wait(srv, [t])[t]
        assert r.status == 0 and r.chunks == 1
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_launch_ns <= r.t_done_ns
        assert r.t_launch_ns - r.t_submit_ns < 1_000_000


def test_lone_large_job_takes_growing_pieces():
    """One slot, nothing else waiting: the pieces of a large job double (1, 2, 4, 8,
    16 chunks): a 256 MiB job at 16 MiB chunks goes out in five pieces, not sixteen."""
    with rr.Server(8 << 30, max_inflight=1, max_batch_jobs=64, chunk_bytes=16 * MiB, simulated=True,
                   sim_bytes_per_us=200_000.0) as srv:
        big = srv.submit(0, 0x7e0000000000, (8192, 8192), (1, 0), 4)           # 256 MiB
        r = _wait(srv, [big])[big]
        assert r.status == 0 and 2 <= r.chunks <= 6, r.chunks
