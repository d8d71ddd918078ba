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


def test_large_job_is_chunked_and_small_jobs_pass_it():
    with rr.Server(8 << 30, max_inflight=2, max_batch_jobs=64, chunk_bytes=16 * MiB, simulated=True,
                   sim_bytes_per_us=2_000.0) as srv:
        big = srv.submit(0, 0x7e0000000000, (8192, 8192), (1, 0), 4)           # 256 MiB
        time.sleep(0.002)
        small = [srv.submit(0, 0x7f0000000000 + i * MiB, (64, 64), (1, 0), 4) for i in range(20)]
        res = _wait(srv, [big] + small)
        assert res[big].chunks >= 8
        assert all(res[t].chunks == 1 for t in small)
        # every small job finished before the large one
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
