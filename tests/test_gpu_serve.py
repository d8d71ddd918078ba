"""GPU tests of the serving loop: jobs arriving while others run are admitted and
batched, a large job runs whole beside them (several slots) or is cut into pieces
interleaved with them (one slot), and each result equals the same job run alone
with rr_permute and the oracle (tolerance 0)."""
import sys
import time

import numpy as np
import pytest

import oracle
import rr_synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rr():
    assert torch.cuda.is_available()
    import paper_1011_3583_amd as rr
    rr.set_tile_override(0, 0, None)
    return rr


def _drain(srv, tickets, timeout=60.0):
    left, res, t0 = set(tickets), {}, time.time()
    while left and time.time() - t0 < timeout:
        for t in srv.completions():
            if t in left:
                res[t] = srv.poll(t)
                left.discard(t)
        time.sleep(0.0002)
    assert not left, f"{len(left)} tickets did not complete"
    return res


@pytest.mark.parametrize("slots", [3, 1])
def test_mixed_arrivals_alone_equals_in_mix(rr, slots):
    specs = rr_synth.sample_jobs(11, njobs=300, total_range=(1e3, 3e5), footprint_cap=1 << 30)
    specs.append({"dims": (4096, 8192), "perm": (1, 0), "esize": 4})           # 128 MiB, large
    specs.append({"dims": (256, 512, 256), "perm": (2, 1, 0), "esize": 2})     # 64 MiB, large
    host = [rr_synth.random_bytes(5000 + i, int(np.prod(s["dims"])) * s["esize"]) for i, s in enumerate(specs)]
    with rr.Server(8 << 30, max_inflight=slots, max_batch_jobs=64, chunk_bytes=8 << 20) as srv:
        srcs = []
        for h in host:
            p = srv.alloc(h.size)
            t = torch.empty(h.size, dtype=torch.uint8, device="cuda")
            t.copy_(torch.from_numpy(h))
            srcs.append((p, t))
        # move inputs into the server's resident buffers with our own kernel
        for (p, t), h in zip(srcs, host):
            rr.check(rr.permute_raw(p, t.data_ptr(), (h.size,), (0,), 1, torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        g = rr_synth.rng(3)
        order = list(g.permutation(len(specs)))
        tickets = {}
        _say("serving", len(specs), "jobs,", slots, "slots")
        for k, i in enumerate(order):
            s = specs[i]
            tickets[i] = srv.submit(0, srcs[i][0], s["dims"], s["perm"], s["esize"])
            if k % 7 == 0:
                time.sleep(0.0003)      # arrivals spread while earlier batches run
        res = _drain(srv, tickets.values())
        st = srv.stats()
        assert st["batches"] >= 3 and st["completed"] == len(specs)
        big = res[tickets[len(specs) - 2]].chunks
        assert big > 1 if slots == 1 else big == 1, (slots, big)
        for i, s in enumerate(specs):
            r = res[tickets[i]]
            assert r.status == 0, (i, s)
            n = int(np.prod(s["dims"])) * s["esize"]
            out = torch.empty(n, dtype=torch.uint8, device="cuda")
            # view of the server-allocated output
            rr.check(rr.permute_raw(out.data_ptr(), r.dst, (n,), (0,), 1, torch.cuda.current_stream().cuda_stream))
            alone = torch.empty(n, dtype=torch.uint8, device="cuda")
            rr.check(rr.permute_raw(alone.data_ptr(), srcs[i][1].data_ptr(), s["dims"], s["perm"], s["esize"],
                                    torch.cuda.current_stream().cuda_stream))
            torch.cuda.synchronize()
            assert torch.equal(out, alone), (i, s)
            nel = n // s["esize"]
            idx = np.unique(rr_synth.rng(i).integers(0, nel, 64)).astype(np.int64)
            ref = oracle.permute_at(host[i], s["dims"], s["perm"], s["esize"], idx)
            assert np.array_equal(out.view(nel, s["esize"])[torch.from_numpy(idx).cuda()].cpu().numpy(), ref)
            srv.release(tickets[i])
        assert srv.stats()["budget_used"] == sum((h.size + 255) // 256 * 256 for h in host)
        for p, _ in srcs:
            srv.free(p)


def test_failed_batch_then_recovery_on_gpu(rr):
    with rr.Server(1 << 30, max_inflight=2, max_batch_jobs=16, chunk_bytes=0) as srv:
        x = srv.alloc(1 << 20)
        srv.fail_next_batch()
        t1 = srv.submit(0, x, (512, 512), (1, 0), 4)
        r1 = _drain(srv, [t1])[t1]
        assert r1.status == rr.STATUS_CODE["RR_ERR_HIP"]
        t2 = srv.submit(0, x, (512, 512), (1, 0), 4)
        assert _drain(srv, [t2])[t2].status == 0
        srv.release(t1)
        srv.release(t2)
        srv.free(x)
