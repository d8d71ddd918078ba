"""GPU parity at the full benchmark sizes, in the launch configuration the benchmark times.

Every output element is compared with the oracle: outputs of up to 4 GiB are
copied to the host whole and the oracle recomputes them piece by piece
(oracle.permute_range, several pieces at once on host threads); interlace and
de-interlace outputs likewise, plane range by plane range; every job of the
4096-job batch and every served request whole.
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import rr_synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

# host threads for the oracle (the host's share of cores for one GPU)
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
PIECE = 1 << 23          # output elements per oracle piece


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rr():
    assert torch.cuda.is_available()
    import paper_1011_3583_amd as rr
    rr.set_tile_override(0, 0, None)
    return rr


@pytest.fixture(scope="module")
def pool():
    """4 GiB of seeded random bits on the host and on the device (inputs are slices)."""
    host = rr_synth.random_bytes(20251202, 4 << 30)
    dev = torch.from_numpy(host).to("cuda")
    return host, dev


def first_mismatch(x, dims, perm, e, got):
    """Compare a whole permute output (flat host bytes) with the oracle, piece by
    piece on WORKERS threads; the first mismatching output element, or None."""
    n = int(np.prod(dims, dtype=np.int64))
    assert got.size == n * e

    def piece(a):
        c = min(PIECE, n - a)
        ref = oracle.permute_range(x, dims, perm, e, a, c)
        mine = got[a * e:(a + c) * e]
        if np.array_equal(mine, ref):
            return None
        return a + int(np.nonzero((mine.reshape(c, e) != ref.reshape(c, e)).any(axis=1))[0][0])

    with ThreadPoolExecutor(WORKERS) as ex:
        bad = [r for r in ex.map(piece, range(0, n, PIECE)) if r is not None]
    return min(bad) if bad else None


@pytest.mark.parametrize("case", list(range(len(rr_synth.DENSE_CASES))))
def test_dense_full_size(rr, pool, case):
    host, dev = pool
    name, dims, perm = rr_synth.DENSE_CASES[case]
    out = None
    for e in rr_synth.ESIZES:
        n = int(np.prod(dims, dtype=np.int64))
        nb = n * e
        _say(name, dims, perm, e, nb)
        del out
        out = torch.empty(nb, dtype=torch.uint8, device="cuda")
        st = rr.permute_raw(out.data_ptr(), dev.data_ptr(), dims, perm, e,
                            stream=torch.cuda.current_stream().cuda_stream)
        assert st == 0, rr.last_error()
        torch.cuda.synchronize()
        bad = first_mismatch(host[:nb], dims, perm, e, out.cpu().numpy())
        assert bad is None, (name, perm, e, "first wrong output element", bad)


@pytest.mark.parametrize("case", list(range(len(rr_synth.INTERLACE_CASES))))
def test_interlace_full_size(rr, pool, case):
    """Interlace of n planes of the pool, and de-interlace of the pool's first n
    planes' bytes read as one joined buffer: every output byte against the
    oracle, plane range by plane range; the joined output also round-trips."""
    host, dev = pool
    name, n, count, e = rr_synth.INTERLACE_CASES[case]
    pb = count * e
    sh = torch.cuda.current_stream().cuda_stream
    _say(name, n, count, e)
    planes_dev = [dev[c * pb:(c + 1) * pb] for c in range(n)]
    joined = torch.empty(n * pb, dtype=torch.uint8, device="cuda")
    assert rr.interlace_raw(joined.data_ptr(), [p.data_ptr() for p in planes_dev], count, e, stream=sh) == 0, \
        rr.last_error()
    torch.cuda.synchronize()
    got = joined.cpu().numpy()

    def inter(a):
        b = min(count, a + PIECE)
        ref = oracle.interlace([host[c * pb + a * e:c * pb + b * e] for c in range(n)], e)
        return np.array_equal(got[a * n * e:b * n * e], ref)

    with ThreadPoolExecutor(WORKERS) as ex:
        assert all(ex.map(inter, range(0, count, PIECE))), (name, "interlace")
    del got
    # de-interlace of the pool's first n*pb bytes (random bits) into n planes
    outs = [torch.empty(pb, dtype=torch.uint8, device="cuda") for _ in range(n)]
    assert rr.deinterlace_raw([o.data_ptr() for o in outs], dev.data_ptr(), count, e, stream=sh) == 0, \
        rr.last_error()
    torch.cuda.synchronize()
    planes = [o.cpu().numpy() for o in outs]

    def deinter(a):
        b = min(count, a + PIECE)
        ref = oracle.deinterlace(host[a * n * e:b * n * e], n, e)
        return all(np.array_equal(planes[c][a * e:b * e], ref[c]) for c in range(n))

    with ThreadPoolExecutor(WORKERS) as ex:
        assert all(ex.map(deinter, range(0, count, PIECE))), (name, "de-interlace")
    # and the interlaced buffer splits back into the original planes
    st = rr.deinterlace_raw([o.data_ptr() for o in outs], joined.data_ptr(), count, e, stream=sh)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    for c in range(n):
        assert torch.equal(outs[c], planes_dev[c]), (name, c)


def test_batched_workload_full_size(rr):
    """The benchmark's 4096-job batch (7.54 GB per side, seeded inputs on the device),
    through a tuned handle replayed as a hipGraph as the benchmark runs it; every job
    compared whole with the oracle."""
    import bench
    specs = rr_synth.sample_jobs(4096_0001, njobs=4096)
    src, dst, offs, sizes = bench._job_buffers(torch, specs)
    jobs = rr.make_jobs([(dst.data_ptr() + o, src.data_ptr() + o, s["dims"], s["perm"], s["esize"])
                         for o, s in zip(offs, specs)])
    _say("batched full size", len(specs), sum(sizes))
    h = rr.Batch(jobs, rr.RR_BATCH_TUNE | rr.RR_BATCH_GRAPH)
    try:
        dst.zero_()
        h.launch(torch.cuda.current_stream())
        torch.cuda.synchronize()
    finally:
        h.close()
    xs, ys = src.cpu().numpy(), dst.cpu().numpy()

    def job_ok(i):
        s, o, nb = specs[i], offs[i], sizes[i]
        return np.array_equal(ys[o:o + nb], oracle.permute(xs[o:o + nb], s["dims"], s["perm"], s["esize"]))

    with ThreadPoolExecutor(WORKERS) as ex:
        ok = list(ex.map(job_ok, range(len(specs))))
    bad = [i for i, v in enumerate(ok) if not v]
    assert not bad, [(i, specs[i]) for i in bad[:5]]


def test_serving_workload_full_size(rr):
    """The serving benchmark's configuration (96 GiB budget, 64 MiB chunks, up to 1024
    jobs per batch, 4 streams) and job mix at full size: 3000 requests drawn from the
    4096-job distribution plus its four 1-4 GiB permutes, arriving in bursts while
    earlier batches run; every result compared whole with the oracle."""
    import time
    small = rr_synth.sample_jobs(5_0001, njobs=4096)
    large = rr_synth.large_jobs(5_0002, count=4)
    g = rr_synth.rng(77)
    picks = [small[int(k)] for k in g.integers(0, len(small), 3000)] + large
    order = [int(k) for k in g.permutation(len(picks))]
    sh = torch.cuda.current_stream().cuda_stream
    with rr.Server(96 << 30, max_inflight=4, max_batch_jobs=1024, chunk_bytes=64 << 20, tick_us=5) as srv:
        inputs = []
        for k, s in enumerate(picks):
            nb = int(np.prod(s["dims"])) * s["esize"]
            t = torch.empty(nb, dtype=torch.uint8, device="cuda")
            t.random_(0, 256, generator=torch.Generator(device="cuda").manual_seed(k))
            p = srv.alloc(nb)
            rr.check(rr.permute_raw(p, t.data_ptr(), (nb,), (0,), 1, sh))
            inputs.append((p, t, nb))
        torch.cuda.synchronize()
        _say("serving full size", len(picks), sum(nb for _, _, nb in inputs))
        tickets = {}
        for n, k in enumerate(order):
            s = picks[k]
            tickets[k] = srv.submit(0, inputs[k][0], s["dims"], s["perm"], s["esize"])
            if n % 50 == 0:
                time.sleep(0.0005)
        left, res, t0 = set(tickets.values()), {}, time.time()
        while left and time.time() - t0 < 300:
            for t in srv.completions():
                if t in left:
                    res[t] = srv.poll(t)
                    left.discard(t)
            time.sleep(0.0002)
        assert not left, f"{len(left)} requests did not complete"
        assert srv.stats()["batches"] > 1
        for k, s in enumerate(picks):
            r = res[tickets[k]]
            assert r.status == 0, (k, s)
            _, t, nb = inputs[k]
            out = torch.empty(nb, dtype=torch.uint8, device="cuda")
            rr.check(rr.permute_raw(out.data_ptr(), r.dst, (nb,), (0,), 1, sh))
            torch.cuda.synchronize()
            bad = first_mismatch(t.cpu().numpy(), s["dims"], s["perm"], s["esize"], out.cpu().numpy())
            assert bad is None, (k, s, "first wrong output element", bad)
            srv.release(tickets[k])
        for p, _, _ in inputs:
            srv.free(p)
