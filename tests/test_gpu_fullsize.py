"""GPU parity at the full benchmark sizes, in the launch configuration the benchmark times.

Outputs of up to 4 GiB are checked on sampled elements the oracle computes one
by one (random positions plus the first and last 64 Ki elements), and the
interlace workloads additionally round-trip through de-interlace.
"""
import sys

import numpy as np
import pytest

import oracle
import rr_synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

NSAMPLE = 200_000


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


def _sample_idx(n, seed):
    g = rr_synth.rng(seed)
    head = np.arange(min(n, 65536), dtype=np.int64)
    tail = np.arange(max(0, n - 65536), n, dtype=np.int64)
    rnd = g.integers(0, n, size=min(n, NSAMPLE), dtype=np.int64)
    return np.unique(np.concatenate([head, tail, rnd]))


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
        idx = _sample_idx(n, case * 100 + e)
        got = out.view(n, e)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
        ref = oracle.permute_at(host[:nb], dims, perm, e, idx)
        assert np.array_equal(got, ref), (name, perm, e)


@pytest.mark.parametrize("case", list(range(len(rr_synth.INTERLACE_CASES))))
def test_interlace_full_size(rr, pool, case):
    host, dev = pool
    name, n, count, e = rr_synth.INTERLACE_CASES[case]
    pb = count * e
    _say(name, n, count, e)
    planes_dev = [dev[c * pb:(c + 1) * pb] for c in range(n)]
    joined = torch.empty(n * pb, dtype=torch.uint8, device="cuda")
    st = rr.interlace_raw(joined.data_ptr(), [p.data_ptr() for p in planes_dev], count, e,
                          stream=torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    idx = _sample_idx(count, 900 + case)
    j = joined.view(count, n, e)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    for c in range(n):
        ref = host[c * pb:(c + 1) * pb].reshape(count, e)[idx]
        assert np.array_equal(j[:, c, :], ref), (name, c)
    # de-interlace the joined buffer back into planes: must equal the originals exactly
    outs = [torch.empty(pb, dtype=torch.uint8, device="cuda") for _ in range(n)]
    st = rr.deinterlace_raw([o.data_ptr() for o in outs], joined.data_ptr(), count, e,
                            stream=torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    for c in range(n):
        assert torch.equal(outs[c], planes_dev[c]), (name, c)


def test_batched_workload_full_size(rr):
    """The benchmark's 4096-job batch (7.54 GB per side, seeded inputs on the device),
    through a tuned handle replayed as a hipGraph as the benchmark runs it; every job
    compared with the oracle on its first and last elements plus 256 random ones."""
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
    for i, (s, o, nb) in enumerate(zip(specs, offs, sizes)):
        n = nb // s["esize"]
        x = src[o:o + nb].cpu().numpy()
        y = dst[o:o + nb].cpu().numpy().reshape(n, s["esize"])
        g = rr_synth.rng(7000 + i)
        idx = np.unique(np.concatenate([[0, n - 1], g.integers(0, n, 256)])).astype(np.int64)
        ref = oracle.permute_at(x, s["dims"], s["perm"], s["esize"], idx)
        assert np.array_equal(y[idx], ref), (i, s)


def test_serving_workload_full_size(rr):
    """The serving benchmark's configuration (96 GiB budget, 64 MiB chunks, up to 1024
    jobs per batch, 4 streams) and job mix at full size: 3000 requests drawn from the
    4096-job distribution plus its four 1-4 GiB permutes, arriving in bursts while
    earlier batches run; every result sampled against the oracle."""
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
            n = nb // s["esize"]
            out = torch.empty(nb, dtype=torch.uint8, device="cuda")
            rr.check(rr.permute_raw(out.data_ptr(), r.dst, (nb,), (0,), 1, sh))
            torch.cuda.synchronize()
            gi = rr_synth.rng(9000 + k)
            idx = np.unique(np.concatenate([[0, n - 1], gi.integers(0, n, 256)])).astype(np.int64)
            ref = oracle.permute_at(t.cpu().numpy(), s["dims"], s["perm"], s["esize"], idx)
            got = out.view(n, s["esize"])[torch.from_numpy(idx).cuda()].cpu().numpy()
            assert np.array_equal(got, ref), (k, s)
            srv.release(tickets[k])
        for p, _, _ in inputs:
            srv.free(p)
