"""GPU tests of batched permutes: every job's bytes equal the oracle and equal the
same job run alone with rr_permute (tolerance 0), for one-shot batches and for
reusable handles (plain, persistent, autotuned, hipGraph replay)."""
import sys

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


def _uneven(seed, njobs, max_elems):
    g = rr_synth.rng(seed)
    out = []
    for _ in range(njobs):
        nd = int(g.integers(1, 6))
        while True:
            dims = tuple(int(g.integers(1, 48)) for _ in range(nd))
            if int(np.prod(dims)) <= max_elems:
                break
        out.append({"dims": dims, "perm": tuple(int(v) for v in g.permutation(nd)),
                    "esize": int(g.choice([1, 2, 3, 4, 6, 8, 12, 16]))})
    return out


class Jobs:
    """Device buffers for a list of job specs, inputs uploaded from seeded host bytes."""

    def __init__(self, rr, specs, seed):
        self.specs = specs
        self.host = [rr_synth.random_bytes(seed * 100_003 + i, int(np.prod(s["dims"])) * s["esize"])
                     for i, s in enumerate(specs)]
        sizes = [h.size for h in self.host]
        offs = np.concatenate([[0], np.cumsum([(n + 255) // 256 * 256 for n in sizes])]).astype(np.int64)
        self.src = torch.zeros(int(offs[-1]) + 256, dtype=torch.uint8, device="cuda")
        self.dst = torch.zeros(int(offs[-1]) + 256, dtype=torch.uint8, device="cuda")
        for i, h in enumerate(self.host):
            if h.size:
                self.src[offs[i]:offs[i] + h.size].copy_(torch.from_numpy(h))
        self.offs, self.sizes = offs, sizes
        self.arr = rr.make_jobs([(self.dst.data_ptr() + int(offs[i]), self.src.data_ptr() + int(offs[i]),
                                  s["dims"], s["perm"], s["esize"]) for i, s in enumerate(specs)])

    def out(self, i):
        return self.dst[self.offs[i]:self.offs[i] + self.sizes[i]].cpu().numpy()

    def outs_device(self):
        return self.dst.clone()


def _check_all_vs_oracle(J, sample=None):
    for i, s in enumerate(J.specs):
        got = J.out(i)
        n = int(np.prod(s["dims"]))
        if sample is None or n <= sample:
            ref = oracle.permute(J.host[i], s["dims"], s["perm"], s["esize"])
            assert np.array_equal(got, ref), (i, s)
        else:
            g = rr_synth.rng(i)
            idx = np.unique(np.concatenate([[0, n - 1], g.integers(0, n, sample)])).astype(np.int64)
            ref = oracle.permute_at(J.host[i], s["dims"], s["perm"], s["esize"], idx)
            assert np.array_equal(got.reshape(n, s["esize"])[idx], ref), (i, s)


def test_batched_uneven_jobs_match_oracle_and_alone(rr):
    specs = _uneven(1, 300, 30000)
    specs += [{"dims": (0, 4), "perm": (1, 0), "esize": 4}, {"dims": (64, 64, 32), "perm": (1, 0, 2), "esize": 4},
              {"dims": (7, 9), "perm": (0, 1), "esize": 2}, {"dims": (512, 512), "perm": (1, 0), "esize": 1}]
    J = Jobs(rr, specs, 1)
    _say("batched one-shot", len(specs))
    rr.check(rr.permute_batched_raw(J.arr, len(specs), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    _check_all_vs_oracle(J)
    batched = J.outs_device()
    # each job alone must give the same bytes
    J.dst.zero_()
    for i in range(len(specs)):
        j = J.arr[i]
        s = specs[i]
        rr.check(rr.permute_raw(j.dst, j.src, s["dims"], s["perm"], s["esize"],
                                torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert torch.equal(J.dst, batched)


def test_batched_repeated_calls_reuse_staging(rr):
    """More calls in flight than staging slots: every result still right."""
    specs = _uneven(2, 40, 5000)
    Js = [Jobs(rr, specs, 10 + k) for k in range(7)]
    for k, J in enumerate(Js):
        _say("staging round", k)
        rr.check(rr.permute_batched_raw(J.arr, len(specs), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    for J in Js:
        _check_all_vs_oracle(J)


def test_batched_calls_on_two_streams_share_side_streams(rr):
    """One-shot batched calls fan their groups out on side streams shared per device:
    calls issued alternately on two streams (each after its own input upload on that
    stream) all finish with every job equal to the oracle."""
    specs = _uneven(4, 64, 8000)
    Js = [Jobs(rr, specs, 30 + k) for k in range(6)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for k, J in enumerate(Js):
        st = streams[k % 2]
        _say("two streams, call", k)
        with torch.cuda.stream(st):
            J.dst.zero_()   # queued on this stream: the batch must run after it
        rr.check(rr.permute_batched_raw(J.arr, len(specs), st.cuda_stream))
    for st in streams:
        st.synchronize()
    for J in Js:
        _check_all_vs_oracle(J)


def test_batched_calls_from_several_host_threads(rr):
    """Four host threads each issue three batched calls of 600 jobs at once, each on
    a stream of its own: the calls plan in slices on the library's planning workers
    (or on threads of their own when those are busy) and share the staging ring and
    side streams; every job equals the oracle."""
    import threading
    specs = _uneven(5, 600, 3000)
    Js = [Jobs(rr, specs, 50 + k) for k in range(4)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in Js]
    errs = []

    def run(k):
        try:
            for _ in range(3):
                rr.check(rr.permute_batched_raw(Js[k].arr, len(specs), streams[k].cuda_stream))
        except Exception as e:   # reported below, on the test's thread
            errs.append(e)

    th = [threading.Thread(target=run, args=(k,)) for k in range(len(Js))]
    _say("four host threads, three batched calls of 600 jobs each")
    for t in th:
        t.start()
    for t in th:
        t.join()
    for st in streams:
        st.synchronize()
    assert not errs, errs
    for J in Js:
        _check_all_vs_oracle(J)


@pytest.mark.parametrize("flags", [0, 4, 2, 1, 1 | 4, 1 | 2])
def test_batch_handle_modes(rr, flags):
    specs = _uneven(3, 120, 20000)
    J = Jobs(rr, specs, 3)
    _say("batch handle flags", flags)
    b = rr.Batch(J.arr, flags)
    info = b.info()
    assert info["ngroups"] >= 2 and info["njobs"] == len(specs)
    if flags & 2:
        assert info["tuned_us"] > 0
    expected = None
    for rep in range(3):
        J.dst.zero_()                              # eager work between replays
        torch.cuda.synchronize()
        b.launch(torch.cuda.current_stream())
        torch.cuda.synchronize()
        if expected is None:
            _check_all_vs_oracle(J)
            expected = J.outs_device()
        else:
            assert torch.equal(J.dst, expected), f"replay {rep} differs"
    b.close()


def test_sampled_uneven_workload(rr):
    """4096 uneven jobs drawn like the batched workload (sizes capped for test time)."""
    specs = rr_synth.sample_jobs(4, njobs=4096, total_range=(1e3, 2e5), footprint_cap=4 << 30)
    J = Jobs(rr, specs, 4)
    _say("sampled workload", len(specs))
    rr.check(rr.permute_batched_raw(J.arr, len(specs), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    _check_all_vs_oracle(J, sample=64)


def test_overlapping_jobs_rejected(rr):
    x = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    base = x.data_ptr()
    # job 1 writes [2048, 6144), inside job 0's output [0, 4096)
    arr = rr.make_jobs([(base, base + 8192, (32, 32), (1, 0), 4),
                        (base + 2048, base + 16384, (32, 32), (1, 0), 4)])
    assert rr.permute_batched_raw(arr, 2, 0) == 3
    assert "overlap" in rr.last_error()
    # job 1 reads [2048, 6144), which overlaps job 0's output [0, 4096)
    arr = rr.make_jobs([(base, base + 8192, (32, 32), (1, 0), 4),
                        (base + 20000, base + 2048, (32, 32), (1, 0), 4)])
    assert rr.permute_batched_raw(arr, 2, 0) == 3
    assert not x.any()  # nothing was launched


def test_batched_short_runs_sharing_lines(rr):
    """Runs of 64-127 bytes that share input lines load through the caches with each
    XCD taking a contiguous range of a job's blocks: a batch of such jobs (and the
    same jobs launched alone) equals the oracle."""
    specs = [{"dims": (60, 70, 33), "perm": (1, 0, 2), "esize": 2}, {"dims": (90, 110, 9), "perm": (1, 0, 2), "esize": 8},
             {"dims": (300, 200, 100), "perm": (1, 0, 2), "esize": 1}, {"dims": (40, 50, 30, 24), "perm": (2, 0, 1, 3), "esize": 4},
             {"dims": (1001, 999), "perm": (1, 0), "esize": 4}]
    J = Jobs(rr, specs, 9)
    for s, j in zip(specs, J.arr):
        d = rr.plan_describe(s["dims"], s["perm"], s["esize"], j.dst, j.src)
        if d["class"] == "run":
            assert d["cached"] == "1", d
    _say("batched short runs", len(specs))
    b = rr.Batch(J.arr, 0)
    b.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    b.close()
    _check_all_vs_oracle(J)
    J.dst.zero_()
    for i, s in enumerate(specs):
        j = J.arr[i]
        rr.check(rr.permute_raw(j.dst, j.src, s["dims"], s["perm"], s["esize"], torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    _check_all_vs_oracle(J)


def test_large_one_shot_batch_in_chunks(rr):
    """A one-shot batch of 2500 jobs is validated whole, then planned and launched
    in chunks: every job equals the oracle; a batch whose last job is invalid
    fails with that job's index and writes nothing."""
    specs = _uneven(21, 2500, 6000)
    J = Jobs(rr, specs, 21)
    _say("one-shot chunked", len(specs))
    for _ in range(2):   # twice: the second call reuses the ring slots
        J.dst.zero_()
        rr.check(rr.permute_batched_raw(J.arr, len(specs), torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        _check_all_vs_oracle(J)
    J.dst.fill_(0x77)
    torch.cuda.synchronize()
    bad = rr.make_jobs([(J.arr[i].dst, J.arr[i].src, s["dims"], s["perm"], s["esize"]) for i, s in enumerate(specs[:-1])] +
                       [(J.arr[len(specs) - 1].dst, J.arr[len(specs) - 1].src, (4, 4), (0, 0), 4)])
    st = rr.permute_batched_raw(bad, len(specs), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == rr.STATUS_CODE["RR_ERR_INVALID_ARG"], st
    assert f"job {len(specs) - 1}" in rr.last_error()
    assert bool((J.dst == 0x77).all())


def test_small_jobs_take_the_batch_shape(rr):
    """With no tile override, jobs of at most 128 MiB per side planned into a batch
    take 512-byte input and 256-byte output row targets, output-order traversal and
    cached tile accesses: the batch's workgroups add up to the jobs' single-permute
    grids under that override (and not to their built-in grids), and every output
    equals the oracle."""
    rr.tune_clear()
    specs = rr_synth.sample_jobs(779, njobs=96, total_range=(1e3, 3e5))
    J = Jobs(rr, specs, 41)
    _say("small-job batch shape", len(specs))
    b = rr.Batch(J.arr, 0)
    total = sum(g["workgroups"] for g in b.groups())

    def grids(**kw):
        rr.set_tile_override(weave=False, **kw)
        try:
            return sum(int(rr.plan_describe(s["dims"], s["perm"], s["esize"], j.dst, j.src)["grid"])
                       for s, j in zip(specs, J.arr))
        finally:
            rr.set_tile_override(0, 0, None)

    small = grids(in_row_bytes=512, out_row_bytes=256, order_out=True, cache=3)
    builtin = grids()
    assert total == small, (total, small, builtin)
    assert small != builtin
    b.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    _check_all_vs_oracle(J)
