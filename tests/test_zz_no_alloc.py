"""GPU test of rr_permute_batched_noalloc, the batched entry point that allocates
nothing (its job table lives in the library's fixed device array): on two calls
in a row on one stream, the second with fewer and smaller jobs, every job's bytes
equal what rr_permute_batched writes for it and equal the oracle (tolerance 0);
device memory in use does not change across the calls; a batch whose table would
not fit is refused before anything is written."""
import ctypes
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


def _specs(seed, njobs, max_dim, max_elems):
    g = rr_synth.rng(seed)
    out = []
    for _ in range(njobs):
        nd = int(g.integers(1, 6))
        while True:
            dims = tuple(int(g.integers(1, max_dim + 1)) for _ in range(nd))
            if int(np.prod(dims)) <= max_elems:
                break
        out.append({"dims": dims, "perm": tuple(int(v) for v in g.permutation(nd)),
                    "esize": int(g.choice([1, 2, 3, 4, 6, 8, 12, 16]))})
    return out


class _Buffers:
    """One source and two destination allocations holding every job at 256-byte offsets."""

    def __init__(self, rr, specs, seed):
        self.specs = specs
        self.host = [rr_synth.random_bytes(seed * 7919 + i, int(np.prod(s["dims"])) * s["esize"])
                     for i, s in enumerate(specs)]
        sizes = [h.size for h in self.host]
        self.offs = np.concatenate([[0], np.cumsum([(n + 255) // 256 * 256 for n in sizes])]).astype(np.int64)
        total = int(self.offs[-1]) + 256
        self.src = torch.zeros(total, dtype=torch.uint8, device="cuda")
        self.ref = torch.zeros(total, dtype=torch.uint8, device="cuda")
        self.out = torch.zeros(total, dtype=torch.uint8, device="cuda")
        for i, h in enumerate(self.host):
            if h.size:
                self.src[self.offs[i]:self.offs[i] + h.size].copy_(torch.from_numpy(h))

    def jobs(self, rr, dst):
        return rr.make_jobs([(dst.data_ptr() + int(self.offs[i]), self.src.data_ptr() + int(self.offs[i]),
                              s["dims"], s["perm"], s["esize"]) for i, s in enumerate(self.specs)])

    def check(self, label):
        ref = self.ref.cpu().numpy()
        out = self.out.cpu().numpy()
        for i, s in enumerate(self.specs):
            a, n = int(self.offs[i]), self.host[i].size
            want = oracle.permute(self.host[i], s["dims"], s["perm"], s["esize"])
            assert np.array_equal(ref[a:a + n], want), f"{label}: rr_permute_batched job {i} {s}"
            assert np.array_equal(out[a:a + n], want), f"{label}: noalloc job {i} {s}"


def _mem_in_use():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return total.value - free.value


def test_noalloc_matches_batched_two_calls():
    import paper_1011_3583_amd as rr
    rr.set_tile_override(0, 0, None)
    big = _Buffers(rr, _specs(501, 400, 40, 60_000), 1)
    small = _Buffers(rr, _specs(502, 37, 12, 2_000), 2)
    stream = torch.cuda.current_stream()
    # warm-up: the table array's address is looked up on the first call
    _say("noalloc warm-up", len(small.specs), "jobs")
    rr.check(rr.permute_batched_noalloc_raw(small.jobs(rr, small.out), len(small.specs), stream))
    torch.cuda.synchronize()
    small.out.zero_()
    torch.cuda.synchronize()
    _say("reference: rr_permute_batched", len(big.specs), "then", len(small.specs), "jobs")
    rr.check(rr.permute_batched_raw(big.jobs(rr, big.ref), len(big.specs), stream))
    rr.check(rr.permute_batched_raw(small.jobs(rr, small.ref), len(small.specs), stream))
    torch.cuda.synchronize()
    before = _mem_in_use()
    _say("noalloc: two calls in a row on one stream,", len(big.specs), "then", len(small.specs), "jobs")
    rr.check(rr.permute_batched_noalloc_raw(big.jobs(rr, big.out), len(big.specs), stream))
    rr.check(rr.permute_batched_noalloc_raw(small.jobs(rr, small.out), len(small.specs), stream))
    torch.cuda.synchronize()
    after = _mem_in_use()
    big.check("first call")
    small.check("second call")
    assert after == before, f"device memory in use changed across the calls: {before} -> {after}"


def test_noalloc_refuses_oversized_table():
    import paper_1011_3583_amd as rr
    rr.set_tile_override(0, 0, None)
    # 7000 small transposes: about 4.7 MB of tile arguments, over the 4 MiB table
    specs = [{"dims": (7, 9), "perm": (1, 0), "esize": 4}] * 7000
    bufs = _Buffers(rr, specs, 3)
    _say("noalloc oversized table", len(specs), "jobs (validated on the host, nothing launched)")
    st = rr.permute_batched_noalloc_raw(bufs.jobs(rr, bufs.out), len(specs), torch.cuda.current_stream())
    assert st == rr.STATUS_CODE["RR_ERR_UNSUPPORTED"], rr.last_error()
    assert "4 MiB" in rr.last_error()
    torch.cuda.synchronize()
    assert int(bufs.out.count_nonzero()) == 0
