"""GPU parity of rr_gather / rr_copy_range (the read kernel's index-set and
range access patterns, Sec. III.A) against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import rr_synth
from tests.test_emulated_kernels import gather_cases, gather_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    import paper_1011_3583_amd as rr
    assert torch.cuda.is_available()
    rr.lib()
    return rr


def run_gpu(rr, j, soff=0, doff=0):
    import torch
    e = j["esize"]
    x = j["input"]
    count = len(j["idx"]) if "idx" in j else j["count"]
    print(f"gather n={j['src_count']} e={e} count={count} indexed={'idx' in j} "
          f"start={j.get('start')} stride={j.get('stride')}", flush=True)
    src = torch.empty(x.size + soff + 16, dtype=torch.uint8, device="cuda")
    src[soff:soff + x.size].copy_(torch.from_numpy(x))
    n = count * e
    dst = torch.full((n + doff + 16,), 0x5A, dtype=torch.uint8, device="cuda")
    bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    if "idx" in j:
        idx = torch.from_numpy(np.ascontiguousarray(j["idx"])).cuda()
        st = rr.gather_raw(dst.data_ptr() + doff, src.data_ptr() + soff, j["src_count"], idx.data_ptr(), count, e,
                           bad.data_ptr(), sh)
    else:
        st = rr.copy_range_raw(dst.data_ptr() + doff, src.data_ptr() + soff, j["src_count"], j["start"],
                               j["stride"], count, e, sh)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert (out[:doff] == 0x5A).all() and (out[doff + n:] == 0x5A).all(), "wrote outside the output"
    return out[doff:doff + n], int(bad.item())


def test_gather_and_range_cases(rr):
    for k, j in enumerate(gather_cases(5, 120)):
        got, nbad = run_gpu(rr, j, soff=(k % 3) * 5, doff=(k % 5) * 3)
        ref, ref_bad = gather_ref(j)
        assert np.array_equal(got, ref)
        if "idx" in j:
            assert nbad == ref_bad


def test_gather_large(rr):
    """Several thousand workgroups (grid-stride): 16 Mi random and sorted indices
    into a 64 MiB table, and long strided / reversed ranges."""
    g = rr_synth.rng(71)
    for e in (4, 16):
        n = (64 << 20) // e
        x = rr_synth.random_bytes(72 + e, n * e)
        for sort in (False, True):
            idx = g.integers(0, n, 1 << 24).astype(np.int64)
            if sort:
                idx.sort()
            j = dict(src_count=n, esize=e, idx=idx, input=x)
            got, nbad = run_gpu(rr, j)
            ref, _ = gather_ref(j)
            assert nbad == 0 and np.array_equal(got, ref)
        for start, stride in ((0, 3), (n - 1, -1), (5, 2)):
            cnt = (n - 1 - start) // stride + 1 if stride > 0 else start // -stride + 1
            j = dict(src_count=n, esize=e, start=start, stride=stride, count=cnt, input=x)
            got, _ = run_gpu(rr, j)
            assert np.array_equal(got, gather_ref(j)[0])
