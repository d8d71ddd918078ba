"""GPU parity of rr_reorder (N-to-M reorder with base and range, Sec. III.B)
against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import rr_synth
from tests.test_emulated_kernels import REORDER_CASES, SELECT_CASES, random_boxes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    import paper_1011_3583_amd as rr
    assert torch.cuda.is_available()
    rr.lib()
    rr.set_tile_override()
    return rr


def gpu_reorder(rr, x, dims, base, range_, order, e, soff=0, doff=0):
    import torch
    n = int(np.prod([range_[o] for o in order], dtype=np.int64)) * e if order else e
    src = torch.empty(x.size + soff + 16, dtype=torch.uint8, device="cuda")
    src[soff:soff + x.size].copy_(torch.from_numpy(x))
    dst = torch.full((n + doff + 16,), 0x5A, dtype=torch.uint8, device="cuda")
    st = rr.reorder_raw(dst.data_ptr() + doff, src.data_ptr() + soff, dims, base, range_, order, e,
                        torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert (out[:doff] == 0x5A).all() and (out[doff + n:] == 0x5A).all(), "wrote outside the output"
    return out[doff:doff + n]


def check(rr, dims, base, range_, order, e, seed, soff=0, doff=0):
    print(f"reorder dims={dims} base={base} range={range_} order={order} e={e} off={soff}/{doff}", flush=True)
    x = rr_synth.random_bytes(seed, int(np.prod(dims, dtype=np.int64)) * e)
    got = gpu_reorder(rr, x, dims, base, range_, order, e, soff, doff)
    ref = oracle.reorder_slice(x, dims, base, range_, order, e)
    assert np.array_equal(got, ref), (dims, base, range_, order, e)


def test_reorder_cases(rr):
    for i, (d, b, r, o, e) in enumerate(REORDER_CASES):
        check(rr, d, b, r, o, e, 11000 + i)
        check(rr, d, b, r, o, e, 11050 + i, soff=3, doff=5)


def test_reorder_random_boxes(rr):
    for i, (d, b, r, o, e) in enumerate(random_boxes(91, 150)):
        check(rr, d, b, r, o, e, 11100 + i)


def test_reorder_large_boxes(rr):
    """Several tiles per launch: crops of the dense benchmark shapes, a channel of
    an HWC image (gather), a slab (copy), a 4-D box with a fixed axis."""
    cases = [((512, 512, 64), (13, 7, 0), (480, 500, 64), (2, 0, 1), 4),
             ((1024, 1024, 4), (0, 0, 2), (1024, 1024, 1), (0, 1), 1),
             ((1024, 1024, 4), (0, 0, 1), (1024, 1024, 2), (1, 0, 2), 2),
             ((2048, 1024), (100, 0), (1000, 1024), (0, 1), 4),
             ((64, 128, 128, 16), (5, 3, 0, 0), (50, 1, 128, 16), (3, 2, 0), 2),
             ((300, 301, 17), (1, 2, 3), (290, 297, 13), (1, 2, 0), 8)]
    for i, (d, b, r, o, e) in enumerate(cases):
        check(rr, d, b, r, o, e, 11300 + i)


def test_reorder_with_unaligned_micro_tiles(rr):
    rr.set_tile_override(umt=1)
    try:
        for i, (d, b, r, o, e) in enumerate(REORDER_CASES):
            check(rr, d, b, r, o, e, 11400 + i)
    finally:
        rr.set_tile_override()


def test_reorder_strided_select(rr):
    """One component of interleaved records (the select kernel): every case at
    aligned pointers, at element-aligned offsets, and at odd offsets (the gather)."""
    for i, (d, b, r, o, e) in enumerate(SELECT_CASES):
        assert rr.reorder_describe(d, b, r, o, e, 1 << 20, 1 << 30)["class"] == "select"
        check(rr, d, b, r, o, e, 12000 + i)
        check(rr, d, b, r, o, e, 12050 + i, soff=3 * e, doff=e)
        check(rr, d, b, r, o, e, 12100 + i, soff=1, doff=3)


def test_channel_of_rgba_image_full_size(rr):
    """The benchmark's channel extraction: channel 2 of a 16384 x 16384 RGBA image
    (1 GiB in, 256 MiB out), every output byte against the oracle."""
    dims, base, rng, order, e = (16384, 16384, 4), (0, 0, 2), (16384, 16384, 1), (0, 1), 1
    assert rr.reorder_describe(dims, base, rng, order, e, 1 << 20, 1 << 30)["class"] == "select"
    check(rr, dims, base, rng, order, e, 12200)
