"""GPU parity: librr on cuda:0 against the CPU oracle, bit for bit.

Small and medium problems are compared element by element over the whole
output; the full-size dense and interlace workloads are compared on sampled
output elements the oracle computes one by one, plus the head and tail of the
output.  Every case prints its name before it runs.
"""
import itertools
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
    assert torch.cuda.is_available(), "GPU tests need cuda:0"
    import paper_1011_3583_amd as rr
    rr.lib()
    rr.set_tile_override(0, 0, None)
    return rr


def _dev_buf(nbytes, off=0):
    """A device byte buffer with a usable window of nbytes starting `off` bytes past a
    256-byte-aligned base."""
    t = torch.empty(nbytes + off + 16, dtype=torch.uint8, device="cuda")
    return t, t.data_ptr() + off


def _upload(x, off=0):
    t, p = _dev_buf(x.size, off)
    if x.size:
        t[off:off + x.size].copy_(torch.from_numpy(x))
    return t, p


def _download(t, off, n):
    return t[off:off + n].cpu().numpy()


def gpu_permute(rr, x, dims, perm, e, soff=0, doff=0):
    n = x.size
    ts, ps = _upload(x, soff)
    td, pd = _dev_buf(n, doff)
    td.fill_(0x5A)
    st = rr.permute_raw(pd, ps, dims, perm, e, stream=torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    out = _download(td, doff, n)
    # nothing written outside the window
    guard = td.cpu().numpy()
    assert np.all(guard[:doff] == 0x5A) and np.all(guard[doff + n:] == 0x5A)
    return out


def check_permute(rr, dims, perm, e, seed, soff=0, doff=0):
    _say("permute", dims, perm, e, soff, doff)
    x = rr_synth.random_bytes(seed, int(np.prod(dims, dtype=np.int64)) * e)
    got = gpu_permute(rr, x, dims, perm, e, soff, doff)
    ref = oracle.permute(x, dims, perm, e)
    assert np.array_equal(got, ref), (dims, perm, e, soff, doff)


def test_small_dense_transpose_1024(rr):
    """1024x1024 transpose of 4-byte random bit patterns."""
    check_permute(rr, (1024, 1024), (1, 0), 4, 1)


def test_brute_force_small_ranks(rr):
    shapes = {1: (7,), 2: (5, 3), 3: (3, 5, 2), 4: (2, 3, 1, 5)}
    seed = 0
    for nd, dims in shapes.items():
        for perm in itertools.permutations(range(nd)):
            for e in (1, 2, 3, 4, 5, 6, 7, 8, 12, 16):
                seed += 1
                check_permute(rr, dims, perm, e, seed, soff=seed % 16, doff=(seed * 7) % 16)


def test_rank5_all_perms(rr):
    for i, perm in enumerate(itertools.permutations(range(5))):
        check_permute(rr, (2, 3, 2, 4, 2), perm, (1, 2, 4, 8, 16)[i % 5], 1000 + i)


@pytest.mark.parametrize("e", [1, 2, 4, 8, 16])
def test_wide_vectors_and_partial_tiles(rr, e):
    cases = [((48, 80), (1, 0)), ((272, 48), (1, 0)), ((32, 48, 64), (2, 1, 0)),
             ((32, 48, 64), (1, 2, 0)), ((32, 48, 64), (2, 0, 1)), ((16, 32, 48), (0, 2, 1)),
             ((33, 47), (1, 0)), ((129, 3, 65), (2, 1, 0)), ((16, 16, 16, 16), (0, 3, 1, 2)),
             ((16, 16, 16, 16), (0, 2, 3, 1)), ((8, 8, 8, 8, 8), (4, 2, 0, 3, 1)),
             ((1000, 3), (1, 0)), ((3, 1000), (1, 0)), ((4, 100, 3, 6), (1, 3, 0, 2))]
    for i, (dims, perm) in enumerate(cases):
        check_permute(rr, dims, perm, e, 2000 + i)
        check_permute(rr, dims, perm, e, 3000 + i, soff=(e % 16) or 4, doff=8)


def test_medium_ragged_multi_tile(rr):
    """Sizes spanning many tiles with ragged tails on every tiled axis."""
    for i, (dims, perm, e) in enumerate([((1000, 1001), (1, 0), 4), ((333, 444, 5), (2, 0, 1), 2),
                                         ((97, 129, 65), (2, 1, 0), 1), ((32, 32, 32, 32, 32), (4, 2, 0, 3, 1), 1),
                                         ((64, 65, 66, 7), (3, 1, 0, 2), 8), ((513, 257), (1, 0), 16),
                                         ((255, 257, 3), (1, 2, 0), 12), ((3000, 17), (1, 0), 6)]):
        check_permute(rr, dims, perm, e, 4000 + i)


def test_tile_overrides(rr):
    try:
        k = 0
        for rbi, rbo in [(64, 64), (128, 512), (512, 128), (1024, 64), (2048, 2048)]:
            for order in (False, True):
                rr.set_tile_override(rbi, rbo, order)
                for dims, perm, e in [((96, 80), (1, 0), 1), ((40, 24, 48), (2, 0, 1), 4),
                                      ((40, 24, 48), (1, 2, 0), 2), ((20, 36, 16), (2, 1, 0), 8),
                                      ((17, 31), (1, 0), 16), ((12, 12, 12, 12), (3, 1, 2, 0), 12)]:
                    k += 1
                    check_permute(rr, dims, perm, e, 5000 + k)
    finally:
        rr.set_tile_override(0, 0, None)


def test_size_zero_and_one(rr):
    for i, (dims, perm, e) in enumerate([((0, 5), (1, 0), 4), ((5, 0, 3), (2, 0, 1), 2),
                                         ((1, 1, 1), (2, 1, 0), 8), ((1,), (0,), 16),
                                         ((1, 7, 1, 9), (3, 2, 1, 0), 4)]):
        check_permute(rr, dims, perm, e, 6000 + i)


def test_paper_table1_orders(rr):
    """Table 1: all six orders of the fastest-first 128x256x512 set, 4-byte elements."""
    sizes = rr_synth.PAPER_TABLE1_SIZES
    dims = tuple(reversed(sizes))
    x = rr_synth.random_bytes(7, int(np.prod(dims)) * 4)
    for order in itertools.permutations(range(3)):
        perm = rr.order_to_perm(order)
        _say("table1", order, perm)
        got = gpu_permute(rr, x, dims, perm, 4)
        ref = oracle.reorder_paper(x, sizes, order, 4)
        assert np.array_equal(got, ref), order


def test_paper_table2_reorders(rr):
    """Table 2's four reorders in the paper's notation, 4-byte elements."""
    for i, (sizes, order) in enumerate(rr_synth.PAPER_TABLE2):
        dims = tuple(reversed(sizes))
        perm = rr.order_to_perm(order)
        _say("table2", sizes, order, perm)
        x = rr_synth.random_bytes(70 + i, int(np.prod(dims)) * 4)
        got = gpu_permute(rr, x, dims, perm, 4)
        assert np.array_equal(got, oracle.reorder_paper(x, sizes, order, 4)), order


# ----------------------------------------------------------------- interlace
def gpu_interlace(rr, planes, e, off=0):
    n = len(planes)
    count = planes[0].size // e
    dev = [_upload(p, off) for p in planes]
    td, pd = _dev_buf(n * count * e, off)
    st = rr.interlace_raw(pd, [p for _, p in dev], count, e, stream=torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    return _download(td, off, n * count * e)


def gpu_deinterlace(rr, x, n, e, off=0):
    count = x.size // (n * e)
    ts, ps = _upload(x, off)
    outs = [_dev_buf(count * e, off) for _ in range(n)]
    st = rr.deinterlace_raw([p for _, p in outs], ps, count, e, stream=torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    return [_download(t, off, count * e) for t, _ in outs]


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_interlace_deinterlace_small(rr, n):
    for i, (count, e) in enumerate([(1, 4), (37, 1), (64, 4), (129, 2), (256, 8), (50, 16), (33, 3),
                                    (48, 12), (5000, 4), (4099, 1)]):
        _say("interlace", n, count, e)
        planes = [rr_synth.random_bytes(7000 + 100 * n + 10 * i + c, count * e) for c in range(n)]
        off = (i * 5) % 16
        assert np.array_equal(gpu_interlace(rr, planes, e, off), oracle.interlace(planes, e))
        x = rr_synth.random_bytes(8000 + 100 * n + i, n * count * e)
        got = gpu_deinterlace(rr, x, n, e, (i * 3) % 16)
        ref = oracle.deinterlace(x, n, e)
        for c in range(n):
            assert np.array_equal(got[c], ref[c]), (n, count, e, c)


def test_paper_table3_interlace_counts(rr):
    """Table 3's four to nine arrays at 2^24 4-byte elements each (reduced to 2^22 here)."""
    count = 1 << 22
    for n in range(4, 10):
        _say("table3", n)
        planes = [rr_synth.random_bytes(300 + 10 * n + c, count * 4) for c in range(n)]
        joined = gpu_interlace(rr, planes, 4)
        assert np.array_equal(joined, oracle.interlace(planes, 4))
        back = gpu_deinterlace(rr, joined, n, 4)
        assert all(np.array_equal(b, p) for b, p in zip(back, planes))


def test_flat_read_and_merged_store_paths(rr):
    """Aligned interlace shapes that take the flat-read and merged-store paths (the
    LDS tile, with the register path switched off)."""
    rr.set_tile_override(weave=False)
    try:
        for n, e in [(2, 4), (4, 1), (3, 4), (8, 2), (2, 8), (16, 1), (5, 4)]:
            count = 3 * 4096 + 48
            _say("flat/merge", n, e)
            planes = [rr_synth.random_bytes(9300 + 10 * n + c, count * e) for c in range(n)]
            assert np.array_equal(gpu_interlace(rr, planes, e), oracle.interlace(planes, e))
            x = rr_synth.random_bytes(9400 + n, n * count * e)
            got = gpu_deinterlace(rr, x, n, e)
            ref = oracle.deinterlace(x, n, e)
            assert all(np.array_equal(g, r) for g, r in zip(got, ref)), (n, e)
        # permutes whose input tile is one contiguous range of short rows
        for i, (dims, perm, e) in enumerate([((4096, 3), (1, 0), 4), ((64, 48, 6), (2, 0, 1), 2),
                                             ((2048, 5, 2), (1, 2, 0), 8)]):
            assert i == 2 or int(rr.plan_describe(dims, perm, e, 1 << 20, 1 << 30)["flags"]) & 4, dims
            check_permute(rr, dims, perm, e, 9500 + i)
    finally:
        rr.set_tile_override()


def test_short_output_rows_line_fill(rr):
    """Interlace-shaped permutes and interlaces of 2..16 sets of 1..8-byte elements,
    whose micro-tile edge the planner picks by store line fill, over several tiles."""
    from tests.test_emulated_kernels import SHORT_ROW_G
    count = 4104
    rr.set_tile_override(weave=False)   # the tile path (most of these fit the register interlace)
    try:
        for (e, n), g in SHORT_ROW_G.items():
            assert rr.plan_describe((n, count), (1, 0), e, 1 << 30, 1 << 31)["g"] == str(g)
            check_permute(rr, (n, count), (1, 0), e, 9600 + 17 * n + e)
            _say("interlace line fill", n, e)
            planes = [rr_synth.random_bytes(9700 + 17 * n + e + 1000 * c, count * e) for c in range(n)]
            assert np.array_equal(gpu_interlace(rr, planes, e), oracle.interlace(planes, e)), (n, e)
    finally:
        rr.set_tile_override()


@pytest.mark.parametrize("e", [1, 2, 4, 8])
def test_register_interlace(rr, e):
    """Interlace and de-interlace of 2-8 sets on 16-byte boundaries with a whole number
    of 16-byte vectors each, through the register path where the planner picks it;
    bit-exact with the joined side as planned, streamed or through the caches, over
    several workgroups plus a partial one and at 2^16 + 3 vectors per set."""
    base = 1 << 40   # describe only reads pointer values
    try:
        for cache in (None, 0, 3):
            rr.set_tile_override(cache=cache)
            for n in range(2, 9):
                for nvec in (773, (1 << 16) + 3):
                    count = nvec * 16 // e
                    pb = count * e
                    fake = [base + n * pb + (c + 1) * (pb + 4096) for c in range(n)]
                    for de in (False, True):
                        d = rr.interlace_describe(base, fake, count, e, de)
                        if d["class"] == "weave":
                            assert d["cached"] == ("1" if cache == 3 or (cache is None and not de and n % 2)
                                                   else "0"), (cache, d)
                    _say("register interlace", cache, n, nvec, e)
                    planes = [rr_synth.random_bytes(12000 + 100 * n + 10 * e + c, pb) for c in range(n)]
                    assert np.array_equal(gpu_interlace(rr, planes, e), oracle.interlace(planes, e)), (n, e)
                    x = rr_synth.random_bytes(12500 + 100 * n + e, n * pb)
                    got = gpu_deinterlace(rr, x, n, e)
                    assert all(np.array_equal(g, r) for g, r in zip(got, oracle.deinterlace(x, n, e))), (n, e)
    finally:
        rr.set_tile_override()


def test_register_interlace_permutes(rr):
    """Small-axis transposes, batched or not, through the register interlace (and at
    a 4-byte offset through the tile), bit-exact."""
    from tests.test_emulated_kernels import WEAVE_PERMUTES
    for i, (dims, perm, e, kind) in enumerate(WEAVE_PERMUTES):
        assert rr.plan_describe(dims, perm, e, 1 << 30, 1 << 31)["class"] == kind, (dims, perm, e)
        check_permute(rr, dims, perm, e, 12600 + i)
        check_permute(rr, dims, perm, e, 12700 + i, 4, 4)


def test_flat_read_byte_tail(rr):
    """Inputs that end inside a 16-byte vector: the flat read's last tile copies its
    final bytes one by one."""
    for n, e in [(3, 1), (5, 1), (6, 1), (3, 2), (5, 2), (3, 4), (5, 4), (7, 8)]:
        count = 2 * 4096 + 1 + 2 * n
        assert int(rr.plan_describe((count, n), (1, 0), e, 1 << 30, 1 << 31)["flags"]) & 4
        check_permute(rr, (count, n), (1, 0), e, 9800 + 10 * n + e)
        _say("deinterlace byte tail", n, e)
        x = rr_synth.random_bytes(9900 + 10 * n + e, n * count * e)
        got = gpu_deinterlace(rr, x, n, e)
        assert all(np.array_equal(g, r) for g, r in zip(got, oracle.deinterlace(x, n, e))), (n, e)


def test_autotuned_plans_stay_exact(rr):
    """Tuning runs every candidate shape; the cached winner must still be bit-exact."""
    try:
        for i, (dims, perm, e) in enumerate([((512, 384), (1, 0), 4), ((96, 80, 72), (2, 0, 1), 1),
                                             ((32, 32, 32, 32), (3, 1, 0, 2), 2), ((300, 7, 50), (2, 1, 0), 8)]):
            _say("tune", dims, perm, e)
            x = rr_synth.random_bytes(700 + i, int(np.prod(dims)) * e)
            ts, ps = _upload(x)
            td, pd = _dev_buf(x.size)
            best, default = rr.tune_permute(pd, ps, dims, perm, e, torch.cuda.current_stream().cuda_stream)
            assert best > 0 and default >= best * 0.999
            td.zero_()
            rr.check(rr.permute_raw(pd, ps, dims, perm, e, torch.cuda.current_stream().cuda_stream))
            torch.cuda.synchronize()
            assert np.array_equal(_download(td, 0, x.size), oracle.permute(x, dims, perm, e))
    finally:
        rr.tune_clear()


def test_ragged_and_flat_output_paths(rr):
    """Odd extents take the ragged 16-byte row paths (unaligned vectors); three-set
    interlace takes the flat output path."""
    for i, (dims, perm, e, so, do) in enumerate([((1001, 999), (1, 0), 4, 0, 0), ((257, 131), (1, 0), 2, 0, 0),
                                                 ((33, 45, 77), (2, 0, 1), 8, 0, 0), ((17, 19, 23), (1, 2, 0), 1, 0, 0),
                                                 ((301, 299), (1, 0), 2, 2, 6), ((45, 17, 3, 29), (3, 0, 2, 1), 4, 4, 12),
                                                 ((999, 1001), (1, 0), 1, 1, 3), ((63, 65, 67), (2, 1, 0), 2, 0, 2)]):
        check_permute(rr, dims, perm, e, 9600 + i, soff=so, doff=do)
    count = 5000 + 7
    planes = [rr_synth.random_bytes(9610 + c, count * 4) for c in range(3)]
    assert np.array_equal(gpu_interlace(rr, planes, 4), oracle.interlace(planes, 4))
    x = rr_synth.random_bytes(9620, 3 * count * 4)
    got = gpu_deinterlace(rr, x, 3, 4)
    assert all(np.array_equal(g, r) for g, r in zip(got, oracle.deinterlace(x, 3, 4)))


@pytest.mark.parametrize("max_g", [16, 8, 4, 2, 1])
def test_micro_tile_caps(rr, max_g):
    """Every micro-tile edge the planner or tuner can choose, at each unit size,
    with several tiles per launch and partial last tiles."""
    rr.set_tile_override(max_g=max_g)
    try:
        for i, (dims, perm, e) in enumerate([((1024, 1040), (1, 0), 1), ((320, 272, 48), (2, 0, 1), 2),
                                             ((96, 80, 160), (1, 2, 0), 4), ((64, 48, 112), (2, 1, 0), 8),
                                             ((48, 16, 32, 80), (3, 1, 0, 2), 1)]):
            check_permute(rr, dims, perm, e, 9700 + 10 * max_g + i)
    finally:
        rr.set_tile_override()


def test_forced_ragged_on_aligned_shapes(rr):
    """The ragged row paths give the oracle's bytes where micro-tiles would be chosen."""
    rr.set_tile_override(force_ragged=True)
    try:
        for i, (dims, perm, e) in enumerate([((1024, 1040), (1, 0), 1), ((320, 272, 48), (2, 0, 1), 2),
                                             ((96, 80, 160), (1, 2, 0), 4), ((64, 48, 112), (2, 1, 0), 8)]):
            check_permute(rr, dims, perm, e, 9800 + i)
    finally:
        rr.set_tile_override()


def test_stacked_small_transposes(rr):
    """Batches of small transposes along a leading axis share tiles (stacked
    mode), including the shapes of the uneven-job workload's worst cases."""
    from tests.test_emulated_kernels import STACKED_CASES
    cases = list(STACKED_CASES) + [((487424, 3, 3), (0, 2, 1), 2), ((225498, 4, 6), (0, 2, 1), 8),
                                   ((454, 63, 2, 120), (1, 0, 3, 2), 4), ((20480, 2, 2), (0, 2, 1), 2)]
    for i, (dims, perm, e) in enumerate(cases):
        d = rr.plan_describe(dims, perm, e, 1 << 20, 1 << 30)
        assert int(d["flags"]) & 128, (dims, d)
        check_permute(rr, dims, perm, e, 9900 + i)


CACHE_CASES = [((1001, 999), (1, 0), 4), ((777, 345, 9), (1, 2, 0), 8), ((3001, 257), (1, 0), 2),
               ((301, 203, 41), (2, 0, 1), 1), ((139, 100, 12), (2, 1, 0), 16), ((512, 256, 64), (0, 2, 1), 4),
               ((20000, 3, 3), (0, 2, 1), 2), ((96, 100, 104), (0, 2, 1), 1)]


@pytest.mark.parametrize("xcd", [False, True])
@pytest.mark.parametrize("cache", [0, 1, 2, 3])
def test_cache_policies(rr, cache, xcd):
    """Every global-access flavour (non-temporal / cached loads / cached stores /
    both), with and without XCD tile ranges, gives the oracle's bytes: single
    permutes (aligned, odd and stacked shapes), interlace and de-interlace, and a
    batch of uneven jobs."""
    rr.set_tile_override(cache=cache, xcd=xcd)
    try:
        for i, (dims, perm, e) in enumerate(CACHE_CASES):
            f = int(rr.plan_describe(dims, perm, e, 1 << 20, 1 << 30)["flags"])
            assert (f >> 10) & 3 == cache and bool(f & 256) == xcd, (dims, f)
            check_permute(rr, dims, perm, e, 9960 + i)
        for n, count, e in [(3, 5007, 4), (4, 4099, 1), (8, 3000, 2)]:
            _say("interlace cache", cache, xcd, n, count, e)
            planes = [rr_synth.random_bytes(9970 + 10 * n + c, count * e) for c in range(n)]
            assert np.array_equal(gpu_interlace(rr, planes, e), oracle.interlace(planes, e))
            x = rr_synth.random_bytes(9980 + n, n * count * e)
            got = gpu_deinterlace(rr, x, n, e)
            assert all(np.array_equal(g, r) for g, r in zip(got, oracle.deinterlace(x, n, e)))
        _say("batched cache", cache, xcd)
        from tests.test_gpu_batched import Jobs, _check_all_vs_oracle, _uneven
        J = Jobs(rr, _uneven(7 + cache, 120, 20000), 7 + cache)
        rr.check(rr.permute_batched_raw(J.arr, len(J.specs), torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        _check_all_vs_oracle(J)
    finally:
        rr.set_tile_override()


@pytest.mark.parametrize("xcd", [False, True])
def test_diagonal_tile_order(rr, xcd):
    """Diagonal tile order (with and without XCD ranges) gives the oracle's bytes on
    tile grids of two and three axes with partial tiles (a one-axis grid has no
    diagonal and keeps plain order)."""
    rr.set_tile_override(diag=True, xcd=xcd)
    try:
        for i, (dims, perm, e) in enumerate([((1000, 1000), (1, 0), 4), ((130, 70, 90), (2, 0, 1), 2),
                                             ((64, 48, 40), (1, 2, 0), 8), ((20, 30, 40, 50), (3, 1, 0, 2), 1),
                                             ((2048, 2048), (1, 0), 16)]):
            d = rr.plan_describe(dims, perm, e, 1 << 20, 1 << 30)
            assert bool(int(d["flags"]) & 4096) == (int(d["ngrid"]) >= 2), (dims, d)
            check_permute(rr, dims, perm, e, 9990 + i)
    finally:
        rr.set_tile_override()


FILL_CASES = [((611, 39), (1, 0), 8), ((3, 7, 94, 117), (0, 3, 2, 1), 8), ((257, 131), (1, 0), 2),
              ((1, 1, 427, 81, 15), (1, 4, 0, 2, 3), 4), ((13, 2, 21, 69), (1, 3, 2, 0), 2),
              ((17, 2, 1024, 3, 4), (3, 0, 4, 1, 2), 2), ((1024, 48), (1, 0), 8), ((57, 8, 2, 7), (3, 2, 0, 1), 8),
              ((95, 214, 1, 77), (3, 2, 0, 1), 16), ((333, 71), (1, 0), 1), ((431, 1001, 31), (2, 0, 1), 2),
              ((223, 100, 100, 12), (3, 1, 0, 2), 16), ((559, 1000, 24), (2, 1, 0), 4)]


@pytest.mark.parametrize("fill", [False, True])
def test_fill_refit(rr, fill):
    """Odd extents with and without the fill refit (fewer, fuller tiles: whole short
    axes, even splits), on aligned and offset pointers, give the oracle's bytes."""
    rr.set_tile_override(fill=fill)
    try:
        for i, (dims, perm, e) in enumerate(FILL_CASES):
            check_permute(rr, dims, perm, e, 9900 + i)
            check_permute(rr, dims, perm, e, 9950 + i, soff=e % 16 or 4, doff=(3 * e) % 16 or 12)
    finally:
        rr.set_tile_override()


def test_xcd_tile_ranges(rr):
    """Contiguous tile ranges per XCD give the same bytes (tile counts not a
    multiple of 8 included)."""
    rr.set_tile_override(xcd=True)
    try:
        for i, (dims, perm, e) in enumerate([((1024, 1040), (1, 0), 1), ((320, 272, 48), (2, 0, 1), 2),
                                             ((1001, 999), (1, 0), 4), ((64, 48, 112), (2, 1, 0), 8),
                                             ((20000, 3, 3), (0, 2, 1), 2)]):
            assert int(rr.plan_describe(dims, perm, e, 1 << 20, 1 << 30)["flags"]) & 256
            check_permute(rr, dims, perm, e, 9950 + i)
    finally:
        rr.set_tile_override()


def test_unaligned_micro_tiles(rr):
    """Odd extents and misaligned pointers on G x G micro-tiles with unaligned
    vector accesses (and partial micro-tiles), at several tiles per launch."""
    from tests.test_emulated_kernels import UMT_CASES
    big = [((4095, 4097), (1, 0), e, 0, 0) for e in (1, 2, 4, 8)] + \
          [((255, 257, 259), (2, 1, 0), 4, 0, 0), ((255, 257, 259), (1, 2, 0), 2, 2, 2),
           ((255, 257, 259), (2, 0, 1), 1, 1, 0), ((1000, 999), (1, 0), 8, 8, 16)]
    rr.set_tile_override(umt=1)
    try:
        nu = 0
        for i, (dims, perm, e, so, do) in enumerate(list(UMT_CASES) + big):
            d = rr.plan_describe(dims, perm, e, (1 << 20) + do, (1 << 30) + so)
            nu += bool(int(d["flags"]) & 512)
            check_permute(rr, dims, perm, e, 9960 + i, soff=so, doff=do)
        assert nu >= len(UMT_CASES) + len(big) - 2
        rr.set_tile_override(umt=2)
        for i, (dims, perm, e) in enumerate([((4096, 4096), (1, 0), 4), ((512, 512, 256), (2, 0, 1), 2),
                                             ((64, 128, 128, 64), (0, 3, 1, 2), 1)]):
            assert int(rr.plan_describe(dims, perm, e, 1 << 20, 1 << 30)["flags"]) & 512
            check_permute(rr, dims, perm, e, 9990 + i)
    finally:
        rr.set_tile_override()


def test_unaligned_run_vectors(rr):
    """Output runs of R >= 64 bytes that aligned 16-byte vectors do not fit move as
    unaligned 16-byte vectors, the last of each run overlapping its neighbour."""
    from tests.test_emulated_kernels import UA_RUN_CASES
    big = [((64, 48, 1001), (1, 0, 2), 1, 3, 5), ((300, 200, 70), (1, 0, 2), 1, 1, 0),
           ((40, 50, 30, 24), (2, 0, 1, 3), 4, 4, 12), ((500, 400, 9), (1, 0, 2), 8, 8, 0)]
    for i, (dims, perm, e, so, do) in enumerate(list(UA_RUN_CASES) + big):
        check_permute(rr, dims, perm, e, 9700 + i, soff=so, doff=do)
    for dims, perm, e, so, do in big:
        d = rr.plan_describe(dims, perm, e, (1 << 20) + do, (1 << 30) + so)
        assert d["class"] == "run" and d["vec"] == "16" and d["ua"] == "1", d
