"""CPU runs of the library's kernel bodies (planner + per-thread code) against the oracle.

The emulator executes every workgroup and thread of each launch on the host
under AddressSanitizer, so these tests prove the GPU index arithmetic stays in
bounds and produces the oracle's bytes, for the same plans the GPU runs.
"""
import itertools

import numpy as np
import pytest

import oracle
import rr_synth
from tests import emu_runner


def _perm_job(dims, perm, e, seed, **kw):
    n = int(np.prod(dims, dtype=np.int64)) * e
    return dict(op="permute", dims=tuple(dims), perm=tuple(perm), esize=e,
                input=rr_synth.random_bytes(seed, n), **kw)


def _check(jobs):
    res = emu_runner.run(jobs)
    for j, (status, out) in zip(jobs, res):
        assert status.startswith("ok"), (j.get("dims"), j.get("perm"), status)
        if j["op"] == "permute":
            ref = oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])
            assert np.array_equal(out, ref), (j["dims"], j["perm"], j["esize"], j.get("src_off"),
                                              j.get("dst_off"), status)
        elif j["op"] == "interlace":
            ref = oracle.interlace(j["planes"], j["esize"])
            assert np.array_equal(out, ref), (j["n"], j["count"], j["esize"], status)
        else:
            ref = oracle.deinterlace(j["input"], j["n"], j["esize"])
            for c in range(j["n"]):
                assert np.array_equal(out[c], ref[c]), (j["n"], j["count"], j["esize"], c, status)
    return res


def test_emu_brute_force_small_ranks():
    """Every permutation of ranks 1-4 on odd extents, several element sizes and misalignments."""
    jobs = []
    shapes = {1: (7,), 2: (5, 3), 3: (3, 5, 2), 4: (2, 3, 1, 5)}
    seed = 0
    for nd, dims in shapes.items():
        for perm in itertools.permutations(range(nd)):
            for e in (1, 2, 3, 4, 8, 12, 16):
                seed += 1
                jobs.append(_perm_job(dims, perm, e, seed, src_off=seed % 16, dst_off=(seed * 7) % 16))
    _check(jobs)


def test_emu_rank5_all_perms_aligned():
    jobs = []
    for i, perm in enumerate(itertools.permutations(range(5))):
        e = (1, 2, 4, 8, 16)[i % 5]
        jobs.append(_perm_job((2, 3, 2, 4, 2), perm, e, 1000 + i))
    _check(jobs)


@pytest.mark.parametrize("e", [1, 2, 4, 8, 16])
def test_emu_wide_vectors_and_partial_tiles(e):
    """Extents that are multiples of 16 (full 16-byte micro-tiles) plus ragged tails."""
    jobs = []
    cases = [((48, 80), (1, 0)), ((272, 48), (1, 0)), ((32, 48, 64), (2, 1, 0)),
             ((32, 48, 64), (1, 2, 0)), ((32, 48, 64), (2, 0, 1)), ((16, 32, 48), (0, 2, 1)),
             ((33, 47), (1, 0)), ((129, 3, 65), (2, 1, 0)), ((16, 16, 16, 16), (0, 3, 1, 2)),
             ((16, 16, 16, 16), (0, 2, 3, 1)), ((8, 8, 8, 8, 8), (4, 2, 0, 3, 1))]
    for i, (dims, perm) in enumerate(cases):
        jobs.append(_perm_job(dims, perm, e, 2000 + i))
        jobs.append(_perm_job(dims, perm, e, 3000 + i, src_off=e % 16 or 4, dst_off=8))
    _check(jobs)


def test_emu_multi_axis_tiles_small_extents():
    """Short fastest axes force several axes per tile side (5-D 16^5, odd minor extents)."""
    jobs = []
    for i, (dims, perm) in enumerate([((16, 16, 16, 16, 16), (4, 2, 0, 3, 1)),
                                      ((9, 7, 5, 3), (3, 2, 1, 0)),
                                      ((4, 100, 3, 6), (1, 3, 0, 2)),
                                      ((2, 3, 64, 3, 2), (2, 4, 0, 3, 1)),
                                      ((1000, 3), (1, 0)), ((3, 1000), (1, 0))]):
        for e in (1, 2, 4):
            jobs.append(_perm_job(dims, perm, e, 4000 + 10 * i + e))
    _check(jobs)


def test_emu_tile_overrides_and_orders():
    """Autotuner search space: every row-size pair and both tile traversal orders."""
    jobs = []
    k = 0
    for rbi, rbo in [(64, 64), (128, 512), (512, 128), (1024, 64), (64, 1024), (2048, 2048)]:
        for order in (0, 1):
            for dims, perm, e in [((96, 80), (1, 0), 1), ((40, 24, 48), (2, 0, 1), 4),
                                  ((40, 24, 48), (1, 2, 0), 2), ((20, 36, 16), (2, 1, 0), 8),
                                  ((17, 31), (1, 0), 16), ((12, 12, 12, 12), (3, 1, 2, 0), 12)]:
                k += 1
                jobs.append(_perm_job(dims, perm, e, 5000 + k, in_rb=rbi, out_rb=rbo, order=order))
    _check(jobs)


@pytest.mark.parametrize("max_g", [16, 8, 4, 2, 1])
def test_emu_micro_tile_caps(max_g):
    """Every micro-tile edge the planner or tuner can choose, for every unit size,
    with tiles that end part-way through a micro-tile row."""
    jobs = []
    k = 0
    for dims, perm, e in [((96, 80), (1, 0), 1), ((64, 48, 40), (2, 0, 1), 2), ((48, 40, 32), (1, 2, 0), 4),
                          ((32, 24, 16), (2, 1, 0), 8), ((96, 16, 80), (2, 1, 0), 1), ((16, 16, 16, 16), (3, 1, 0, 2), 2)]:
        for rb in ((0, 0), (128, 128), (512, 64)):
            k += 1
            jobs.append(_perm_job(dims, perm, e, 7000 + 31 * max_g + k, in_rb=rb[0], out_rb=rb[1], max_g=max_g))
    res = _check(jobs)
    gs = {dict(t.split("=", 1) for t in st.split()[1:] if "=" in t)["g"] for st, _ in res}
    assert str(max_g) in gs


def test_emu_forced_ragged_on_aligned_shapes():
    """The ragged row paths give the oracle's bytes on shapes that would take micro-tiles."""
    jobs = []
    for i, (dims, perm, e) in enumerate([((96, 80), (1, 0), 1), ((64, 48, 40), (2, 0, 1), 2),
                                         ((48, 40, 32), (1, 2, 0), 4), ((32, 24, 16), (2, 1, 0), 8)]):
        jobs.append(_perm_job(dims, perm, e, 7500 + i, ragged=True))
    res = _check(jobs)
    for st, _ in res:
        flags = int(dict(t.split("=", 1) for t in st.split()[1:] if "=" in t)["flags"])
        assert flags & 16 and flags & (32 | 64), st


STACKED_CASES = [((1000, 3, 3), (0, 2, 1), 2), ((2000, 4, 6), (0, 2, 1), 8), ((777, 5, 7), (0, 2, 1), 1),
                 ((3000, 2, 2), (0, 2, 1), 4), ((100, 17, 13), (0, 2, 1), 8), ((50, 64, 48), (0, 2, 1), 1),
                 ((5, 7, 3, 4), (1, 0, 3, 2), 4), ((6, 50, 9, 11), (1, 0, 3, 2), 2),
                 ((3, 4, 40, 5, 6), (2, 0, 1, 4, 3), 1), ((9, 11, 30, 2, 3), (0, 2, 1, 4, 3), 8)]


def test_emu_stacked_small_transposes():
    """Last two axes swapped and small: several whole transposes share a tile,
    read as one contiguous range; written as one range (C also next in the
    output) or one run per transpose; partial last tile along C."""
    jobs = [_perm_job(d, p, e, 7800 + i) for i, (d, p, e) in enumerate(STACKED_CASES)]
    res = _check(jobs)
    for st, _ in res:
        kv = dict(t.split("=", 1) for t in st.split()[1:] if "=" in t)
        assert int(kv["flags"]) & 128 and int(kv["tc"]) > 1, st


def test_emu_stacked_in_batches_and_chunks():
    """Stacked tiles inside a batch, whole and cut into workgroup ranges."""
    sub = [_perm_job(d, p, e, 7900 + i) for i, (d, p, e) in enumerate(STACKED_CASES[:6])]
    sub.append(_perm_job((40, 24, 48), (2, 0, 1), 4, 7990))
    for chunk in (0, 3):
        res = emu_runner.run([dict(op="batched", jobs=sub, chunk=chunk)])
        st, outs = res[0]
        assert st.startswith("ok"), st
        for j, o in zip(sub, outs):
            assert np.array_equal(o, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), (j["dims"], chunk)


def test_emu_xcd_tile_ranges():
    """Tiles handed out as one contiguous range per XCD cover every tile once
    (the emulator checks the block -> tile map is a bijection), for tile counts
    below, at and above a multiple of 8."""
    jobs = []
    for i, (dims, perm, e) in enumerate([((96, 80), (1, 0), 1), ((64, 48, 40), (2, 0, 1), 2),
                                         ((300, 37), (1, 0), 4), ((32, 24, 16), (2, 1, 0), 8),
                                         ((1000, 3, 3), (0, 2, 1), 2), ((130, 130), (1, 0), 4)]):
        jobs.append(_perm_job(dims, perm, e, 7700 + i, xcd=True, in_rb=64, out_rb=64))
    res = _check(jobs)
    for st, _ in res:
        assert int(dict(t.split("=", 1) for t in st.split()[1:] if "=" in t)["flags"]) & 256, st


UMT_CASES = [((1001, 999), (1, 0), 4, 0, 0), ((257, 131), (1, 0), 2, 0, 0), ((33, 45, 77), (2, 0, 1), 8, 0, 0),
             ((17, 19, 23), (1, 2, 0), 1, 0, 0), ((301, 299), (1, 0), 2, 2, 6), ((45, 17, 3, 29), (3, 0, 2, 1), 4, 0, 0),
             ((96, 80), (1, 0), 4, 4, 8), ((64, 48, 40), (2, 0, 1), 1, 1, 3), ((9, 7, 33, 13), (2, 3, 1, 0), 2, 0, 0),
             ((5, 16, 11, 24), (0, 3, 2, 1), 1, 0, 0), ((129, 67), (1, 0), 8, 8, 0), ((31, 37, 41), (2, 1, 0), 1, 0, 0)]


def test_emu_diagonal_tile_order():
    """Diagonal tile order (second-fastest tile coordinate skewed by the fastest)
    covers every tile once: tile grids of 2-4 axes, partial tiles, both traversal
    orders, with and without XCD ranges."""
    jobs = []
    cases = [((1000, 1000), (1, 0), 4), ((130, 70, 90), (2, 0, 1), 2), ((64, 48, 40), (1, 2, 0), 8),
             ((20, 30, 40, 50), (3, 1, 0, 2), 1), ((33, 47), (1, 0), 16), ((512, 384), (1, 0), 1)]
    for i, (dims, perm, e) in enumerate(cases):
        for order in (0, 1):
            for xcd in (False, True):
                jobs.append(_perm_job(dims, perm, e, 7600 + 10 * i + 2 * order + xcd, diag=True, order=order,
                                      xcd=xcd, in_rb=64, out_rb=64))
    res = _check(jobs)
    assert any(int(st.split("flags=")[1].split()[0]) & 4096 for st, _ in res)


FILL_CASES = [((611, 39), (1, 0), 8), ((3, 7, 94, 117), (0, 3, 2, 1), 8), ((257, 131), (1, 0), 2),
              ((1, 1, 427, 81, 15), (1, 4, 0, 2, 3), 4), ((13, 2, 21, 69), (1, 3, 2, 0), 2),
              ((17, 2, 1024, 3, 4), (3, 0, 4, 1, 2), 2), ((1024, 48), (1, 0), 8), ((57, 8, 2, 7), (3, 2, 0, 1), 8),
              ((95, 214, 1, 77), (3, 2, 0, 1), 16), ((333, 71), (1, 0), 1)]


def test_emu_fill_refit():
    """Odd extents refit for fewer, fuller tiles (whole short axes, even splits) move
    every element once, with the refit on and off, on aligned and offset pointers."""
    def ntiles(st):
        return int(st.split("ntiles=")[1].split()[0])

    jobs = []
    for i, (dims, perm, e) in enumerate(FILL_CASES):
        for fill in (False, True):
            jobs.append(_perm_job(dims, perm, e, 7700 + 2 * i + fill, fill=fill))
            jobs.append(_perm_job(dims, perm, e, 7750 + 2 * i + fill, fill=fill,
                                  src_off=e % 16 or 4, dst_off=(3 * e) % 16 or 12))
    res = _check(jobs)
    fewer = 0
    for k in range(0, len(res), 4):
        off_plain, on_plain = ntiles(res[k][0]), ntiles(res[k + 2][0])
        assert on_plain <= off_plain, (FILL_CASES[k // 4], res[k][0], res[k + 2][0])
        fewer += on_plain * 8 <= off_plain * 7
    assert fewer >= len(FILL_CASES) // 2, fewer


def test_emu_unaligned_micro_tiles():
    """Odd extents and misaligned pointers keep G x G micro-tiles with unaligned
    vector accesses; partial micro-tiles at tile edges move element by element."""
    jobs = [_perm_job(d, p, e, 9650 + i, src_off=so, dst_off=do, umt=1) for i, (d, p, e, so, do) in enumerate(UMT_CASES)]
    res = _check(jobs)
    flags = [int(st.split("flags=")[1].split()[0]) for st, _ in res]
    assert sum(bool(f & 512) for f in flags) >= len(flags) - 2, flags
    # multi-axis A sides, tiles whose extents G does not divide
    assert any(f & 512 and int(st.split("nA=")[1].split()[0]) > 1 for f, (st, _) in zip(flags, res)), res
    for rb in ((64, 64), (512, 128)):
        _check([_perm_job(d, p, e, 9680 + i, src_off=so, dst_off=do, in_rb=rb[0], out_rb=rb[1], umt=1)
                for i, (d, p, e, so, do) in enumerate(UMT_CASES)])
    # everywhere, aligned shapes included
    res = _check([_perm_job(d, p, e, 9690 + i, umt=2) for i, (d, p, e) in enumerate(
        [((96, 80), (1, 0), 1), ((64, 48, 40), (2, 0, 1), 2), ((48, 40, 32), (1, 2, 0), 4), ((32, 24, 16), (2, 1, 0), 8)])])
    assert all(int(st.split("flags=")[1].split()[0]) & 512 for st, _ in res), res


def test_emu_unaligned_micro_tiles_in_batches():
    jobs = [_perm_job(d, p, e, 9700 + i) for i, (d, p, e, so, do) in enumerate(UMT_CASES)]
    for chunk in (0, 2):
        st, outs = emu_runner.run([dict(op="batched", jobs=jobs, chunk=chunk, umt=1)])[0]
        assert st.startswith("ok"), st
        for j, o in zip(jobs, outs):
            assert np.array_equal(o, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), (j["dims"], chunk)


def _reorder_job(dims, base, range_, order, e, seed, **kw):
    n = int(np.prod(dims, dtype=np.int64)) * e
    return dict(op="reorder", dims=tuple(dims), base=tuple(base), range=tuple(range_), order=tuple(order), esize=e,
                input=rr_synth.random_bytes(seed, n), **kw)


def random_boxes(seed, count, max_rank=5, max_dim=40, max_in_bytes=4 << 20):
    """Random N-to-M reorders: rank 1..max_rank, a random subset and order of kept
    axes, random base and range inside each extent (fixed axes at a random index);
    inputs of at most max_in_bytes at 16-byte elements."""
    g = rr_synth.rng(seed)
    out = []
    for _ in range(count):
        nd = int(g.integers(1, max_rank + 1))
        dims = [int(g.integers(1, max_dim + 1)) for _ in range(nd)]
        while int(np.prod(dims)) * 16 > max_in_bytes:
            k = int(np.argmax(dims))
            dims[k] = max(1, dims[k] // 2)
        m = int(g.integers(0, nd + 1))
        order = [int(v) for v in g.permutation(nd)[:m]]
        base, rng = [], []
        for d in range(nd):
            b = int(g.integers(0, dims[d]))
            if d in order:
                b = int(g.integers(0, max(1, dims[d] // 3)))
                rng.append(int(g.integers(1, dims[d] - b + 1)))
            else:
                rng.append(1)
            base.append(b)
        out.append((dims, base, rng, order, int(g.choice([1, 2, 4, 8, 3, 12]))))
    return out


REORDER_CASES = [((5, 7, 3), (1, 2, 0), (3, 4, 3), (1, 0, 2), 4), ((6, 8), (1, 2), (4, 5), (1, 0), 2),
                 ((4, 5, 6), (0, 1, 2), (4, 1, 3), (2, 0), 1), ((4, 5, 6), (1, 1, 1), (1, 1, 1), (), 8),
                 ((3, 4, 5, 6), (0, 1, 0, 2), (3, 2, 5, 1), (2, 0, 1), 4), ((8, 9), (0, 3), (8, 1), (0,), 4),
                 ((10, 4), (0, 0), (10, 4), (0, 1), 2), ((70, 90, 4), (3, 5, 1), (60, 80, 1), (1, 0), 4),
                 ((64, 96, 3), (0, 0, 0), (64, 96, 3), (2, 0, 1), 2), ((40, 50, 60), (2, 3, 4), (30, 40, 50), (2, 1, 0), 1),
                 ((128, 130), (1, 1), (120, 127), (1, 0), 8), ((9, 40, 33, 8), (1, 2, 3, 0), (7, 30, 28, 8), (3, 1, 2, 0), 2)]


def test_emu_reorder_boxes():
    """N-to-M reorders (Sec. III.B's base and range): tiled boxes, gathered boxes
    (innermost axis dropped or cut), copies, single elements, all against the oracle."""
    jobs = [_reorder_job(*c[:4], c[4], 8100 + i) for i, c in enumerate(REORDER_CASES)]
    jobs += [_reorder_job(d, b, r, o, e, 8200 + i) for i, (d, b, r, o, e) in enumerate(random_boxes(77, 80))]
    res = emu_runner.run(jobs)
    classes = set()
    for j, (st, out) in zip(jobs, res):
        assert st.startswith("ok"), (j["dims"], j["base"], j["range"], j["order"], st)
        ref = oracle.reorder_slice(j["input"], j["dims"], j["base"], j["range"], j["order"], j["esize"])
        assert np.array_equal(out, ref), (j["dims"], j["base"], j["range"], j["order"], j["esize"], st)
        classes.add(st.split("class=")[1].split()[0])
    assert {"tile", "run", "copy"} <= classes, classes


def test_emu_reorder_offsets_and_unaligned_micro_tiles():
    jobs = [_reorder_job(*c[:4], c[4], 8300 + i, src_off=3, dst_off=5) for i, c in enumerate(REORDER_CASES)]
    jobs += [_reorder_job(*c[:4], c[4], 8400 + i, umt=1) for i, c in enumerate(REORDER_CASES)]
    for j, (st, out) in zip(jobs, emu_runner.run(jobs)):
        assert st.startswith("ok"), st
        ref = oracle.reorder_slice(j["input"], j["dims"], j["base"], j["range"], j["order"], j["esize"])
        assert np.array_equal(out, ref), (j["dims"], j["base"], j["range"], j["order"], st)


SELECT_CASES = [
    # one channel of interleaved records: (dims, base, range, order, element bytes)
    ((64, 96, 4), (0, 0, 2), (64, 96, 1), (0, 1), 1),          # RGBA plane, fused to one row
    ((64, 96, 4), (0, 0, 3), (64, 96, 1), (0, 1), 1),          # last channel: the span ends at the buffer's end
    ((50, 64, 4), (3, 5, 1), (40, 50, 1), (0, 1), 1),          # a crop: rows of 50, not a multiple of 16
    ((33, 17, 3), (0, 0, 1), (33, 17, 1), (0, 1), 4),          # xyz floats, M = 3
    ((40, 37, 2), (0, 0, 1), (40, 37, 1), (0, 1), 8),          # complex doubles, M = 2
    ((7, 9, 11, 4), (1, 0, 2, 0), (5, 9, 9, 1), (1, 0, 2), 2),  # outer axes transposed
    ((300, 3), (0, 2), (300, 1), (0,), 2),                      # rank-1 output
    ((31, 29, 2), (0, 0, 0), (31, 29, 1), (0, 1), 4),
]


def test_emu_reorder_strided_select():
    """Boxes that keep a strided fastest axis (one component of interleaved
    records) plan to the select kernel and match the oracle, at aligned and
    offset pointers (an offset below the element size falls back to the gather)."""
    jobs = [_reorder_job(*c[:4], c[4], 8600 + i) for i, c in enumerate(SELECT_CASES)]
    jobs += [_reorder_job(*c[:4], c[4], 8700 + i, src_off=c[4] * 3, dst_off=c[4]) for i, c in enumerate(SELECT_CASES)]
    jobs += [_reorder_job(*c[:4], c[4], 8800 + i, src_off=1, dst_off=3) for i, c in enumerate(SELECT_CASES)]
    classes = []
    for j, (st, out) in zip(jobs, emu_runner.run(jobs)):
        assert st.startswith("ok"), st
        ref = oracle.reorder_slice(j["input"], j["dims"], j["base"], j["range"], j["order"], j["esize"])
        assert np.array_equal(out, ref), (j["dims"], j["base"], j["range"], j["order"], st)
        classes.append(st.split("class=")[1].split()[0])
    n = len(SELECT_CASES)
    assert classes[:2 * n] == ["select"] * (2 * n), classes


def test_emu_size_zero_and_one():
    jobs = [_perm_job((0, 5), (1, 0), 4, 1), _perm_job((5, 0, 3), (2, 0, 1), 2, 2),
            _perm_job((1, 1, 1), (2, 1, 0), 8, 3), _perm_job((1,), (0,), 16, 4),
            _perm_job((1, 7, 1, 9), (3, 2, 1, 0), 4, 5), _perm_job((256, 256, 1, 4), (3, 2, 0, 1), 1, 6)]
    _check(jobs)


def test_emu_run_copy_class():
    """Permutes that keep the fastest axis: contiguous runs copied without LDS."""
    jobs = []
    for i, (dims, perm, e) in enumerate([((64, 64, 32), (1, 0, 2), 4), ((8, 9, 10, 64), (2, 0, 1, 3), 2),
                                         ((7, 5, 33), (1, 0, 2), 8), ((3, 4, 5, 6), (2, 1, 0, 3), 16)]):
        jobs.append(_perm_job(dims, perm, e, 6000 + i))
        jobs.append(_perm_job(dims, perm, e, 6100 + i, src_off=3, dst_off=5))
    res = _check(jobs)
    assert any("class=run" in s for s, _ in res)


def test_emu_config1_transpose():
    """1024x1024 transpose of 4-byte elements (the small dense case)."""
    _check([_perm_job((1024, 1024), (1, 0), 4, 77)])


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_emu_interlace_deinterlace(n):
    jobs = []
    for i, (count, e) in enumerate([(1, 4), (37, 1), (64, 4), (129, 2), (256, 8), (50, 16), (33, 3), (48, 12)]):
        planes = [rr_synth.random_bytes(7000 + 100 * n + 10 * i + c, count * e) for c in range(n)]
        jobs.append(dict(op="interlace", n=n, count=count, esize=e, planes=planes, off=(i * 5) % 16))
        jobs.append(dict(op="deinterlace", n=n, count=count, esize=e, off=(i * 3) % 16,
                         input=rr_synth.random_bytes(8000 + 100 * n + i, n * count * e)))
    _check(jobs)


def test_emu_interlace_large_counts():
    """Counts spanning several tiles with ragged tails, the three interlace workloads' shapes."""
    jobs = []
    for n, e in [(2, 4), (4, 1), (3, 4)]:
        count = 3 * 4096 + 17 * (5 - n)
        planes = [rr_synth.random_bytes(9000 + c, count * e) for c in range(n)]
        jobs.append(dict(op="interlace", n=n, count=count, esize=e, planes=planes))
        jobs.append(dict(op="deinterlace", n=n, count=count, esize=e,
                         input=rr_synth.random_bytes(9100 + n, n * count * e)))
    _check(jobs)


def test_emu_flat_read_and_merged_store_paths():
    """Aligned interlace workloads whose plans take the flat-read (de-interlace) and the
    merged 16-byte-store (interlace with G == n) paths."""
    jobs = []
    for n, e in [(2, 4), (4, 1), (3, 4), (8, 2), (2, 8), (16, 1), (5, 4)]:
        count = 3 * 4096 + 48
        planes = [rr_synth.random_bytes(9300 + 10 * n + c, count * e) for c in range(n)]
        jobs.append(dict(op="interlace", n=n, count=count, esize=e, planes=planes, weave=False))
        jobs.append(dict(op="deinterlace", n=n, count=count, esize=e, weave=False,
                         input=rr_synth.random_bytes(9400 + n, n * count * e)))
    res = _check(jobs)
    flags = [int(s.split("flags=")[1].split()[0]) for s, _ in res]
    assert any(f & 4 for f in flags[1::2]), "no de-interlace plan took the flat read"
    assert any(f & 8 for f in flags[0::2]), "no interlace plan took the merged store"
    # permutes whose input tile is one contiguous range of short rows
    jobs = [_perm_job((4096, 3), (1, 0), 4, 9500, weave=False), _perm_job((64, 48, 6), (2, 0, 1), 2, 9501, weave=False),
            _perm_job((2048, 5, 2), (1, 2, 0), 8, 9502, weave=False)]
    assert all(int(s.split("flags=")[1].split()[0]) & 4 for s, _ in _check(jobs)[:2])


# Micro-tile edge the planner keeps for interlace-shaped problems (n short output
# rows of e-byte elements): micro-tiles survive only where a wave's stores still
# fill at least half (1-2-byte elements) or more than half (4-16-byte elements)
# of each line they touch, else G falls back toward the G = 1 vector paths.
SHORT_ROW_G = {(1, 2): 2, (1, 4): 4, (1, 8): 2, (1, 16): 2,
               (2, 2): 2, (2, 4): 4, (2, 8): 2, (2, 16): 2,
               (4, 2): 2, (4, 4): 1, (4, 8): 1, (4, 16): 1,
               (8, 2): 1, (8, 4): 1, (8, 8): 1, (8, 16): 2}


def test_emu_short_output_rows_line_fill():
    """Interlace-shaped permutes and interlaces of 2..16 sets of 1..8-byte elements:
    the planner's micro-tile edge follows the store line-fill rule and every plan
    stays bit-exact (several tiles plus a partial one)."""
    count = 4104
    jobs, keys = [], []
    for (e, n), g in SHORT_ROW_G.items():
        jobs.append(_perm_job((n, count), (1, 0), e, 9600 + 17 * n + e, weave=False))
        planes = [rr_synth.random_bytes(9700 + 17 * n + e + 1000 * c, count * e) for c in range(n)]
        jobs.append(dict(op="interlace", n=n, count=count, esize=e, planes=planes, weave=False))
        keys += [(e, n, g)] * 2
    res = _check(jobs)
    for j, (e, n, g), (status, _) in zip(jobs, keys, res):
        got = int(status.split(" g=")[1].split()[0])
        assert got == g, (e, n, got, g, status)
        if j["op"] == "interlace":   # plane-table plans stream both sides, no XCD ranges
            assert int(status.split("flags=")[1].split()[0]) & (1024 | 2048 | 256) == 0, status


@pytest.mark.parametrize("e", [1, 2, 4, 8])
def test_emu_register_interlace(e):
    """Interlace and de-interlace of 2-8 sets on 16-byte boundaries with a whole number
    of 16-byte vectors per set take the register path where the planner picks it
    (several workgroups plus a partial one) and match the oracle; a misaligned set,
    a partial vector or the override keep the LDS tile, also bit-exact.  Every case
    is planned as the library plans it for aligned pointers."""
    import paper_1011_3583_amd as rr
    base = 1 << 40

    def planned(n, count, de, off):
        pb = count * e
        planes = [base + off + n * pb + (c + 1) * (pb + 4096) for c in range(n)]
        return rr.interlace_describe(base + off, planes, count, e, de)["class"]

    jobs, want = [], []
    for n in range(2, 9):
        for off, count, weave in [(0, 773 * 16 // e, True), (16, 64 * 16 // e + 16 // e, True),
                                  (0, 773 * 16 // e, False), (4, 300 * 16 // e, True), (0, 300 * 16 // e + 1, True)]:
            seed = 11000 + 100 * n + 10 * e + off + count % 7 + int(weave)
            planes = [rr_synth.random_bytes(seed + c, count * e) for c in range(n)]
            jobs.append(dict(op="interlace", n=n, count=count, esize=e, planes=planes, off=off, weave=weave))
            jobs.append(dict(op="deinterlace", n=n, count=count, esize=e, off=off, weave=weave,
                             input=rr_synth.random_bytes(seed + 50, n * count * e)))
            want += [planned(n, count, de, off) if weave else "tile" for de in (False, True)]
    assert want.count("weave") >= 20, want.count("weave")
    res = _check(jobs)
    for j, k, (status, _) in zip(jobs, want, res):
        assert f"class={k}" in status, (j["op"], j["n"], j["count"], j["off"], status)


# Permutes that swap the two fastest axes where one has 2-8 entries, with or
# without a batch axis in front: (dims, perm, element bytes, class).  Whole
# 16-byte vectors per set take the register interlace; a partial vector, nine
# sets or batched sets under 4 KiB keep the tile.
WEAVE_PERMUTES = [((3, 4096), (1, 0), 4, "weave"), ((4096, 3), (1, 0), 4, "weave"),
                  ((2, 24576), (1, 0), 8, "weave"), ((24576, 2), (1, 0), 8, "weave"),
                  ((8, 6208), (1, 0), 1, "weave"), ((6208, 5), (1, 0), 2, "weave"),
                  ((5, 3, 12352), (0, 2, 1), 2, "weave"), ((4, 3072, 7), (0, 2, 1), 4, "weave"),
                  ((3, 4, 2056), (0, 2, 1), 8, "weave"), ((2, 8208, 6), (0, 2, 1), 1, "weave"),
                  ((3, 4097), (1, 0), 4, "tile"), ((9, 4096), (1, 0), 4, "tile"),
                  ((1000, 3, 64), (0, 2, 1), 4, "tile")]


def test_emu_register_interlace_permutes():
    """Small-axis transposes (interlace / de-interlace shaped, batched or not) run the
    register interlace where it applies and match the oracle; at a 4-byte offset
    they take the tile, also bit-exact."""
    jobs, want = [], []
    for i, (dims, perm, e, kind) in enumerate(WEAVE_PERMUTES):
        jobs.append(_perm_job(dims, perm, e, 12600 + i))
        jobs.append(_perm_job(dims, perm, e, 12700 + i, src_off=4, dst_off=4))
        want += [kind, "tile"]
    res = _check(jobs)
    for j, k, (status, _) in zip(jobs, want, res):
        assert f"class={k}" in status, (j["dims"], j.get("src_off"), status)
    batches = [int(st.split("batches=")[1].split()[0]) for (st, _), k in zip(res, want) if k == "weave"]
    assert max(batches) == 5 and min(batches) == 1, batches


def test_emu_flat_read_byte_tail():
    """De-interlace-shaped permutes and de-interlaces whose input is not a whole number
    of 16-byte vectors: tiles read their range as vectors and the last tile's final
    bytes one by one (flat read), bit-exact; a slower axis whose stride is not a
    multiple of 16 bytes keeps the per-row read."""
    jobs = []
    for n, e in [(3, 1), (5, 1), (6, 1), (3, 2), (5, 2), (3, 4), (5, 4), (7, 8)]:
        count = 2 * 4096 + 1 + 2 * n
        jobs.append(_perm_job((count, n), (1, 0), e, 9800 + 10 * n + e))
        jobs.append(dict(op="deinterlace", n=n, count=count, esize=e,
                         input=rr_synth.random_bytes(9900 + 10 * n + e, n * count * e)))
    res = _check(jobs)
    for j, (status, _) in zip(jobs, res):
        assert int(status.split("flags=")[1].split()[0]) & 4, (j.get("dims"), j.get("n"), status)
    res = _check([_perm_job((5, 999, 5), (0, 2, 1), 2, 9990), _perm_job((3, 2001, 3), (0, 2, 1), 1, 9991)])
    for status, _ in res:
        assert not int(status.split("flags=")[1].split()[0]) & 4, status


def _batched_jobs(seed, njobs, max_elems=20000):
    g = rr_synth.rng(seed)
    jobs = []
    for i in range(njobs):
        nd = int(g.integers(1, 6))
        while True:
            dims = tuple(int(g.integers(1, 40)) for _ in range(nd))
            if int(np.prod(dims)) <= max_elems:
                break
        perm = tuple(int(v) for v in g.permutation(nd))
        e = int(g.choice([1, 2, 3, 4, 6, 8, 12, 16]))
        jobs.append(_perm_job(dims, perm, e, seed * 1000 + i))
    return jobs


def test_emu_batched_many_jobs_threaded_planning():
    """1200 small jobs (planned on several host threads, as batches of 256 jobs or
    more are) of every element size and ranks 2-4: each equals the oracle alone."""
    g = rr_synth.rng(4242)
    jobs = []
    for i in range(1200):
        nd = int(g.integers(2, 5))
        dims = tuple(int(x) for x in g.integers(1, 13, nd))
        perm = tuple(int(x) for x in g.permutation(nd))
        jobs.append(_perm_job(dims, perm, int(g.choice([1, 2, 4, 8, 16])), 50000 + i))
    status, outs = emu_runner.run([dict(op="batched", jobs=jobs)])[0]
    assert status.startswith("ok"), status
    for j, out in zip(jobs, outs):
        assert np.array_equal(out, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), \
            (j["dims"], j["perm"], j["esize"])


def test_emu_batched_planning_passes_reuse_the_host_workers():
    """Several batches of 600 jobs in one process, each planned in slices on the
    library's host worker threads: an invalid batch in between reports its lowest
    invalid job (of two, in different slices), and the batches after it still
    plan and run bit-exact."""
    first, second = _batched_jobs(61, 600, 4000), _batched_jobs(62, 600, 4000)
    bad = _batched_jobs(63, 600, 4000)
    for k in (520, 450):   # (0, 0) is not a permutation: job 450 is the lowest invalid one
        bad[k] = _perm_job((2, 3), (0, 0), 4, 9000 + k)
    res = emu_runner.run([dict(op="batched", jobs=first), dict(op="batched", jobs=bad),
                          dict(op="batched", jobs=second)])
    assert res[1][0].startswith("err") and " job 450 " in res[1][0], res[1][0]
    for (status, outs), jobs in ((res[0], first), (res[2], second)):
        assert status.startswith("ok"), status
        for j, out in zip(jobs, outs):
            assert np.array_equal(out, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), \
                (j["dims"], j["perm"], j["esize"])


def test_emu_batched_planning_from_several_threads_at_once():
    """Four host threads plan the same 600-job batch six times each at once, sharing
    the library's planning workers (a pass that finds them busy starts threads of
    its own): every plan equals the single-threaded one byte for byte, and the batch
    runs bit-exact."""
    jobs = _batched_jobs(64, 600, 4000)
    status, outs = emu_runner.run([dict(op="batched", jobs=jobs, chunk=-4)])[0]
    assert status.startswith("ok"), status
    for j, out in zip(jobs, outs):
        assert np.array_equal(out, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), \
            (j["dims"], j["perm"], j["esize"])


@pytest.mark.parametrize("seed,opts", [(1, (0, 0, 0)), (2, (512, 256, 0)), (3, (256, 1024, 1))])
def test_emu_batched_uneven_jobs(seed, opts):
    """A batch of uneven jobs of every kernel family: each job equals the oracle alone."""
    jobs = _batched_jobs(seed, 60)
    jobs.append(_perm_job((0, 4), (1, 0), 4, 5))           # empty job inside a batch
    jobs.append(_perm_job((64, 64, 32), (1, 0, 2), 4, 6))  # run-copy family
    jobs.append(_perm_job((7, 9), (0, 1), 2, 7))           # identity -> copy family
    rbi, rbo, order = opts
    res = emu_runner.run([dict(op="batched", jobs=jobs, in_rb=rbi, out_rb=rbo, order=order)])
    status, outs = res[0]
    assert status.startswith("ok"), status
    assert int(status.split("groups=")[1].split()[0]) >= 3
    for j, out in zip(jobs, outs):
        assert np.array_equal(out, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), \
            (j["dims"], j["perm"], j["esize"])


@pytest.mark.parametrize("chunk", [1, 3])
def test_emu_chunked_entries(chunk):
    """Jobs cut into ranges of their own workgroups, ranges of different jobs
    interleaved in one batch table (how the server spreads a large job)."""
    jobs = _batched_jobs(7 + chunk, 25)
    jobs += [_perm_job((300, 200), (1, 0), 4, 70), _perm_job((64, 64, 32), (1, 0, 2), 4, 71),
             _perm_job((50000,), (0,), 2, 72), _perm_job((40, 30, 20), (2, 1, 0), 8, 73)]
    res = emu_runner.run([dict(op="batched", jobs=jobs, chunk=chunk)])
    status, outs = res[0]
    assert status.startswith("ok"), status
    for j, out in zip(jobs, outs):
        assert np.array_equal(out, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), \
            (j["dims"], j["perm"], j["esize"])


def test_emu_ragged_and_flat_output_paths():
    """Odd extents (no 16-byte micro-tiles possible) take the ragged 16-byte row paths
    (or a flat input range where a refit tile holds whole input rows); interlace of
    three sets takes the flat output path; both stay bit-exact."""
    jobs = [_perm_job((1001, 999), (1, 0), 4, 9600), _perm_job((257, 131), (1, 0), 2, 9601),
            _perm_job((33, 45, 77), (2, 0, 1), 8, 9602), _perm_job((17, 19, 23), (1, 2, 0), 1, 9603),
            _perm_job((301, 299), (1, 0), 2, 9604, src_off=2, dst_off=6),
            _perm_job((45, 17, 3, 29), (3, 0, 2, 1), 4, 9605)]
    res = _check(jobs)
    flags = [int(s.split("flags=")[1].split()[0]) for s, _ in res]
    assert all(f & (16 | 4) and f & (64 | 32) for f in flags), flags
    assert any(f & 16 for f in flags), flags
    assert any(f & 64 for f in flags) and any(f & 32 for f in flags), flags
    count = 5000 + 7
    planes = [rr_synth.random_bytes(9610 + c, count * 4) for c in range(3)]
    res = _check([dict(op="interlace", n=3, count=count, esize=4, planes=planes),
                  dict(op="deinterlace", n=3, count=count, esize=4, input=rr_synth.random_bytes(9620, 3 * count * 4))])
    assert int(res[0][0].split("flags=")[1].split()[0]) & 32


def gather_cases(seed, count):
    """Index sets (uniform, sorted, repeated, with out-of-range entries) and ranges
    (positive, negative, zero strides) over element sizes 1-16."""
    g = rr_synth.rng(seed)
    out = []
    for t in range(count):
        e = int(g.choice([1, 2, 3, 4, 6, 8, 12, 16]))
        n = int(g.integers(1, 3000))
        kind = t % 4
        if kind == 0:
            idx = g.integers(0, n, int(g.integers(1, 5000)))
        elif kind == 1:
            idx = np.sort(g.integers(0, n, int(g.integers(1, 5000))))
        elif kind == 2:
            idx = g.integers(-3, n + 3, int(g.integers(1, 3000)))   # some rejected
        else:
            idx = None
        if idx is not None:
            out.append(dict(op="gather", src_count=n, esize=e, idx=idx.astype(np.int64),
                            input=rr_synth.random_bytes(9000 + t, n * e)))
        else:
            start = int(g.integers(0, n))
            stride = int(g.choice([1, 2, 3, -1, -2, 0, 7]))
            if stride > 0:
                cnt = (n - 1 - start) // stride + 1
            elif stride < 0:
                cnt = start // -stride + 1
            else:
                cnt = int(g.integers(1, 100))
            out.append(dict(op="gather", src_count=n, esize=e, start=start, stride=stride, count=cnt,
                            input=rr_synth.random_bytes(9000 + t, n * e)))
    return out


def gather_ref(j):
    e = j["esize"]
    if "idx" in j:
        idx = j["idx"]
        ok = (idx >= 0) & (idx < j["src_count"])
        ref = oracle.gather(j["input"], np.where(ok, idx, 0), e).reshape(-1, e)
        ref[~ok] = 0
        return ref.reshape(-1), int((~ok).sum())
    return oracle.copy_range(j["input"], j["start"], j["stride"], j["count"], e), 0


def test_emu_gather_and_range():
    """Index-set and range reads (Sec. III.A) against the oracle; rejected indices
    read as zeros and are counted."""
    jobs = gather_cases(5, 120)
    jobs[3]["src_off"], jobs[3]["dst_off"] = 3, 5
    for j, (st, out) in zip(jobs, emu_runner.run(jobs)):
        assert st.startswith("ok"), st
        ref, nbad = gather_ref(j)
        assert np.array_equal(out, ref), (j.get("start"), j.get("stride"), j["esize"], st)
        assert int(st.split("bad=")[1]) == nbad, st


def stencil_tolerance(x, radius, weights, shape):
    """Per-point bound on |fp32 result - exact|: the fp32 evaluation of n products
    (n = 4r + 1 for a star, (2r + 1)^2 for a box) and the final rounding add at most
    (n + 2) * 2^-24 * sum |w * x| over the stencil's points."""
    from scipy import ndimage
    r = radius
    n = 4 * r + 1 if shape == 0 else (2 * r + 1) ** 2
    w = np.abs(np.asarray(weights, dtype=np.float32).astype(np.float64))
    if shape == 0:
        k = np.zeros((2 * r + 1, 2 * r + 1))
        k[r, r] = w[0]
        for d in range(1, r + 1):
            k[r - d, r] = k[r + d, r] = k[r, r - d] = k[r, r + d] = w[d]
    else:
        k = w.reshape(2 * r + 1, 2 * r + 1)
    s = ndimage.correlate(np.abs(x.astype(np.float64)), k, mode="constant")
    return (n + 2) * 2.0 ** -24 * s + 1e-30


def check_stencil(out, x, radius, weights, shape):
    ref = oracle.stencil2d(x, radius, weights, shape)
    tol = stencil_tolerance(x, radius, weights, shape)
    err = np.abs(out.astype(np.float64) - ref)
    r = radius
    edge = np.ones(x.shape, dtype=bool)
    edge[r:x.shape[0] - r, r:x.shape[1] - r] = False
    assert np.array_equal(out[edge], x[edge]), "edge points must keep their input"
    bad = err > tol
    assert not bad.any(), (int(bad.sum()), float((err / tol).max()))


STENCIL_GRIDS_SMALL = [(1, 1), (3, 3), (9, 9), (64, 128), (65, 129), (130, 300), (200, 131), (7, 500)]


def test_emu_stencil_fd_orders_and_box():
    """FD stencils of orders I-IV and random box stencils on grids spanning several
    64 x 128 tiles, ragged edges and grids smaller than the stencil."""
    jobs = []
    g = rr_synth.rng(17)
    for t, (rows, cols) in enumerate(STENCIL_GRIDS_SMALL):
        x = rr_synth.random_grid(300 + t, rows, cols)
        for r, c in rr_synth.FD_LAPLACIAN.items():
            jobs.append(dict(op="stencil", grid=x, radius=r, weights=c, shape=0))
        r = int(g.integers(1, 5))
        jobs.append(dict(op="stencil", grid=x, radius=r, shape=1,
                         weights=g.uniform(-1, 1, (2 * r + 1) ** 2).astype(np.float32)))
    for j, (st, out) in zip(jobs, emu_runner.run(jobs)):
        assert st.startswith("ok"), st
        check_stencil(out, j["grid"], j["radius"], j["weights"], j["shape"])


UA_RUN_CASES = [
    # permutes that keep the fastest axis, with output runs of R >= 64 bytes that
    # aligned 16-byte vectors do not fit.  (dims, perm, element bytes, src offset, dst offset)
    ((7, 9, 33), (1, 0, 2), 2, 3, 1),          # R = 66, both sides misaligned
    ((4, 3, 4097), (1, 0, 2), 1, 1, 0),        # long odd runs
    ((5, 6, 100), (1, 0, 2), 1, 0, 0),         # R = 100
    ((3, 4, 5, 24), (2, 0, 1, 3), 4, 4, 0),    # R = 96 at 4-byte alignment, rank 4
    ((6, 5, 9), (1, 0, 2), 8, 8, 8),           # R = 72 at 8-byte alignment
    ((2, 3, 5, 127), (3, 1, 0, 2), 1, 0, 0),   # not a run: stays exact on the tile path
]


def test_emu_unaligned_run_vectors():
    """Runs moved as 16-byte vectors at any alignment, the last one overlapping
    its neighbour, against the oracle."""
    jobs = [_perm_job(d, p, e, 8900 + i, src_off=so, dst_off=do) for i, (d, p, e, so, do) in enumerate(UA_RUN_CASES)]
    res = _check(jobs)
    for st, _ in res[:-1]:
        assert "class=run" in st and "vec=16" in st and "ua=1" in st, st
    # runs shorter than a line that share lines load through the caches, each XCD
    # taking a contiguous range of blocks (R = 66, 100, 96, 72 here)
    assert sum("cached=1" in st for st, _ in res) >= 3, res


@pytest.mark.parametrize("chunk", [0, 2])
def test_emu_cached_runs_in_batches(chunk):
    """Short runs that share input lines, batched (each XCD a contiguous range of a
    job's blocks), whole and cut into workgroup ranges, next to other jobs."""
    jobs = [_perm_job(d, p, e, 9750 + i, src_off=so, dst_off=do) for i, (d, p, e, so, do) in enumerate(UA_RUN_CASES)]
    jobs += [_perm_job((60, 70, 33), (1, 0, 2), 2, 9760), _perm_job((90, 11, 9), (1, 0, 2), 8, 9761),
             _perm_job((33, 45, 77), (2, 0, 1), 8, 9762)]
    st, outs = emu_runner.run([dict(op="batched", jobs=jobs, chunk=chunk)])[0]
    assert st.startswith("ok"), st
    for j, o in zip(jobs, outs):
        assert np.array_equal(o, oracle.permute(j["input"], j["dims"], j["perm"], j["esize"])), (j["dims"], chunk)
