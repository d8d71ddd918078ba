"""Host-side checks of librr: the C ABI loads and exports what include/rr.h declares,
and validation / canonicalisation / planning behave as documented.  No GPU is
touched: every call here returns before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import rr_synth
import paper_1011_3583_amd as rr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "rr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rr_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = rr.lib()
    names = _header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), f"librr.so does not export {n}"
    assert set(names) == set(rr.EXPORTS)
    assert b"gfx950" in L.rr_version()


def test_status_strings():
    for code, name in rr.STATUS.items():
        assert rr.lib().rr_status_string(code).decode() == name


def test_order_to_perm_matches_paper_reading():
    table = {(0, 2, 1): (1, 0, 2), (1, 0, 2): (0, 2, 1), (1, 2, 0): (2, 0, 1), (2, 0, 1): (1, 2, 0),
             (2, 1, 0): (2, 1, 0), (1, 0, 2, 3): (0, 1, 3, 2), (3, 2, 0, 1): (2, 3, 1, 0),
             (3, 0, 2, 1, 4): (0, 3, 2, 4, 1)}
    for order, perm in table.items():
        assert rr.order_to_perm(order) == perm
    # and the converted perm reproduces the oracle's paper-notation reorder
    for sizes, order in [((4, 3, 2), (1, 2, 0)), ((3, 2, 5, 2), (3, 0, 2, 1))]:
        x = rr_synth.random_bytes(5, int(np.prod(sizes)) * 4)
        a = oracle.reorder_paper(x, sizes, order, 4)
        b = oracle.permute(x, tuple(reversed(sizes)), rr.order_to_perm(order), 4)
        assert np.array_equal(a, b)
    with pytest.raises(rr.RRError):
        rr.order_to_perm((0, 0, 1))


def _status(dims, perm, e, dst=0x100000, src=0x900000):
    return rr.permute_raw(dst, src, dims, perm, e, stream=0)


def test_validation_errors_return_before_launch():
    assert _status((4, 4), (0, 0), 4) == 1          # not a permutation
    assert _status((4, 4), (1, 0), 0) == 1          # elem_size
    assert _status((4, 4), (1, 0), 17) == 1
    assert _status((4, -1), (1, 0), 4) == 1         # negative extent
    assert _status(tuple([2] * 9), tuple(range(9)), 1) == 4  # rank > 8
    assert _status((1 << 40, 1 << 30), (1, 0), 4) == 2       # overflow
    assert _status((4, 4), (1, 0), 4, dst=0x1000, src=0x1008) == 3  # alias
    assert _status((4, 4), (1, 0), 4, dst=0, src=0x1000) == 1       # NULL
    assert "permutation" in rr.last_error() or "NULL" in rr.last_error()
    # zero elements: nothing to do, no launch, OK even with NULL pointers
    assert _status((0, 5), (1, 0), 4, dst=0, src=0) == 0
    # interlace validation
    assert rr.interlace_raw(0x1000, [0x100000, 0x200000], 16, 0) == 1
    assert rr.interlace_raw(0x1000, [0x100000] * 17, 16, 4) == 1
    assert rr.interlace_raw(0x100000, [0x100000, 0x200000], 16, 4) == 3
    assert rr.deinterlace_raw([0x200000, 0x200010], 0x100000, 16, 4) == 3  # planes overlap
    assert rr.interlace_raw(0x1000, [0x100000, 0x200000], 0, 4) == 0


CANON = [
    # (dims, perm, esize) -> (class, canonical dims, canonical perm, element bytes)
    ((512, 512, 256), (0, 1, 2), 4, "copy", "", "", 2**26 * 4),
    ((512, 512, 256), (0, 2, 1), 4, "tile", "512,512,256", "0,2,1", 4),
    ((512, 512, 256), (1, 0, 2), 4, "run", "512,512", "1,0", 1024),
    ((512, 512, 256), (1, 2, 0), 4, "tile", "512,131072", "1,0", 4),
    ((512, 512, 256), (2, 0, 1), 4, "tile", "262144,256", "1,0", 4),
    ((512, 512, 256), (2, 1, 0), 4, "tile", "512,512,256", "2,1,0", 4),
    ((64, 128, 128, 64), (0, 3, 1, 2), 2, "tile", "64,16384,64", "0,2,1", 2),
    ((64, 128, 128, 64), (0, 2, 3, 1), 2, "tile", "64,128,8192", "0,2,1", 2),
    ((32, 32, 32, 32, 32), (4, 2, 0, 3, 1), 1, "tile", "32,32,32,32,32", "4,2,0,3,1", 1),
    ((16384, 16384), (1, 0), 16, "tile", "16384,16384", "1,0", 16),
    ((256, 16, 1, 256, 16), (0, 3, 2, 4, 1), 4, "tile", "256,16,4096", "0,2,1", 4),
    ((1, 256, 256, 256), (0, 1, 3, 2), 4, "tile", "256,256,256", "0,2,1", 4),  # Table 2 row 2 squeezed
]


@pytest.mark.parametrize("dims,perm,e,cls,cdims,cperm,eb", CANON)
def test_canonical_forms(dims, perm, e, cls, cdims, cperm, eb):
    d = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    assert d["class"] == cls
    if cls != "copy":
        assert d["dims"] == cdims and d["perm"] == cperm
    assert int(d["esize_bytes"]) == eb


def test_canonical_form_is_equivalent_to_the_original():
    """The rewritten problem (squeezed, fused, element-folded) moves the same bytes."""
    g = rr_synth.rng(31)
    for t in range(150):
        nd = int(g.integers(1, 7))
        dims = tuple(int(g.choice([1, 1, 2, 3, 4, 5])) for _ in range(nd))
        perm = tuple(int(v) for v in g.permutation(nd))
        e = int(g.integers(1, 17))
        d = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
        x = rr_synth.random_bytes(t, int(np.prod(dims)) * e)
        ref = oracle.permute(x, dims, perm, e)
        eb = int(d["esize_bytes"])
        if d["class"] in ("copy",) or d["dims"] == "":
            assert np.array_equal(ref, x)
            continue
        cd = tuple(int(v) for v in d["dims"].split(","))
        cp = tuple(int(v) for v in d["perm"].split(","))
        assert np.array_equal(oracle.permute(x, cd, cp, eb), ref), (dims, perm, e, d)


def test_plan_uses_widest_vectors_on_aligned_buffers():
    # 1-byte elements: 16-byte row reads, 8x8 micro-tiles (8-byte stores) by default
    d = rr.plan_describe((16384, 16384), (1, 0), 1, dst=1 << 20, src=1 << 30)
    assert (d["unit"], d["g"], d["win"]) == ("1", "8", "16")
    rr.set_tile_override(max_g=16)
    d = rr.plan_describe((16384, 16384), (1, 0), 1, dst=1 << 20, src=1 << 30)
    rr.set_tile_override()
    assert (d["unit"], d["g"], d["win"]) == ("1", "16", "16")
    d = rr.plan_describe((1024, 1024), (1, 0), 4, dst=1 << 20, src=1 << 30)
    assert (d["unit"], d["g"], d["win"]) == ("4", "4", "16")
    # misaligned base pointer -> narrower access, still a valid plan
    d = rr.plan_describe((1024, 1024), (1, 0), 4, dst=(1 << 20) + 2, src=1 << 30)
    assert d["unit"] == "2"


def test_interlace_plan_classes():
    """2-8 sets of 1-8-byte elements on 16-byte boundaries, a whole number of 16-byte
    vectors each, are joined and split in registers -- except an interlace whose tile
    writes whole 16-byte vectors of merged short rows, an eight-set de-interlace and
    an interlace of eight sets of 4-8-byte elements, which keep the tile.  The joined side is streamed, but for the stores of an
    interlace of an odd number of sets, unless the cache override says otherwise.  Any
    other case keeps the LDS tile, as does the override that switches the register
    path off."""
    base = 1 << 40   # describe only reads pointer values

    def cls(n, count, e, off=0, de=False, key="class"):
        pb = count * e
        planes = [base + n * pb + (c + 1) * (pb + 4096) + off for c in range(n)]
        return rr.interlace_describe(base + off, planes, count, e, de)[key]

    merged = 0
    for n in range(2, 9):
        for e in (1, 2, 4, 8):
            count = 1000 * 16 // e
            rr.set_tile_override(weave=False)
            try:
                tile_merges = bool(int(cls(n, count, e, key="flags")) & 8)
            finally:
                rr.set_tile_override()
            merged += tile_merges
            assert cls(n, count, e) == ("tile" if tile_merges or (n == 8 and e >= 4) else "weave"), (n, e)
            assert cls(n, count, e, de=True) == ("weave" if n <= 7 else "tile"), (n, e)
            if not tile_merges and not (n == 8 and e >= 4):
                assert cls(n, count, e, key="cached") == str(n % 2)
                # two 64-group chunks per wave up to three sets, one from four on
                assert cls(n, count, e, key="chunks") == ("2" if n <= 3 else "1")
            if n <= 7:
                assert cls(n, count, e, de=True, key="cached") == "0"
                assert cls(n, count, e, de=True, key="chunks") == ("2" if n <= 4 else "1")
            assert cls(n, count, e, off=4) == "tile"             # misaligned
            assert cls(n, count + 1, e) == "tile"                # partial vector
    assert 0 < merged < 28   # complex64 pairs and RGBA bytes keep the tile's merged stores
    assert cls(8, 4096, 1) == "weave" and cls(8, 4096, 4) == "tile"
    assert cls(2, 1 << 20, 4) == cls(4, 1 << 20, 1) == "tile"
    assert cls(9, 4096, 4) == cls(2, 4096, 3) == cls(2, 4096, 16) == "tile"
    assert cls(1, 4096, 4) == "copy"
    assert cls(3, 0, 4) == "empty"
    rr.set_tile_override(cache=3)
    try:
        assert cls(4, 4096, 4, key="cached") == cls(3, 4096, 4, de=True, key="cached") == "1"
        rr.set_tile_override(cache=0)
        assert cls(3, 4096, 4, key="cached") == "0"
        rr.set_tile_override(cache=2)   # writes cached: the interlace's joined side only
        assert cls(3, 4096, 4, key="cached") == "1" and cls(3, 4096, 4, de=True, key="cached") == "0"
        rr.set_tile_override(weave=False)
        assert cls(3, 4096, 4) == cls(3, 4096, 4, de=True) == "tile"
    finally:
        rr.set_tile_override()
    with pytest.raises(rr.RRError):   # a plane overlapping the joined buffer
        rr.interlace_describe(base, [base + 8, base + (1 << 30)], 1024, 4)


def test_tuning_cache_changes_the_plan_and_round_trips(tmp_path):
    """A cached tile shape for a canonical problem is used by later plans of it."""
    K = rr.tune_context() + "|"
    L = rr.lib()
    rr.tune_clear()
    dims, perm, e = (16384, 16384), (1, 0), 4
    base = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    path = tmp_path / "tune.txt"
    key_line = K + "r2:e4:a16/16:d16384,16384:p1,0 1024 256 1 0 64\n"
    path.write_text(key_line)
    rr.tune_load(str(path))
    tuned = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    assert (tuned["TA"], tuned["TB"]) != (base["TA"], base["TB"])
    assert tuned["TA"] == "256"                      # 1024-byte input rows of 4-byte elements
    out = tmp_path / "saved.txt"
    rr.tune_save(str(out))
    assert key_line.strip() in out.read_text()
    # an explicit override wins over the cache
    rr.set_tile_override(128, 128, None)
    assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)["TA"] == "32"
    rr.set_tile_override(0, 0, None)
    rr.tune_clear()
    assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30) == base
    bad = tmp_path / "bad.txt"
    bad.write_text("key 99999 1 0\n")
    with pytest.raises(rr.RRError):
        rr.tune_load(str(bad))


def test_cache_policy_by_line_alignment():
    """Tiles whose rows all start on 128-byte lines stream both sides
    (non-temporal); when rows share lines with neighbouring tiles, stores go
    through the caches with XCD tile ranges, whatever the element size;
    interlace stays streamed; an explicit policy or XCD choice replaces the
    planner's."""
    LD, ST, XCD = 1024, 2048, 256

    def flags(dims, perm, e):
        return int(rr.plan_describe(dims, perm, e, dst=1 << 30, src=1 << 31)["flags"])

    rr.set_tile_override()
    for dims, perm, e in [((512, 512, 256), (0, 2, 1), 4), ((64, 16384, 64), (0, 2, 1), 16),
                          ((512, 131072), (1, 0), 8), ((16384, 16384), (1, 0), 1),
                          ((512, 512, 256), (2, 1, 0), 2)]:
        assert flags(dims, perm, e) & (LD | ST | XCD) == 0, (dims, perm, e)
    for dims, perm, e in [((1001, 999), (1, 0), 4), ((1398, 1000, 24), (2, 1, 0), 8),
                          ((32761, 4097), (1, 0), 2), ((8651, 1001, 31), (2, 0, 1), 1),
                          ((4095, 4097), (1, 0), 16)]:
        assert flags(dims, perm, e) & (LD | ST | XCD) == ST | XCD, (dims, perm, e)
    # stacked small transposes: a tile's sub-tiles are one contiguous block on both sides
    assert flags((1 << 20, 4, 8), (0, 2, 1), 4) & (128 | LD | ST | XCD) == 128
    assert flags((1000, 3, 3), (0, 2, 1), 2) & (128 | LD | ST | XCD) == 128 | ST | XCD
    # a misaligned base alone splits lines too
    assert int(rr.plan_describe((4096, 4096), (1, 0), 4, dst=(1 << 30) + 64, src=1 << 31)["flags"]) & ST
    try:
        for pol, want in [(0, 0), (1, LD), (2, ST), (3, LD | ST)]:
            rr.set_tile_override(cache=pol)
            assert flags((1001, 999), (1, 0), 4) & (LD | ST) == want
            assert flags((512, 512, 256), (0, 2, 1), 4) & (LD | ST) == want
        rr.set_tile_override(cache=1, xcd=False)
        assert flags((1001, 999), (1, 0), 4) & (LD | XCD) == LD
        rr.set_tile_override(xcd=True)
        assert flags((512, 512, 256), (0, 2, 1), 4) & (LD | ST | XCD) == XCD
        rr.set_tile_override(cache=1)      # cached on aligned rows: no automatic XCD ranges
        assert flags((512, 512, 256), (0, 2, 1), 4) & (LD | ST | XCD) == LD
        rr.set_tile_override(cache=1)      # rows that share lines: XCD ranges with the cached side
        assert flags((1001, 999), (1, 0), 4) & (LD | ST | XCD) == LD | XCD
        for bad in (8 | 64, 5 << 24):
            with pytest.raises(rr.RRError):
                rr.check(rr.lib().rr_set_tile_override(0, 0, bad))
    finally:
        rr.set_tile_override()


def test_fill_refit_plans():
    """Odd extents: the refit takes a short axis whole and evens out the other for
    fewer tiles within the tile size; evenly divided (dense) shapes keep their plans;
    both fill flags together are rejected."""
    rr.tune_clear()

    def desc(dims, perm, e, fill):
        rr.set_tile_override(fill=fill)
        try:
            return rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
        finally:
            rr.set_tile_override()

    off, on = desc((611, 39), (1, 0), 8, False), desc((611, 39), (1, 0), 8, True)
    assert (off["TA"], off["TB"], off["ntiles"]) == ("32", "64", "20")
    ta, tb = int(on["TA"]), int(on["TB"])
    assert int(on["ntiles"]) <= 13 and int(on["ntiles"]) == -(-39 // ta) * -(-611 // tb)
    assert ta * 8 >= 128 and tb * 8 >= 256                 # rows at least half their targets
    assert (ta * 8) % 16 == 0 or ta == 39                  # 16-byte rows unless whole
    assert (tb * 8) % 16 == 0 and tb * ((ta * 8 + 15) // 16 * 16) <= 16384   # tile within 16 KiB
    # 1-byte units: refit rows stay multiples of 16 bytes (no per-byte tails)
    on1, off1 = desc((4325, 1001, 31), (2, 0, 1), 2, True), desc((4325, 1001, 31), (2, 0, 1), 2, False)
    assert int(on1["ntiles"]) * 8 <= int(off1["ntiles"]) * 7 and (int(on1["TB"]) * 2) % 16 == 0
    assert rr.plan_describe((611, 39), (1, 0), 8, dst=1 << 20, src=1 << 30)["ntiles"] == on["ntiles"]
    for dims, perm, e in [((4096, 4096), (1, 0), 4), ((512, 512, 256), (2, 0, 1), 2),
                          ((32, 32, 32, 32, 32), (4, 2, 0, 3, 1), 16), ((1000, 1000), (1, 0), 4)]:
        assert desc(dims, perm, e, True) == desc(dims, perm, e, False), dims
    # a saving under an eighth keeps the row-target shape
    assert desc((32761, 4097), (1, 0), 2, True) == desc((32761, 4097), (1, 0), 2, False)
    with pytest.raises(rr.RRError):
        rr.check(rr.lib().rr_set_tile_override(0, 0, (1 << 27) | (1 << 28)))
    rr.set_tile_override()


def test_batched_planning_reports_lowest_invalid_job():
    """Batches of 1024 jobs or more plan on several host threads; validation still
    names the lowest invalid job, and nothing is launched (no GPU is touched)."""
    specs = []
    for i in range(2048):
        src = (1 << 32) + i * 4096
        specs.append([src + (1 << 36), src, (16, 32), (1, 0), 4])
    specs[1900][3] = (0, 0)          # not a permutation
    specs[700][2] = (16, -3)         # negative extent
    specs[1201][4] = 17              # element size out of range
    with pytest.raises(rr.RRError) as ei:
        rr.check(rr.permute_batched_raw([tuple(s) for s in specs]))
    assert "job 700" in str(ei.value), str(ei.value)
    specs[700][2] = (16, 32)
    with pytest.raises(rr.RRError) as ei:
        rr.check(rr.permute_batched_raw([tuple(s) for s in specs]))
    assert "job 1201" in str(ei.value), str(ei.value)


def test_micro_tile_cap_from_override_and_cache(tmp_path):
    """The micro-tile edge G can be capped by the override and by a cached entry."""
    K = rr.tune_context() + "|"
    rr.tune_clear()
    dims, perm, e = (4096, 4096), (1, 0), 1
    assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)["g"] == "8"
    for g in (16, 8, 4, 2, 1):
        rr.set_tile_override(max_g=g)
        assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)["g"] == str(g)
    rr.set_tile_override()
    with pytest.raises(rr.RRError):
        rr.set_tile_override(max_g=3)
    rr.set_tile_override()
    path = tmp_path / "tune.txt"
    path.write_text(K + "r2:e1:a16/16:d4096,4096:p1,0 128 128 1 8\n\n")
    rr.tune_load(str(path))
    d = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    assert (d["g"], d["TA"], d["TB"]) == ("8", "128", "128")
    out = tmp_path / "saved.txt"
    rr.tune_save(str(out))
    assert K + "r2:e1:a16/16:d4096,4096:p1,0 128 128 1 8" in out.read_text()
    rr.tune_clear()
    path.write_text(K + "r2:e1:a16/16:d4096,4096:p1,0 0 0 -1 0 0 1\n")
    rr.tune_load(str(path))
    assert int(rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)["flags"]) & 256
    rr.tune_clear()
    path.write_text(K + "r2:e4:a16/16:d1001,999:p1,0 0 0 -1 0 0 0 1\n")
    rr.tune_load(str(path))
    assert int(rr.plan_describe((1001, 999), (1, 0), 4, dst=1 << 20, src=1 << 30)["flags"]) & 512
    rr.tune_clear()
    assert not int(rr.plan_describe((1001, 999), (1, 0), 4, dst=1 << 20, src=1 << 30)["flags"]) & 512
    # the cache-policy field: 2 = writes through the caches, and no XCD ranges (xcd 0)
    path.write_text(K + "r2:e4:a16/16:d1001,999:p1,0 0 0 -1 0 0 0 0 2\n")
    rr.tune_load(str(path))
    f = int(rr.plan_describe((1001, 999), (1, 0), 4, dst=1 << 20, src=1 << 30)["flags"])
    assert f & 2048 and not f & 1024 and not f & 256
    assert K + "r2:e4:a16/16:d1001,999:p1,0 0 0 -1 0 0 0 0 2 0 -1" in (rr.tune_save(str(out)) or out.read_text())
    path.write_text(K + "r2:e4:a16/16:d1001,999:p1,0 0 0 -1 0 0 0 0 2 1\n")   # diagonal tile order
    rr.tune_clear()
    rr.tune_load(str(path))
    assert int(rr.plan_describe((1001, 999), (1, 0), 4, dst=1 << 20, src=1 << 30)["flags"]) & 4096
    rr.tune_clear()
    # the fill field: 0 keeps the row-target tiles of an odd extent
    refit = rr.plan_describe((611, 39), (1, 0), 8, dst=1 << 20, src=1 << 30)
    path.write_text(K + "r2:e8:a16/16:d611,39:p1,0 0 0 -1 0 0 -1 0 -1 0 0\n")
    rr.tune_load(str(path))
    d = rr.plan_describe((611, 39), (1, 0), 8, dst=1 << 20, src=1 << 30)
    assert (d["TA"], d["TB"], d["ntiles"]) == ("32", "64", "20") and d["ntiles"] != refit["ntiles"]
    rr.tune_clear()
    for bad in ("k 0 0 0 3\n", "k 0 0 0 8 65\n", "k 0 0 0 8 2\n", "k 0 0 0 8 16 2\n", "k 0 0 0 8 16 1 3\n",
                "k 0 0 0 8 16 -2\n", "k 0 0 0 8 16 1 1 4\n", "k 0 0 0 8 16 1 1 -2\n",
                "k 0 0 0 8 16 1 1 1 2\n", "k 0 0 0 8 16 1 1 1 0 2\n", "k 0 0 0 8 16 1 1 1 0 -2\n",
                "k 0 0 0 8 16 1 1 1 0 0 0\n", "k 0 0\n"):
        (tmp_path / "bad.txt").write_text(bad)
        with pytest.raises(rr.RRError):
            rr.tune_load(str(tmp_path / "bad.txt"))
    rr.tune_clear()


def test_no_kernel_uses_scratch():
    """Every kernel keeps its state in registers and LDS: a private-memory
    copy of the argument struct or a register spill costs each wave dozens of
    extra memory instructions per tile."""
    import json
    from paper_1011_3583_amd import build as rrbuild
    path = os.path.join(rrbuild.OBJ, rrbuild.RESOURCES)
    if not os.path.exists(path):
        pytest.skip("library not built in-tree")
    res = json.load(open(path))
    kernels = {k: v for k, v in res.items() if "k_" in k}
    assert any("k_tile" in k for k in kernels)
    used = {k: v["ScratchSize [bytes/lane]"] for k, v in kernels.items() if v["ScratchSize [bytes/lane]"]}
    assert not used, used


def test_reorder_validation_and_aliasing():
    """rr_reorder (N-to-M with base and range) rejects bad boxes before any launch."""
    dims = (4, 5, 6)
    ok = dict(dst=0x100000, src=0x1000)
    st = lambda b, r, o, e=4, **kw: rr.reorder_raw(kw.get("dst", ok["dst"]), kw.get("src", ok["src"]), dims, b, r, o, e)
    assert st((0, 0, 0), (4, 5, 6), (2, 0, 0)) == 1       # repeated axis
    assert st((0, 0, 0), (4, 5, 6), (3, 0)) == 1          # axis out of range
    assert st((0, 0, 0), (4, 5, 7), (2, 1, 0)) == 1       # range past the extent
    assert st((0, 0, 5), (4, 5, 2), (2, 1, 0)) == 1       # base + range past the extent
    assert st((0, 5, 0), (4, 1, 6), (2, 0)) == 1          # fixed axis base outside
    assert st((-1, 0, 0), (4, 5, 6), (2, 1, 0)) == 1      # negative base
    assert st((0, 0, 0), (4, 5, 6), (2, 1, 0), 0) == 1    # elem_size
    assert rr.reorder_raw(0x1000, 0x1000, (2,) * 9, None, None, tuple(range(9)), 1) == 4   # rank > 8
    assert st((0, 0, 0), (4, 5, 6), (2, 1, 0), dst=0, src=0x1000) == 1   # NULL
    # aliasing: the box (rows 2..3: bytes 240..479 from src) against dst's 240 bytes
    assert st((2, 0, 0), (2, 5, 6), (1, 2, 0), dst=0x1000, src=0x1000 - 100) == 3
    assert st((2, 0, 0), (2, 5, 6), (1, 2, 0), dst=0x1000 + 300, src=0x1000) == 3
    assert st((2, 0, 0), (2, 5, 6), (1, 2, 0), dst=0x1000 + 479, src=0x1000) == 3
    # empty boxes are a no-op even with NULL pointers
    assert rr.reorder_raw(0, 0, dims, (0, 0, 0), (0, 5, 6), (0, 1, 2), 4) == 0


def test_reorder_plans_match_permute_and_classes():
    """A full box with every axis kept plans exactly like rr_permute; boxes that
    keep the input's fastest axis contiguous tile; keeping it strided by 2-4 elements
    selects; dropping it or a wider stride gathers."""
    for dims, perm, e in [((512, 512, 256), (2, 0, 1), 4), ((64, 128, 128, 64), (0, 3, 1, 2), 2), ((4096, 4096), (1, 0), 1)]:
        a = rr.reorder_describe(dims, None, None, perm, e, dst=1 << 20, src=1 << 30)
        b = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
        assert a == b
    # a 2-D crop of a 3-D array, transposed: strided box, tile class
    d = rr.reorder_describe((70, 90, 40), (3, 5, 7), (60, 80, 30), (2, 1, 0), 4, dst=1 << 20, src=1 << 30)
    assert d["class"] == "tile" and d["dims"] == "60,80,30"
    # channel 2 of an HWC image: the kept fastest axis is strided (4 bytes apart) -> select
    d = rr.reorder_describe((256, 256, 4), (0, 0, 2), None, (0, 1), 1, dst=1 << 20, src=1 << 30)
    assert d["class"] == "select" and d["dims"] == "65536" and d["stride"] == "4" and d["m"] == "4"
    # one channel of 5-channel records (stride of 5 elements): gathered element by element
    d = rr.reorder_describe((256, 256, 5), (0, 0, 2), None, (0, 1), 1, dst=1 << 20, src=1 << 30)
    assert d["class"] == "run"
    # a column of a matrix (the fastest axis dropped) -> gather
    d = rr.reorder_describe((100, 64), (0, 7), (100, 1), (0,), 4, dst=1 << 20, src=1 << 30)
    assert d["class"] == "run"
    # rows 10..19 of a matrix: one contiguous range -> copy
    d = rr.reorder_describe((100, 64), (10, 0), (10, 64), (0, 1), 4, dst=1 << 20, src=1 << 30)
    assert d["class"] == "copy" and d["bytes"] == str(10 * 64 * 4)


def test_gather_and_range_validation():
    assert rr.gather_raw(0x100000, 0x1000, 10, 0x200000, 5, 0) == 1          # elem_size
    assert rr.gather_raw(0x100000, 0x1000, 10, 0x200000, -1, 4) == 1         # count
    assert rr.gather_raw(0x100000, 0x1000, 10, 0, 5, 4) == 1                 # NULL idx
    assert rr.gather_raw(0x1000, 0x1000, 10, 0x200000, 5, 4) == 3            # dst overlaps src
    assert rr.gather_raw(0x200010, 0x1000, 10, 0x200000, 5, 4) == 3          # dst overlaps idx
    assert rr.gather_raw(0, 0, 10, 0, 0, 4) == 0                             # empty: no-op
    assert rr.copy_range_raw(0x100000, 0x1000, 10, 0, 1, 11, 4) == 1         # past the end
    assert rr.copy_range_raw(0x100000, 0x1000, 10, 9, 2, 2, 4) == 1
    assert rr.copy_range_raw(0x100000, 0x1000, 10, 2, -1, 4, 4) == 1         # before the start
    assert rr.copy_range_raw(0x100000, 0x1000, 10, -1, 1, 1, 4) == 1
    assert rr.copy_range_raw(0x1000 + 8, 0x1000, 10, 0, 1, 5, 4) == 3        # dst inside the bytes read
    assert rr.copy_range_raw(0, 0, 10, 3, 1, 0, 4) == 0                      # empty: no-op
    assert rr.copy_range_raw(0x100000, 0x1000, 1 << 62, 0, 1 << 40, 1 << 30, 4) == 2   # overflow


def test_stencil_validation():
    w = [-4.0, 1.0]
    assert rr.stencil2d_raw(0x100000, 0x200000, 16, 16, 0, w) == 1          # radius
    assert rr.stencil2d_raw(0x100000, 0x200000, 16, 16, 5, w) == 1
    assert rr.stencil2d_raw(0x100000, 0x200000, 16, 16, 1, w, shape=2) == 1
    assert rr.stencil2d_raw(0x100000, 0x200000, -1, 16, 1, w) == 1          # rows
    assert rr.stencil2d_raw(0x100002, 0x200000, 16, 16, 1, w) == 1          # alignment
    assert rr.stencil2d_raw(0x100000, 0x100000 + 512, 16, 16, 1, w) == 3    # overlap
    assert rr.stencil2d_raw(0, 0, 0, 16, 1, w) == 0                         # empty grid
    assert rr.stencil2d_raw(0x100000, 0x200000, 1 << 40, 1 << 40, 1, w) == 2


def test_override_is_safe_across_threads():
    """Planning on several threads while another flips the process-wide override:
    every plan is one of the two consistent outcomes (the override is read as a
    locked snapshot)."""
    import threading
    dims, perm, e = (4096, 4096), (1, 0), 1
    rr.set_tile_override()
    base = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    rr.set_tile_override(max_g=4)
    capped = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    rr.set_tile_override()
    ok = {base["g"] + base["TA"] + base["TB"], capped["g"] + capped["TA"] + capped["TB"]}
    seen, errors = set(), []

    def plan():
        try:
            for _ in range(400):
                d = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
                seen.add(d["g"] + d["TA"] + d["TB"])
        except Exception as ex:   # pragma: no cover - reported below
            errors.append(ex)

    def flip():
        for k in range(400):
            rr.set_tile_override(max_g=4 if k % 2 else 0)

    ts = [threading.Thread(target=plan) for _ in range(4)] + [threading.Thread(target=flip)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    rr.set_tile_override()
    assert not errors and seen <= ok, (errors, seen, ok)


def test_tuning_file_of_another_device_or_runtime_is_skipped(tmp_path):
    """Tuned shapes were timed on one device and HIP runtime: lines keyed with
    another architecture or runtime version are skipped on load, lines of this
    process's context are used, and a malformed line stores nothing."""
    ctx = rr.tune_context()
    arch, ver = ctx.split("@hip")
    assert arch and ver.isdigit(), ctx
    rr.tune_clear()
    dims, perm, e = (16384, 16384), (1, 0), 4
    base = rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)
    body = "r2:e4:a16/16:d16384,16384:p1,0 1024 256 1 0 64\n"
    path = tmp_path / "tune.txt"
    for other in ("gfx942:sramecc+:xnack-@hip" + ver, arch + "@hip" + str(int(ver) + 1)):
        path.write_text(other + "|" + body)
        rr.tune_load(str(path))
        assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30) == base, other
    path.write_text("gfx942:sramecc+:xnack-@hip1|" + body + ctx + "|" + body)
    rr.tune_load(str(path))
    assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30)["TA"] == "256"
    out = tmp_path / "saved.txt"
    rr.tune_save(str(out))
    assert out.read_text() == ctx + "|" + body.replace("64\n", "64 0 0 -1 0 -1\n")
    rr.tune_clear()
    # a key without any context is malformed; nothing of the file is stored
    path.write_text(ctx + "|" + body + body)
    with pytest.raises(rr.RRError):
        rr.tune_load(str(path))
    assert rr.plan_describe(dims, perm, e, dst=1 << 20, src=1 << 30) == base


def test_diagonal_order_by_default():
    """2-D transposes of 1-8-byte elements whose rows are a power of two of at least
    4 KiB on both sides (16 MiB or more per side) take the diagonal tile order by
    default; other pitches, 16-byte elements, small problems and higher ranks keep
    the plain order; the override switches it either way."""
    def diag(dims, e, perm=(1, 0)):
        return bool(int(rr.plan_describe(dims, perm, e, dst=1 << 30, src=1 << 33)["flags"]) & 4096)

    for e in (1, 2, 4, 8):
        assert diag((8192, 8192), e) and diag((16384, 4096), e) and diag((4096, 16384), e), e
    assert diag((4096, 4096), 1)
    assert not diag((8192, 8192), 16)
    assert not diag((8320, 8192), 4) and not diag((16000, 16000), 4) and not diag((12288, 12288), 1)
    assert not diag((1024, 1024), 4)                       # 4 MiB: below the measured sizes
    assert not diag((512, 512, 256), 4, (2, 1, 0))         # rank 3
    rr.set_tile_override(diag=False)
    try:
        assert not diag((8192, 8192), 4)
        rr.set_tile_override(diag=True)
        assert diag((8320, 8192), 4)
        with pytest.raises(rr.RRError):
            rr.check(rr.lib().rr_set_tile_override(0, 0, 128 | (1 << 30)))
    finally:
        rr.set_tile_override()
