"""Pins for the CPU oracle: it is checked against things other than itself.

* hand-worked fixtures written from the definitions (tests/golden),
* the paper's statement that order [0 1 2] is a plain memcpy (Table 1, first row),
* NumPy's own transpose / stack / reshape (an independent library routine),
* brute force over every permutation of small ranks and odd extents,
* algebraic invariants: inverse, composition, interlace o de-interlace = id,
  the element-size split,
* the paper's fastest-first notation against the row-major one.

Each planted mistake (mutant build of the oracle) must fail at least one pin.
"""
import itertools

import numpy as np
import pytest

import oracle
import rr_synth
from tests import golden_io


def _iota(n):
    return (np.arange(n) % 256).astype(np.uint8)


def _np_permute(x_bytes, dims, perm, esize):
    """NumPy's transpose on a (dims..., esize) byte view; independent of the oracle."""
    a = x_bytes.reshape(tuple(dims) + (esize,))
    return np.ascontiguousarray(np.transpose(a, tuple(perm) + (len(dims),))).reshape(-1)


def paper_order_to_numpy_perm(order):
    """Fastest-first order o -> row-major perm: perm[j] = N-1-o[N-1-j] (reading of Sec. III.B)."""
    n = len(order)
    return tuple(n - 1 - order[n - 1 - j] for j in range(n))


# --------------------------------------------------------------------------- pins
def pin_golden(golden_dir, m=0):
    for case in golden_io.load_all(golden_dir):
        op = case["op"]
        e = case.get("esize", [4])[0]
        if op == "permute":
            n = int(np.prod(case["dims"])) * e
            got = oracle.permute(_iota(n), case["dims"], case["perm"], e, mutant=m)
            if got.tolist() != case["expect"]:
                return False
        elif op == "reorder_paper":
            n = int(np.prod(case["sizes"])) * e
            got = oracle.reorder_paper(_iota(n), case["sizes"], case["order"], e, mutant=m)
            if got.tolist() != case["expect"]:
                return False
            dims = list(reversed(case["sizes"]))
            got2 = oracle.permute(_iota(n), dims, case["numpy_perm"], e, mutant=m)
            if got2.tolist() != case["expect"]:
                return False
        elif op == "reorder_slice":
            n = int(np.prod(case["dims"])) * e
            got = oracle.reorder_slice(_iota(n), case["dims"], case["base"], case["range"],
                                       case.get("order", []), e, mutant=m)
            if got.tolist() != case["expect"]:
                return False
        elif op == "gather":
            n = case["src_count"][0] * e
            got = oracle.gather(_iota(n), case["idx"], e, mutant=m)
            if got.tolist() != case["expect"]:
                return False
        elif op == "copy_range":
            n = case["src_count"][0] * e
            got = oracle.copy_range(_iota(n), case["start"][0], case["stride"][0], case["count"][0], e, mutant=m)
            if got.tolist() != case["expect"]:
                return False
        elif op == "stencil":
            rows, cols = case["rows"][0], case["cols"][0]
            x = np.arange(rows * cols, dtype=np.float32).reshape(rows, cols)
            got = oracle.stencil2d(x, case["radius"][0], case["weights"], case["shape"][0], mutant=m)
            if got.reshape(-1).tolist() != [float(v) for v in case["expect"]]:
                return False
        elif op == "interlace":
            planes = [np.array(p, dtype=np.uint8) for p in case["planes"]]
            got = oracle.interlace(planes, e, mutant=m)
            if got.tolist() != case["expect"]:
                return False
        elif op == "deinterlace":
            n = int(case["input"][1])
            got = oracle.deinterlace(_iota(n), case["n"][0], e, mutant=m)
            if [g.tolist() for g in got] != case["expect_planes"]:
                return False
        else:
            raise AssertionError(f"unknown op {op}")
    return True


def pin_identity_is_memcpy(m=0):
    """Table 1, first row: order [0 1 2] is the memcpy reference."""
    for dims, e in [((5, 7, 3), 4), ((2, 3, 4, 5), 3), ((17,), 16)]:
        n = int(np.prod(dims)) * e
        x = rr_synth.random_bytes(11, n)
        if not np.array_equal(oracle.permute(x, dims, tuple(range(len(dims))), e, mutant=m), x):
            return False
    return True


def pin_numpy_random(m=0, trials=60):
    g = rr_synth.rng(1234)
    for t in range(trials):
        nd = int(g.integers(1, 6))
        dims = tuple(int(g.integers(1, 7)) for _ in range(nd))
        perm = tuple(int(v) for v in g.permutation(nd))
        e = int(g.integers(1, 17))
        x = rr_synth.random_bytes(100 + t, int(np.prod(dims)) * e)
        if not np.array_equal(oracle.permute(x, dims, perm, e, mutant=m),
                              _np_permute(x, dims, perm, e)):
            return False
    return True


def pin_brute_force(m=0, max_ndim=5):
    """Every permutation of rank <= max_ndim on odd extents, against NumPy."""
    ext = (3, 2, 5, 1, 2)
    for nd in range(1, max_ndim + 1):
        dims = ext[:nd]
        for e in (1, 3, 8):
            x = rr_synth.random_bytes(7 * nd + e, int(np.prod(dims)) * e)
            for perm in itertools.permutations(range(nd)):
                if not np.array_equal(oracle.permute(x, dims, perm, e, mutant=m),
                                      _np_permute(x, dims, perm, e)):
                    return False
    return True


def pin_inverse_and_composition(m=0):
    g = rr_synth.rng(77)
    for t in range(20):
        nd = int(g.integers(2, 6))
        dims = tuple(int(g.integers(1, 6)) for _ in range(nd))
        p = tuple(int(v) for v in g.permutation(nd))
        q = tuple(int(v) for v in g.permutation(nd))
        e = int(g.choice([1, 2, 4, 5]))
        x = rr_synth.random_bytes(500 + t, int(np.prod(dims)) * e)
        y = oracle.permute(x, dims, p, e, mutant=m)
        pdims = tuple(dims[k] for k in p)
        inv = tuple(int(v) for v in np.argsort(p))
        if not np.array_equal(oracle.permute(y, pdims, inv, e, mutant=m), x):
            return False
        # permute(permute(x, p), q) == permute(x, p[q])
        z = oracle.permute(y, pdims, q, e, mutant=m)
        pq = tuple(p[k] for k in q)
        if not np.array_equal(z, oracle.permute(x, dims, pq, e, mutant=m)):
            return False
    return True


def pin_esize_split(m=0):
    """An e-byte element permute equals a 1-byte permute with the bytes as an extra last axis."""
    for dims, perm, e in [((4, 3, 5), (2, 0, 1), 6), ((3, 7), (1, 0), 16), ((2, 3, 2, 3), (3, 1, 0, 2), 3)]:
        x = rr_synth.random_bytes(9, int(np.prod(dims)) * e)
        a = oracle.permute(x, dims, perm, e, mutant=m)
        b = oracle.permute(x, tuple(dims) + (e,), tuple(perm) + (len(dims),), 1, mutant=m)
        if not np.array_equal(a, b):
            return False
    return True


def pin_interlace_numpy(m=0):
    for n, count, e in [(2, 37, 4), (3, 50, 4), (4, 64, 1), (9, 13, 2), (1, 5, 8), (16, 3, 16)]:
        planes = [rr_synth.random_bytes(40 + c, count * e) for c in range(n)]
        got = oracle.interlace(planes, e, mutant=m)
        ref = np.stack([p.reshape(count, e) for p in planes], axis=1).reshape(-1)
        if not np.array_equal(got, ref):
            return False
        back = oracle.deinterlace(got, n, e, mutant=m)
        if not all(np.array_equal(b, p) for b, p in zip(back, planes)):
            return False
        x = rr_synth.random_bytes(90, n * count * e)
        split = oracle.deinterlace(x, n, e, mutant=m)
        ref_split = x.reshape(count, n, e).transpose(1, 0, 2)
        if not all(np.array_equal(split[c], ref_split[c].reshape(-1)) for c in range(n)):
            return False
    # Sec. III.C example: complex numbers split into real and imaginary planes.
    z = rr_synth.random_bytes(5, 8 * 100).view(np.complex64)
    re, im = oracle.deinterlace(z.view(np.uint8), 2, 4)
    if not (np.array_equal(re.view(np.float32).view(np.uint32), z.real.view(np.uint32))
            and np.array_equal(im.view(np.float32).view(np.uint32), z.imag.view(np.uint32))):
        return False
    return True


def pin_paper_notation(m=0):
    """Every fastest-first order of ranks 2..4 equals the converted row-major permute."""
    for sizes in [(3, 2), (4, 3, 2), (2, 3, 1, 5)]:
        n = len(sizes)
        x = rr_synth.random_bytes(3, int(np.prod(sizes)) * 2)
        for order in itertools.permutations(range(n)):
            a = oracle.reorder_paper(x, sizes, order, 2, mutant=m)
            b = oracle.permute(x, tuple(reversed(sizes)), paper_order_to_numpy_perm(order), 2, mutant=m)
            c = _np_permute(x, tuple(reversed(sizes)), paper_order_to_numpy_perm(order), 2)
            if not (np.array_equal(a, b) and np.array_equal(a, c)):
                return False
    return True


def _np_reorder_slice(x_bytes, dims, base, range_, order, esize):
    """NumPy slicing + transpose on a (dims..., esize) byte view; independent of the oracle."""
    a = x_bytes.reshape(tuple(dims) + (esize,))
    idx = tuple(slice(base[d], base[d] + range_[d]) if d in order else base[d] for d in range(len(dims)))
    sub = a[idx]                                # kept axes, in input order, then the byte axis
    kept = sorted(order)
    axes = tuple(kept.index(o) for o in order) + (len(order),)
    return np.ascontiguousarray(np.transpose(sub, axes)).reshape(-1)


def _random_slices(seed, count, max_rank=5):
    g = rr_synth.rng(seed)
    out = []
    for _ in range(count):
        nd = int(g.integers(1, max_rank + 1))
        dims = [int(g.integers(1, 7)) for _ in range(nd)]
        m = int(g.integers(0, nd + 1))
        order = [int(v) for v in g.permutation(nd)[:m]]
        base, range_ = [], []
        for d in range(nd):
            b = int(g.integers(0, dims[d]))
            base.append(b)
            range_.append(int(g.integers(0, dims[d] - b + 1)) if d in order else 1)
        out.append((dims, base, range_, order, int(g.choice([1, 2, 3, 4, 8]))))
    return out


def pin_reorder_slice_numpy(m=0):
    """N-to-M reorder == NumPy slicing (fixed axes indexed, kept axes sliced) + transpose."""
    for i, (dims, base, range_, order, e) in enumerate(_random_slices(31, 300)):
        x = rr_synth.random_bytes(600 + i, int(np.prod(dims)) * e)
        got = oracle.reorder_slice(x, dims, base, range_, order, e, mutant=m)
        if not np.array_equal(got, _np_reorder_slice(x, dims, base, range_, order, e)):
            return False
    return True


def pin_reorder_slice_reduces_to_permute(m=0):
    """With every axis kept at full range the N-to-M reorder is the permute; a box is
    the permute of the box cut out first (NumPy copy)."""
    for dims, perm, e in [((5, 7, 3), (2, 0, 1), 4), ((2, 3, 4, 5), (3, 1, 0, 2), 2)]:
        x = rr_synth.random_bytes(41, int(np.prod(dims)) * e)
        full = oracle.reorder_slice(x, dims, [0] * len(dims), dims, perm, e, mutant=m)
        if not np.array_equal(full, oracle.permute(x, dims, perm, e, mutant=m)):
            return False
        base = [1] * len(dims)
        rng = [d - 1 for d in dims]
        box = np.ascontiguousarray(x.reshape(tuple(dims) + (e,))[tuple(slice(1, d) for d in dims)]).reshape(-1)
        got = oracle.reorder_slice(x, dims, base, rng, perm, e, mutant=m)
        if not np.array_equal(got, oracle.permute(box, rng, perm, e, mutant=m)):
            return False
    return True


def pin_gather_and_range_numpy(m=0):
    """Index-set and range reads == NumPy take / strided slicing on an (n, esize) byte view."""
    g = rr_synth.rng(53)
    for t in range(60):
        e = int(g.choice([1, 2, 3, 4, 8, 16]))
        n = int(g.integers(1, 500))
        x = rr_synth.random_bytes(700 + t, n * e)
        v = x.reshape(n, e)
        idx = g.integers(0, n, int(g.integers(0, 800)))
        if not np.array_equal(oracle.gather(x, idx, e, mutant=m), v[idx].reshape(-1)):
            return False
        start = int(g.integers(0, n))
        stride = int(g.integers(-5, 6))
        if stride > 0:
            count = int(g.integers(0, (n - 1 - start) // stride + 2))
        elif stride < 0:
            count = int(g.integers(0, start // -stride + 2))
        else:
            count = int(g.integers(0, 20))
        ref = np.stack([v[start + i * stride] for i in range(count)]).reshape(-1) if count else np.empty(0, np.uint8)
        if not np.array_equal(oracle.copy_range(x, start, stride, count, e, mutant=m), ref):
            return False
    return True


def pin_gather_invariants(m=0):
    """Identity indices = memcpy; a permutation followed by its inverse = identity;
    a range read equals the gather of the same arithmetic progression."""
    e, n = 4, 257
    x = rr_synth.random_bytes(61, n * e)
    if not np.array_equal(oracle.gather(x, np.arange(n), e, mutant=m), x):
        return False
    p = rr_synth.rng(62).permutation(n)
    y = oracle.gather(x, p, e, mutant=m)
    if not np.array_equal(oracle.gather(y, np.argsort(p), e, mutant=m), x):
        return False
    for start, stride, count in [(3, 7, 30), (250, -4, 60), (9, 0, 5)]:
        prog = start + stride * np.arange(count)
        if not np.array_equal(oracle.copy_range(x, start, stride, count, e, mutant=m), oracle.gather(x, prog, e, mutant=m)):
            return False
    return True


def _interior(a, r):
    return a[r:a.shape[0] - r, r:a.shape[1] - r]


def pin_stencil_closed_forms(m=0):
    """FD stencils of orders I-IV against closed forms evaluated with the very
    float32 weights given: u = i^2 + j^2 (ring k = 4u + 4k^2), u = i^4 and
    u = j^4 (ring k = 4u + 12 i^2 k^2 + 2 k^4); with exact weights these are the
    Laplacians 4 and 12 i^2 (the order-I weights are exact, so 4 exactly)."""
    rows, cols = 24, 20
    i = np.arange(rows, dtype=np.float64)[:, None] * np.ones((1, cols))
    j = np.ones((rows, 1)) * np.arange(cols, dtype=np.float64)[None, :]
    for r, c in rr_synth.FD_LAPLACIAN.items():
        w = np.asarray(c, dtype=np.float32).astype(np.float64)
        s0 = w[0] + 4 * w[1:].sum()
        k = np.arange(1, r + 1, dtype=np.float64)
        wk, kk = w[1:, None, None], k[:, None, None]
        for u, expect in ((i ** 2 + j ** 2, lambda u: u * s0 + 4 * (w[1:] * k ** 2).sum()),
                          (i ** 4, lambda u: u * s0 + (wk * (12 * i ** 2 * kk ** 2 + 2 * kk ** 4)).sum(axis=0)),
                          (j ** 4, lambda u: u * s0 + (wk * (12 * j ** 2 * kk ** 2 + 2 * kk ** 4)).sum(axis=0))):
            got = oracle.stencil2d(u.astype(np.float32), r, c, mutant=m)
            ref = expect(u)
            ref = ref if np.ndim(ref) else np.full(u.shape, ref)
            if not np.allclose(_interior(got, r), _interior(ref, r), rtol=1e-12, atol=1e-9):
                return False
            if not np.array_equal(got[:r], u[:r]) or not np.array_equal(got[:, -r:], u[:, -r:]):
                return False
        if r == 1 and not np.array_equal(_interior(oracle.stencil2d((i ** 2 + j ** 2).astype(np.float32), 1, c,
                                                                    mutant=m), 1), np.full((rows - 2, cols - 2), 4.0)):
            return False
    return True


def pin_stencil_scipy(m=0):
    """Star and box stencils == scipy.ndimage.correlate (float64) on the interior;
    a star equals the box with the star's weights embedded."""
    from scipy import ndimage
    g = rr_synth.rng(81)
    for t in range(12):
        r = int(g.integers(1, 5))
        rows, cols = int(g.integers(2 * r + 1, 40)), int(g.integers(2 * r + 1, 40))
        x = rr_synth.random_grid(90 + t, rows, cols)
        n = 2 * r + 1
        box = g.uniform(-1, 1, (n, n)).astype(np.float32)
        got = oracle.stencil2d(x, r, box, oracle.STENCIL_BOX, mutant=m)
        ref = ndimage.correlate(x.astype(np.float64), box.astype(np.float64), mode="constant")
        if not np.allclose(_interior(got, r), _interior(ref, r), rtol=1e-12, atol=1e-12):
            return False
        star = g.uniform(-1, 1, r + 1).astype(np.float32)
        sbox = np.zeros((n, n), dtype=np.float32)
        sbox[r, r] = star[0]
        for k in range(1, r + 1):
            sbox[r - k, r] = sbox[r + k, r] = sbox[r, r - k] = sbox[r, r + k] = star[k]
        a = oracle.stencil2d(x, r, star, oracle.STENCIL_STAR, mutant=m)
        b = ndimage.correlate(x.astype(np.float64), sbox.astype(np.float64), mode="constant")
        if not np.allclose(_interior(a, r), _interior(b, r), rtol=1e-12, atol=1e-12):
            return False
    return True


def pin_permute_at(m=0):
    dims, perm, e = (6, 5, 7, 3), (3, 0, 2, 1), 4
    x = rr_synth.random_bytes(21, int(np.prod(dims)) * e)
    full = _np_permute(x, dims, perm, e).reshape(-1, e)
    idx = np.array([0, 1, 17, 200, int(np.prod(dims)) - 1], dtype=np.int64)
    return np.array_equal(oracle.permute_at(x, dims, perm, e, idx, mutant=m), full[idx])


def pin_permute_range(m=0, golden_dir=None):
    """Output pieces: every split of the hand-worked permute fixtures, and random
    [a, b) ranges of random shapes against NumPy's transpose."""
    if golden_dir is not None:
        for case in golden_io.load_all(golden_dir):
            if case["op"] != "permute":
                continue
            e = case.get("esize", [4])[0]
            n = int(np.prod(case["dims"]))
            x = _iota(n * e)
            for k in range(n + 1):
                a = oracle.permute_range(x, case["dims"], case["perm"], e, 0, k, mutant=m)
                b = oracle.permute_range(x, case["dims"], case["perm"], e, k, n - k, mutant=m)
                if np.concatenate([a, b]).tolist() != case["expect"]:
                    return False
    g = rr_synth.rng(44)
    for dims, perm, e in [((6, 5, 7, 3), (3, 0, 2, 1), 4), ((9, 11), (1, 0), 3), ((4, 3, 5, 2, 3), (4, 2, 0, 3, 1), 2),
                          ((17, 13, 5), (2, 0, 1), 8)]:
        n = int(np.prod(dims))
        x = rr_synth.random_bytes(22, n * e)
        full = _np_permute(x, dims, perm, e)
        for _ in range(6):
            a = int(g.integers(0, n))
            c = int(g.integers(0, n - a + 1))
            if not np.array_equal(oracle.permute_range(x, dims, perm, e, a, c, mutant=m), full[a * e:(a + c) * e]):
                return False
    return True


ALL_PINS = {
    "identity": lambda gd, m: pin_identity_is_memcpy(m),
    "golden": lambda gd, m: pin_golden(gd, m),
    "numpy": lambda gd, m: pin_numpy_random(m),
    "brute": lambda gd, m: pin_brute_force(m),
    "inverse": lambda gd, m: pin_inverse_and_composition(m),
    "esize_split": lambda gd, m: pin_esize_split(m),
    "interlace": lambda gd, m: pin_interlace_numpy(m),
    "paper_notation": lambda gd, m: pin_paper_notation(m),
    "permute_at": lambda gd, m: pin_permute_at(m),
    "permute_range": lambda gd, m: pin_permute_range(m, gd),
    "reorder_slice_numpy": lambda gd, m: pin_reorder_slice_numpy(m),
    "reorder_slice_permute": lambda gd, m: pin_reorder_slice_reduces_to_permute(m),
    "gather_range_numpy": lambda gd, m: pin_gather_and_range_numpy(m),
    "gather_invariants": lambda gd, m: pin_gather_invariants(m),
    "stencil_closed_forms": lambda gd, m: pin_stencil_closed_forms(m),
    "stencil_scipy": lambda gd, m: pin_stencil_scipy(m),
}


@pytest.mark.parametrize("name", sorted(ALL_PINS))
def test_oracle_pin(name, golden_dir):
    assert oracle.mutant_id(0) == 0
    assert ALL_PINS[name](golden_dir, 0), f"oracle fails pin {name}"


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_planted_mistake_is_caught(mutant, golden_dir):
    """Each planted oracle mistake (gather/scatter swap, dropped term, wrong stride,
    transposed interlace, fixed axes read at 0, box start ignored, index set read
    one late, range start ignored, stencil's vertical neighbours taken along the
    row) must fail at least one pin."""
    oracle.build(mutant, force=False)
    assert oracle.mutant_id(mutant) == mutant
    failed = []
    for name, fn in ALL_PINS.items():
        try:
            ok = fn(golden_dir, mutant)
        except Exception:
            ok = False
        if not ok:
            failed.append(name)
    assert failed, f"mutant {mutant} passed every pin"


def test_paper_table_orders_convert():
    """Orders of Tables 1 and 2 mapped to row-major perms (reading of Sec. III.B)."""
    expect = {
        (0, 2, 1): (1, 0, 2), (1, 0, 2): (0, 2, 1), (1, 2, 0): (2, 0, 1),
        (2, 0, 1): (1, 2, 0), (2, 1, 0): (2, 1, 0), (1, 0, 2, 3): (0, 1, 3, 2),
        (3, 2, 0, 1): (2, 3, 1, 0), (3, 0, 2, 1, 4): (0, 3, 2, 4, 1),
    }
    for order, perm in expect.items():
        assert paper_order_to_numpy_perm(order) == perm


def test_paper_table2_shapes_small_esize():
    """Table 2 reorders (2^24 elements each) at 1-byte elements: paper notation == NumPy."""
    for sizes, order in rr_synth.PAPER_TABLE2[:2]:
        x = rr_synth.random_bytes(8, int(np.prod(sizes)))
        a = oracle.reorder_paper(x, sizes, order, 1)
        c = _np_permute(x, tuple(reversed(sizes)), paper_order_to_numpy_perm(order), 1)
        assert np.array_equal(a, c)
