"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no rearrangement arithmetic: it only produces random bytes,
array shapes, job lists and arrival times from a seed, so that the GPU library
and the CPU oracle can be fed identical inputs without sharing any code.

Workload shapes follow the paper's experiments (3-D permutes of Table 1, the
reorder shapes of Table 2, the interlace sizes of Table 3) and the dense,
batched and served workloads this library is benchmarked on.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def random_bytes(seed: int, nbytes: int) -> np.ndarray:
    """``nbytes`` uniformly random bytes (uint8) from ``seed``."""
    if nbytes == 0:
        return np.empty(0, dtype=np.uint8)
    return np.frombuffer(rng(seed).bytes(int(nbytes)), dtype=np.uint8).copy()


def all_perms(ndim: int):
    return list(itertools.permutations(range(ndim)))


# ---------------------------------------------------------------------------
# Dense workload catalogue
# ---------------------------------------------------------------------------
ESIZES = (1, 2, 4, 8, 16)

#: Dense N-D permutes of random bits: (name, dims, perm).  Every case runs at
#: every element size in ESIZES.
DENSE_CASES = (
    [("3d_512x512x256", (512, 512, 256), p) for p in all_perms(3)]
    + [("4d_64x128x128x64", (64, 128, 128, 64), (0, 3, 1, 2)),
       ("4d_64x128x128x64", (64, 128, 128, 64), (0, 2, 3, 1)),
       ("5d_32^5", (32, 32, 32, 32, 32), (4, 2, 0, 3, 1)),
       ("2d_16384x16384", (16384, 16384), (1, 0))]
)

#: Small first case: 1024x1024 4-byte transpose.
SMALL_CASE = ("2d_1024x1024", (1024, 1024), (1, 0), 4)

#: Interlace workloads: (name, n planes, count per plane, element size).
INTERLACE_CASES = (
    ("complex64_split", 2, 1 << 27, 4),
    ("rgba_u8_planar", 4, 1 << 28, 1),
    ("xyz_f32_soa", 3, 1 << 26, 4),
)

#: The paper's Table 1 shape (fastest-first sizes 128x256x512 -> row-major
#: dims (512, 256, 128)) and Table 2 shapes, written in the paper's notation.
PAPER_TABLE1_SIZES = (128, 256, 512)
PAPER_TABLE2 = (
    ((256, 256, 256), (1, 0, 2)),
    ((256, 256, 256, 1), (1, 0, 2, 3)),
    ((256, 256, 1, 256), (3, 2, 0, 1)),
    ((256, 16, 1, 256, 16), (3, 0, 2, 1, 4)),
)


# ---------------------------------------------------------------------------
# Batched uneven jobs
# ---------------------------------------------------------------------------
def sample_jobs(seed: int, njobs: int = 4096, ndim_range=(2, 5), max_dim: int = 1024,
                total_range=(1e3, 1e7), esizes=(2, 4, 8), footprint_cap: int = 16 << 30):
    """Random uneven permute jobs.

    Each job: ndim ~ U{2..5}; total element count T log-uniform in
    [1e3, min(1e7, max_dim**ndim)]; log2(T) split into ndim random shares, each
    dim clamped to [1, max_dim]; element size uniform over ``esizes``; a random
    axis permutation.  While the summed in+out footprint exceeds
    ``footprint_cap`` the largest job is redrawn from the same stream.

    Returns a list of dicts {dims, perm, esize}.
    """
    g = rng(seed)
    lo_nd, hi_nd = ndim_range

    def draw():
        nd = int(g.integers(lo_nd, hi_nd + 1))
        hi = min(total_range[1], float(max_dim) ** nd)
        lt = g.uniform(math.log(total_range[0]), math.log(hi))
        log2t = lt / math.log(2.0)
        w = g.dirichlet(np.ones(nd))
        dims = []
        for share in w:
            d = int(round(2.0 ** (share * log2t)))
            dims.append(max(1, min(max_dim, d)))
        esize = int(g.choice(esizes))
        perm = tuple(int(x) for x in g.permutation(nd))
        return {"dims": tuple(dims), "perm": perm, "esize": esize}

    jobs = [draw() for _ in range(njobs)]

    def foot(j):
        return 2 * int(np.prod(j["dims"], dtype=np.int64)) * j["esize"]

    total = sum(foot(j) for j in jobs)
    while total > footprint_cap:
        k = max(range(njobs), key=lambda i: foot(jobs[i]))
        total -= foot(jobs[k])
        jobs[k] = draw()
        total += foot(jobs[k])
    return jobs


def large_jobs(seed: int, count: int, lo_bytes: int = 1 << 30, hi_bytes: int = 4 << 30,
               esizes=(2, 4, 8)):
    """Large 3-D/4-D non-identity permutes of lo..hi bytes per side."""
    g = rng(seed)
    out = []
    for _ in range(count):
        nd = int(g.integers(3, 5))
        e = int(g.choice(esizes))
        target = int(g.uniform(lo_bytes, hi_bytes)) // e
        # power-of-two-ish extents whose product is close to target
        log2t = max(nd, int(round(math.log2(max(2, target)))))
        shares = np.full(nd, log2t // nd)
        shares[: log2t % nd] += 1
        g.shuffle(shares)
        dims = tuple(int(1 << int(s)) for s in shares)
        while True:
            perm = tuple(int(x) for x in g.permutation(nd))
            if perm != tuple(range(nd)):
                break
        out.append({"dims": dims, "perm": perm, "esize": e})
    return out


def poisson_arrivals(seed: int, rate_hz: float, count: int) -> np.ndarray:
    """Scheduled arrival times (seconds from 0) of a Poisson process."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_hz, size=count)
    return np.cumsum(gaps)


# 2-D finite-difference stencils of orders I-IV (the paper's measured stencil
# family, Sec. III.D / Fig. 2): the 2-D Laplacian from the textbook central
# differences of the second derivative with accuracy 2, 4, 6 and 8, as star
# weights (center, then one weight per distance along the axes).  They are
# workload parameters (the user's stencil), handed to the library and the oracle alike.
FD_LAPLACIAN = {
    1: (-4.0, 1.0),
    2: (-5.0, 4.0 / 3.0, -1.0 / 12.0),
    3: (-49.0 / 9.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0),
    4: (-205.0 / 36.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0),
}

# stencil grids: Table 4's 4096 x 4096 single-precision data set, and a larger one
STENCIL_GRIDS = [(4096, 4096), (16384, 16384)]


def random_grid(seed: int, rows: int, cols: int) -> np.ndarray:
    """float32 grid of values uniform in [-1, 1) (seeded)."""
    return rng(seed).uniform(-1.0, 1.0, size=(rows, cols)).astype(np.float32)
