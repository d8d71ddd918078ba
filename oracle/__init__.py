"""CPU correctness oracle for the data-rearrangement operations.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never loads it and
shares no code with it.

The arithmetic lives in ``rr_oracle.c`` (plain loop nests, one memcpy per
element); this module only compiles it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rr_oracle.c")


def lib_path(mutant: int = 0) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_mutant{mutant}.so"
    return os.path.join(_HERE, name)


def build(mutant: int = 0, force: bool = True) -> str:
    """Compile the oracle (or a planted-mistake mutant) with gcc."""
    out = lib_path(mutant)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c99", "-shared", "-fPIC", f"-DRR_ORACLE_MUTANT={mutant}",
           "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_libs: dict[int, ctypes.CDLL] = {}


def _lib(mutant: int = 0) -> ctypes.CDLL:
    if mutant not in _libs:
        path = build(mutant, force=False)
        lib = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        lib.oracle_permute.argtypes = [vp, vp, ctypes.c_int, i64p, ip, ctypes.c_int]
        lib.oracle_permute_at.argtypes = [vp, vp, ctypes.c_int, i64p, ip, ctypes.c_int,
                                          i64p, ctypes.c_int64]
        lib.oracle_permute_range.argtypes = [vp, vp, ctypes.c_int, i64p, ip, ctypes.c_int,
                                             ctypes.c_int64, ctypes.c_int64]
        lib.oracle_reorder_paper.argtypes = [vp, vp, ctypes.c_int, i64p, ip, ctypes.c_int]
        lib.oracle_reorder_slice.argtypes = [vp, vp, ctypes.c_int, i64p, i64p, i64p, ctypes.c_int, ip,
                                             ctypes.c_int]
        lib.oracle_gather.argtypes = [vp, vp, ctypes.c_int64, i64p, ctypes.c_int64, ctypes.c_int]
        lib.oracle_copy_range.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int]
        lib.oracle_stencil2d.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp]
        lib.oracle_interlace.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int,
                                         ctypes.c_int64, ctypes.c_int]
        lib.oracle_deinterlace.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_int,
                                           ctypes.c_int64, ctypes.c_int]
        for f in ("oracle_permute", "oracle_permute_at", "oracle_permute_range", "oracle_reorder_paper", "oracle_reorder_slice",
                  "oracle_gather", "oracle_copy_range", "oracle_stencil2d",
                  "oracle_interlace", "oracle_deinterlace", "oracle_mutant_id"):
            getattr(lib, f).restype = ctypes.c_int
        _libs[mutant] = lib
    return _libs[mutant]


def _i64(seq):
    arr = (ctypes.c_int64 * max(1, len(seq)))(*[int(x) for x in seq])
    return arr


def _i32(seq):
    return (ctypes.c_int * max(1, len(seq)))(*[int(x) for x in seq])


def _as_bytes(buf: np.ndarray) -> np.ndarray:
    if not buf.flags.c_contiguous:
        raise ValueError("oracle needs C-contiguous buffers")
    return buf.view(np.uint8).reshape(-1)


def permute(src: np.ndarray, dims, perm, esize: int, mutant: int = 0) -> np.ndarray:
    """Row-major permute of an array of ``prod(dims)`` elements of ``esize`` bytes.

    ``src`` is any C-contiguous buffer holding exactly prod(dims)*esize bytes.
    Returns a flat uint8 array holding the output bytes.
    """
    dims = [int(d) for d in dims]
    perm = [int(p) for p in perm]
    n = int(np.prod(dims, dtype=np.int64)) if dims else 1
    sb = _as_bytes(src)
    if sb.size != n * esize:
        raise ValueError(f"src holds {sb.size} bytes, expected {n * esize}")
    out = np.empty(n * esize, dtype=np.uint8)
    rc = _lib(mutant).oracle_permute(out.ctypes.data, sb.ctypes.data, len(dims), _i64(dims),
                                     _i32(perm), esize)
    if rc != 0:
        raise ValueError("oracle_permute rejected its arguments")
    return out


def permute_at(src: np.ndarray, dims, perm, esize: int, out_index, mutant: int = 0) -> np.ndarray:
    """Output elements at the given output linear indices (shape (count, esize) uint8)."""
    idx = np.ascontiguousarray(np.asarray(out_index, dtype=np.int64))
    sb = _as_bytes(src)
    out = np.empty((idx.size, esize), dtype=np.uint8)
    rc = _lib(mutant).oracle_permute_at(
        out.ctypes.data, sb.ctypes.data, len(dims), _i64(dims), _i32(perm), esize,
        idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.size)
    if rc != 0:
        raise ValueError("oracle_permute_at rejected its arguments")
    return out


def permute_range(src: np.ndarray, dims, perm, esize: int, o_begin: int, o_count: int,
                  mutant: int = 0) -> np.ndarray:
    """Output elements o_begin .. o_begin + o_count - 1 of the permute, as a flat
    uint8 array of o_count * esize bytes.  The C call releases the GIL, so
    several ranges can be computed at once from threads."""
    dims = [int(d) for d in dims]
    perm = [int(p) for p in perm]
    sb = _as_bytes(src)
    out = np.empty(int(o_count) * esize, dtype=np.uint8)
    rc = _lib(mutant).oracle_permute_range(out.ctypes.data, sb.ctypes.data, len(dims), _i64(dims), _i32(perm),
                                           esize, int(o_begin), int(o_count))
    if rc != 0:
        raise ValueError("oracle_permute_range rejected its arguments")
    return out


def reorder_paper(src: np.ndarray, sizes, order, esize: int, mutant: int = 0) -> np.ndarray:
    """Reorder in the paper's fastest-dimension-first notation (flat uint8 result)."""
    sizes = [int(s) for s in sizes]
    n = int(np.prod(sizes, dtype=np.int64))
    sb = _as_bytes(src)
    out = np.empty(n * esize, dtype=np.uint8)
    rc = _lib(mutant).oracle_reorder_paper(out.ctypes.data, sb.ctypes.data, len(sizes),
                                           _i64(sizes), _i32(order), esize)
    if rc != 0:
        raise ValueError("oracle_reorder_paper rejected its arguments")
    return out


def reorder_slice(src: np.ndarray, dims, base, range_, order, esize: int, mutant: int = 0) -> np.ndarray:
    """N-to-M reorder: output axis j runs over input axis order[j] from base for
    range steps; unlisted input axes stay at their base (flat uint8 result)."""
    dims = [int(d) for d in dims]
    base = [int(b) for b in base]
    range_ = [int(r) for r in range_]
    order = [int(o) for o in order]
    n = int(np.prod([range_[o] for o in order], dtype=np.int64)) if order else 1
    sb = _as_bytes(src)
    if sb.size != int(np.prod(dims, dtype=np.int64)) * esize:
        raise ValueError("src does not hold prod(dims) elements")
    out = np.empty(n * esize, dtype=np.uint8)
    rc = _lib(mutant).oracle_reorder_slice(out.ctypes.data, sb.ctypes.data, len(dims), _i64(dims), _i64(base),
                                           _i64(range_), len(order), _i32(order), esize)
    if rc != 0:
        raise ValueError("oracle_reorder_slice rejected its arguments")
    return out


def gather(src: np.ndarray, idx, esize: int, mutant: int = 0) -> np.ndarray:
    """dst[i] = src[idx[i]] over elements of esize bytes (flat uint8 result)."""
    sb = _as_bytes(src)
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(ix.size * esize, dtype=np.uint8)
    rc = _lib(mutant).oracle_gather(out.ctypes.data, sb.ctypes.data, sb.size // esize,
                                    ix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ix.size, esize)
    if rc != 0:
        raise ValueError("oracle_gather rejected its arguments")
    return out


def copy_range(src: np.ndarray, start: int, stride: int, count: int, esize: int, mutant: int = 0) -> np.ndarray:
    """dst[i] = src[start + i*stride] over elements of esize bytes (flat uint8 result)."""
    sb = _as_bytes(src)
    out = np.empty(count * esize, dtype=np.uint8)
    rc = _lib(mutant).oracle_copy_range(out.ctypes.data, sb.ctypes.data, sb.size // esize, int(start), int(stride),
                                        int(count), esize)
    if rc != 0:
        raise ValueError("oracle_copy_range rejected its arguments")
    return out


# stencil shapes: star (weights: center, then one weight per distance along the
# axes) and box (a full (2r+1) x (2r+1) weight matrix)
STENCIL_STAR, STENCIL_BOX = 0, 1


def stencil2d(src: np.ndarray, radius: int, weights, shape: int = STENCIL_STAR, mutant: int = 0) -> np.ndarray:
    """2-D stencil of a (rows, cols) float32 array, evaluated in float64; points
    closer than radius to an edge keep their input value.  Returns float64."""
    x = np.ascontiguousarray(src, dtype=np.float32)
    if x.ndim != 2:
        raise ValueError("stencil2d needs a 2-D array")
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).reshape(-1))
    need = radius + 1 if shape == STENCIL_STAR else (2 * radius + 1) ** 2
    if w.size != need:
        raise ValueError(f"expected {need} weights")
    out = np.empty(x.shape, dtype=np.float64)
    rc = _lib(mutant).oracle_stencil2d(out.ctypes.data, x.ctypes.data, x.shape[0], x.shape[1], int(radius),
                                       int(shape), w.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_stencil2d rejected its arguments")
    return out


def interlace(planes, esize: int, mutant: int = 0) -> np.ndarray:
    """Join n planes (each a buffer of count*esize bytes) with the plane index fastest."""
    bufs = [_as_bytes(p) for p in planes]
    n = len(bufs)
    count = bufs[0].size // esize
    if any(b.size != count * esize for b in bufs):
        raise ValueError("planes must hold equal byte counts")
    out = np.empty(n * count * esize, dtype=np.uint8)
    ptrs = (ctypes.c_void_p * n)(*[b.ctypes.data for b in bufs])
    rc = _lib(mutant).oracle_interlace(out.ctypes.data, ptrs, n, count, esize)
    if rc != 0:
        raise ValueError("oracle_interlace rejected its arguments")
    return out


def deinterlace(src: np.ndarray, n: int, esize: int, mutant: int = 0) -> list:
    """Split an interlaced buffer into n planes (list of flat uint8 arrays)."""
    sb = _as_bytes(src)
    count = sb.size // (n * esize)
    if count * n * esize != sb.size:
        raise ValueError("interlaced buffer is not a whole number of tuples")
    outs = [np.empty(count * esize, dtype=np.uint8) for _ in range(n)]
    ptrs = (ctypes.c_void_p * n)(*[o.ctypes.data for o in outs])
    rc = _lib(mutant).oracle_deinterlace(ptrs, sb.ctypes.data, n, count, esize)
    if rc != 0:
        raise ValueError("oracle_deinterlace rejected its arguments")
    return outs


def mutant_id(mutant: int = 0) -> int:
    return int(_lib(mutant).oracle_mutant_id())
