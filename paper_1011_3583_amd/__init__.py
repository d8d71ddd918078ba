"""Python binding of librr: N-D permute, interlace / de-interlace, batched and
served permutes on one MI355X.

Argument marshalling only.  Every byte is moved by the HIP kernels in
``librr.so`` (built in-tree by ``python -m paper_1011_3583_amd.build``); if the
library is missing this module raises instead of falling back to anything.
PyTorch supplies device memory and streams for the tensor helpers.

Conventions (row-major, NumPy-style perms) follow the C header include/rr.h.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librr.so")

RR_MAX_DIMS = 8
RR_MAX_PLANES = 16

STATUS = {0: "RR_OK", 1: "RR_ERR_INVALID_ARG", 2: "RR_ERR_OVERFLOW", 3: "RR_ERR_ALIAS",
          4: "RR_ERR_UNSUPPORTED", 5: "RR_ERR_NO_MEMORY", 6: "RR_ERR_BUSY",
          7: "RR_ERR_NOT_READY", 8: "RR_ERR_HIP"}
STATUS_CODE = {v: k for k, v in STATUS.items()}
RR_OK, RR_ERR_NOT_READY = 0, 7

EXPORTS = ("rr_permute", "rr_reorder", "rr_gather", "rr_copy_range", "rr_stencil2d", "rr_interlace", "rr_deinterlace",
           "rr_permute_batched", "rr_permute_batched_noalloc",
           "rr_batch_create", "rr_batch_launch", "rr_batch_get_info", "rr_batch_describe", "rr_batch_destroy",
           "rr_serve_create", "rr_serve_alloc", "rr_serve_free", "rr_serve_submit",
           "rr_serve_poll", "rr_serve_completions", "rr_serve_release", "rr_serve_destroy",
           "rr_serve_get_stats", "rr_serve_fail_next_batch",
           "rr_order_to_perm", "rr_plan_describe", "rr_reorder_describe", "rr_interlace_describe",
           "rr_set_tile_override",
           "rr_tune_permute", "rr_tune_save", "rr_tune_load", "rr_tune_clear", "rr_tune_context",
           "rr_status_string", "rr_last_error", "rr_version")


class RRError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


class Job(ctypes.Structure):
    _fields_ = [("dst", ctypes.c_void_p), ("src", ctypes.c_void_p), ("ndim", ctypes.c_int32),
                ("elem_size", ctypes.c_int32), ("dims", ctypes.c_int64 * RR_MAX_DIMS),
                ("perm", ctypes.c_int32 * RR_MAX_DIMS)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_jobs", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("chunk_bytes", ctypes.c_uint64),
                ("tick_us", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("sim_bytes_per_us", ctypes.c_double), ("sim_device_bytes", ctypes.c_uint64)]


RR_SERVE_SIMULATED, RR_SERVE_DIRECT = 1, 2


class JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("chunks", ctypes.c_int32), ("dst", ctypes.c_void_p),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_launch_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("njobs", ctypes.c_int32), ("ngroups", ctypes.c_int32), ("in_row_bytes", ctypes.c_int32),
                ("out_row_bytes", ctypes.c_int32), ("order_out", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("bytes", ctypes.c_uint64), ("tuned_us", ctypes.c_double),
                ("tile_kib", ctypes.c_int32), ("cache", ctypes.c_int32), ("fill", ctypes.c_int32),
                ("force_ragged", ctypes.c_int32)]


RR_BATCH_GRAPH, RR_BATCH_TUNE, RR_BATCH_PERSISTENT, RR_BATCH_SERIAL = 1, 2, 4, 8


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "failed", "batches", "chunks",
                                               "bytes_moved", "budget_peak", "budget_used", "reserved")]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1011_3583_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)
    L.rr_permute.argtypes = [vp, vp, i32, i64p, i32p, i32, vp]
    L.rr_interlace.argtypes = [vp, ctypes.POINTER(vp), i32, i64, i32, vp]
    L.rr_deinterlace.argtypes = [ctypes.POINTER(vp), vp, i32, i64, i32, vp]
    L.rr_permute_batched.argtypes = [ctypes.POINTER(Job), i32, vp]
    L.rr_permute_batched_noalloc.argtypes = [ctypes.POINTER(Job), i32, vp]
    L.rr_batch_create.argtypes = [ctypes.POINTER(Job), i32, i32, ctypes.POINTER(vp)]
    L.rr_batch_launch.argtypes = [vp, vp]
    L.rr_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.rr_batch_describe.argtypes = [vp, ctypes.c_char_p, i32]
    L.rr_batch_destroy.argtypes = [vp]
    L.rr_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
    L.rr_serve_alloc.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
    L.rr_serve_free.argtypes = [vp, vp]
    L.rr_serve_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
    L.rr_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(JobResult)]
    L.rr_serve_release.argtypes = [vp, ctypes.c_uint64]
    L.rr_serve_completions.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32, ctypes.POINTER(ctypes.c_int)]
    L.rr_serve_fail_next_batch.argtypes = [vp]
    L.rr_serve_destroy.argtypes = [vp]
    L.rr_serve_get_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    L.rr_order_to_perm.argtypes = [i32, i32p, i32p]
    L.rr_plan_describe.argtypes = [vp, vp, i32, i64p, i32p, i32, ctypes.c_char_p, i32]
    L.rr_reorder.argtypes = [vp, vp, i32, i64p, i64p, i64p, i32, i32p, i32, vp]
    L.rr_gather.argtypes = [vp, vp, i64, vp, i64, i32, vp, vp]
    L.rr_copy_range.argtypes = [vp, vp, i64, i64, i64, i64, i32, vp]
    L.rr_stencil2d.argtypes = [vp, vp, i64, i64, i32, i32, ctypes.POINTER(ctypes.c_float), vp]
    L.rr_reorder_describe.argtypes = [vp, vp, i32, i64p, i64p, i64p, i32, i32p, i32, ctypes.c_char_p, i32]
    L.rr_interlace_describe.argtypes = [vp, vp, i32, i64, i32, i32, ctypes.c_char_p, i32]
    L.rr_set_tile_override.argtypes = [i32, i32, i32]
    L.rr_tune_context.argtypes = [ctypes.c_char_p, i32]
    L.rr_tune_permute.argtypes = [vp, vp, i32, i64p, i32p, i32, vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    L.rr_tune_save.argtypes = [ctypes.c_char_p]
    L.rr_tune_load.argtypes = [ctypes.c_char_p]
    L.rr_status_string.argtypes = [i32]
    L.rr_status_string.restype = ctypes.c_char_p
    L.rr_last_error.restype = ctypes.c_char_p
    L.rr_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("rr_status_string", "rr_last_error", "rr_version"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def last_error() -> str:
    return lib().rr_last_error().decode()


def check(status: int) -> int:
    if status != RR_OK:
        raise RRError(status, last_error())
    return status


def _i64(seq):
    return (ctypes.c_int64 * max(1, len(seq)))(*[int(x) for x in seq])


def _i32(seq):
    return (ctypes.c_int * max(1, len(seq)))(*[int(x) for x in seq])


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------------- raw pointer API
def permute_raw(dst: int, src: int, dims, perm, elem_size: int, stream=0) -> int:
    """rr_permute on raw device addresses; returns the rr_status (no raise)."""
    return lib().rr_permute(dst, src, len(dims), _i64(dims), _i32(perm), int(elem_size),
                            _stream_handle(stream))


def _opt_i64(seq):
    return None if seq is None else _i64(seq)


def reorder_raw(dst: int, src: int, dims, base, range_, order, elem_size: int, stream=0) -> int:
    """rr_reorder (N-to-M box reorder) on raw device addresses; returns the rr_status.
    base / range_ may be None (zeros / to the end)."""
    return lib().rr_reorder(dst, src, len(dims), _i64(dims), _opt_i64(base), _opt_i64(range_), len(order),
                            _i32(order), int(elem_size), _stream_handle(stream))


def gather_raw(dst: int, src: int, src_count: int, idx: int, count: int, elem_size: int, bad: int = 0,
               stream=0) -> int:
    """rr_gather on raw device addresses (idx: device int64 array; bad: device
    uint64 counter or 0); returns the rr_status."""
    return lib().rr_gather(dst, src, int(src_count), idx, int(count), int(elem_size), bad or None,
                           _stream_handle(stream))


def copy_range_raw(dst: int, src: int, src_count: int, start: int, stride: int, count: int, elem_size: int,
                   stream=0) -> int:
    """rr_copy_range on raw device addresses; returns the rr_status."""
    return lib().rr_copy_range(dst, src, int(src_count), int(start), int(stride), int(count), int(elem_size),
                               _stream_handle(stream))


STENCIL_STAR, STENCIL_BOX = 0, 1


def stencil2d_raw(dst: int, src: int, rows: int, cols: int, radius: int, weights, shape: int = STENCIL_STAR,
                  stream=0) -> int:
    """rr_stencil2d on raw device addresses of float grids; returns the rr_status."""
    w = (ctypes.c_float * max(1, len(weights)))(*[float(x) for x in weights])
    return lib().rr_stencil2d(dst, src, int(rows), int(cols), int(radius), int(shape), w, _stream_handle(stream))


def interlace_raw(dst: int, srcs, count: int, elem_size: int, stream=0) -> int:
    n = len(srcs)
    arr = (ctypes.c_void_p * max(1, n))(*srcs)
    return lib().rr_interlace(dst, arr, n, int(count), int(elem_size), _stream_handle(stream))


def deinterlace_raw(dsts, src: int, count: int, elem_size: int, stream=0) -> int:
    n = len(dsts)
    arr = (ctypes.c_void_p * max(1, n))(*dsts)
    return lib().rr_deinterlace(arr, src, n, int(count), int(elem_size), _stream_handle(stream))


def make_jobs(specs):
    """specs: iterable of (dst_ptr, src_ptr, dims, perm, elem_size) -> ctypes array of Job."""
    specs = list(specs)
    arr = (Job * max(1, len(specs)))()
    for i, (d, s, dims, perm, e) in enumerate(specs):
        if len(dims) > RR_MAX_DIMS:
            raise ValueError("too many dims")
        arr[i].dst, arr[i].src, arr[i].ndim, arr[i].elem_size = d, s, len(dims), e
        for k, v in enumerate(dims):
            arr[i].dims[k] = int(v)
        for k, v in enumerate(perm):
            arr[i].perm[k] = int(v)
    return arr


def permute_batched_raw(jobs, njobs: int | None = None, stream=0) -> int:
    if not isinstance(jobs, ctypes.Array):
        n = len(jobs)
        jobs = make_jobs(jobs)
    else:
        n = len(jobs) if njobs is None else njobs
    return lib().rr_permute_batched(jobs, n, _stream_handle(stream))


def permute_batched_noalloc_raw(jobs, njobs: int | None = None, stream=0) -> int:
    """rr_permute_batched_noalloc: the job table in the library's fixed device array."""
    if not isinstance(jobs, ctypes.Array):
        n = len(jobs)
        jobs = make_jobs(jobs)
    else:
        n = len(jobs) if njobs is None else njobs
    return lib().rr_permute_batched_noalloc(jobs, n, _stream_handle(stream))


class Batch:
    """A reusable batch (rr_batch_create / rr_batch_launch / rr_batch_destroy)."""

    def __init__(self, specs, flags: int = 0):
        self._jobs = specs if isinstance(specs, ctypes.Array) else make_jobs(specs)
        n = len(self._jobs) if not isinstance(specs, ctypes.Array) else len(specs)
        if isinstance(specs, (list, tuple)) and len(specs) == 0:
            n = 0
        h = ctypes.c_void_p()
        check(lib().rr_batch_create(self._jobs, n, int(flags), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        check(lib().rr_batch_launch(self.h, _stream_handle(stream)))

    def info(self) -> dict:
        i = BatchInfo()
        check(lib().rr_batch_get_info(self.h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in BatchInfo._fields_}

    def groups(self) -> list:
        """One dict per kernel group (kernel, jobs, workgroups, bytes per side, lds),
        in storage order (the launch order under RR_BATCH_SERIAL)."""
        buf = ctypes.create_string_buffer(1 << 16)
        check(lib().rr_batch_describe(self.h, buf, len(buf)))
        out = []
        for line in buf.value.decode().splitlines():
            d = dict(kv.split("=", 1) for kv in line.split())
            out.append({k: (v if k == "kernel" else int(v)) for k, v in d.items()})
        return out

    def close(self):
        if self.h:
            check(lib().rr_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def order_to_perm(order):
    n = len(order)
    out = (ctypes.c_int * n)()
    check(lib().rr_order_to_perm(n, _i32(order), out))
    return tuple(out)


def plan_describe(dims, perm, elem_size: int, dst: int = 0, src: int = 0) -> dict:
    buf = ctypes.create_string_buffer(1024)
    check(lib().rr_plan_describe(dst, src, len(dims), _i64(dims), _i32(perm), int(elem_size), buf, 1024))
    out = {}
    for tok in buf.value.decode().split():
        k, v = tok.split("=", 1)
        out[k] = v
    return out


def interlace_describe(flat: int, planes, count: int, elem_size: int, de: bool = False) -> dict:
    """The plan rr_interlace (or, de=True, rr_deinterlace) would run for these pointers."""
    buf = ctypes.create_string_buffer(1024)
    arr = (ctypes.c_void_p * max(1, len(planes)))(*planes)
    check(lib().rr_interlace_describe(flat, arr, len(planes), int(count), int(elem_size), int(bool(de)), buf, 1024))
    return dict(tok.split("=", 1) for tok in buf.value.decode().split())


def reorder_describe(dims, base, range_, order, elem_size: int, dst: int = 0, src: int = 0) -> dict:
    buf = ctypes.create_string_buffer(1024)
    check(lib().rr_reorder_describe(dst, src, len(dims), _i64(dims), _opt_i64(base), _opt_i64(range_), len(order),
                                    _i32(order), int(elem_size), buf, 1024))
    return dict(tok.split("=", 1) for tok in buf.value.decode().split())


def set_tile_override(in_row_bytes: int = 0, out_row_bytes: int = 0, order_out=None,
                      force_ragged: bool = False, max_g: int = 0, tile_kib: int = 0, xcd=None,
                      umt: int = 0, cache=None, diag=None, fill=None, weave: bool = True):
    """order_out: True = output order, False = input order, None = built-in choice.
    force_ragged: plan the odd-shape tile path even where aligned micro-tiles fit.
    max_g: cap on the register micro-tile edge (0 = none, else 1, 2, 4, 8, 16).
    tile_kib: LDS size tiles are shrunk to (0 = 16 KiB, else 4..64).
    xcd: True = each XCD takes a contiguous range of tiles (per job in batches), False =
    never, None = where the cache policy reads or writes through the caches.
    umt: unaligned micro-tiles, 1 on odd shapes (instead of G = 1 rows), 2 everywhere.
    cache: global accesses of tiles, 0 non-temporal, 1 loads cached, 2 stores cached,
    3 both; None = the planner's choice by 128-byte line alignment.
    diag: diagonal tile order, True / False on / off, None = built-in (on for 2-D
    transposes at power-of-two row pitches of 4 KiB or more, 1-8-byte elements).  fill: True / False switch the odd-extent refit (fewer,
    fuller tiles where a tile does not divide an outer axis) on / off, None = built-in.
    weave: False sends every interlace and de-interlace through the LDS tile instead of
    the register path for aligned sets of 1-8-byte elements."""
    flags = 0 if order_out is None else (1 if order_out else 2)
    flags |= 4 if force_ragged else 0
    flags |= int(max_g) << 8
    flags |= int(tile_kib) << 16
    flags |= 0 if xcd is None else (8 if xcd else 64)
    flags |= {0: 0, 1: 16, 2: 32}[int(umt)]
    flags |= 0 if cache is None else (int(cache) + 1) << 24
    flags |= 0 if diag is None else (128 if diag else (1 << 30))
    flags |= 0 if fill is None else ((1 << 27) if fill else (1 << 28))
    flags |= 0 if weave else (1 << 29)
    check(lib().rr_set_tile_override(int(in_row_bytes), int(out_row_bytes), flags))


def tune_permute(dst: int, src: int, dims, perm, elem_size: int, stream=None):
    """Autotune one permute problem (runs it); returns (best_us, default_us)."""
    b, d = ctypes.c_double(), ctypes.c_double()
    check(lib().rr_tune_permute(dst, src, len(dims), _i64(dims), _i32(perm), int(elem_size),
                                _stream_handle(stream), ctypes.byref(b), ctypes.byref(d)))
    return b.value, d.value


def tune_save(path: str):
    check(lib().rr_tune_save(path.encode()))


def tune_load(path: str):
    check(lib().rr_tune_load(path.encode()))


def tune_context() -> str:
    """The prefix of this process's tuning-cache keys ("<arch>@hip<version>")."""
    buf = ctypes.create_string_buffer(256)
    check(lib().rr_tune_context(buf, len(buf)))
    return buf.value.decode()


def tune_clear():
    check(lib().rr_tune_clear())


# ----------------------------------------------------------------- torch helpers
def permute(src, perm, out=None, stream=None):
    """Permute a contiguous CUDA tensor (elements copied as opaque bytes)."""
    import torch
    if not src.is_contiguous():
        raise ValueError("src must be contiguous")
    dims = tuple(src.shape)
    perm = tuple(int(p) for p in perm)
    oshape = tuple(dims[p] for p in perm)
    if out is None:
        out = torch.empty(oshape, dtype=src.dtype, device=src.device)
    check(permute_raw(out.data_ptr(), src.data_ptr(), dims, perm, src.element_size(), stream))
    return out


def interlace(planes, out=None, stream=None):
    import torch
    n = len(planes)
    count = planes[0].numel()
    if out is None:
        out = torch.empty((count, n), dtype=planes[0].dtype, device=planes[0].device)
    check(interlace_raw(out.data_ptr(), [p.data_ptr() for p in planes], count, planes[0].element_size(),
                        stream))
    return out


def deinterlace(src, n: int, outs=None, stream=None):
    import torch
    count = src.numel() // n
    if outs is None:
        outs = [torch.empty(count, dtype=src.dtype, device=src.device) for _ in range(n)]
    check(deinterlace_raw([o.data_ptr() for o in outs], src.data_ptr(), count, src.element_size(), stream))
    return outs


class Server:
    """Thin wrapper over rr_serve_*."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4, max_batch_jobs: int = 1024,
                 queue_capacity: int = 1 << 16, chunk_bytes: int = 64 << 20, tick_us: int = 20,
                 device: int = 0, simulated: bool = False, sim_bytes_per_us: float = 0.0,
                 direct: bool = False, sim_device_bytes: int = 0):
        flags = (RR_SERVE_SIMULATED if simulated else 0) | (RR_SERVE_DIRECT if direct else 0)
        cfg = ServeConfig(device, max_inflight, max_batch_jobs, queue_capacity, hbm_budget_bytes,
                          chunk_bytes, tick_us, flags, float(sim_bytes_per_us), int(sim_device_bytes))
        h = ctypes.c_void_p()
        check(lib().rr_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._cq = (ctypes.c_uint64 * 4096)()

    def alloc(self, nbytes: int) -> int:
        p = ctypes.c_void_p()
        check(lib().rr_serve_alloc(self.h, int(nbytes), ctypes.byref(p)))
        return p.value

    def free(self, ptr: int):
        check(lib().rr_serve_free(self.h, ptr))

    def submit_raw(self, job) -> tuple[int, int]:
        t = ctypes.c_uint64()
        st = lib().rr_serve_submit(self.h, ctypes.byref(job), ctypes.byref(t))
        return st, t.value

    def submit(self, dst, src, dims, perm, elem_size) -> int:
        job = make_jobs([(dst or 0, src, dims, perm, elem_size)])[0]
        st, t = self.submit_raw(job)
        check(st)
        return t

    def poll(self, ticket: int):
        r = JobResult()
        st = lib().rr_serve_poll(self.h, int(ticket), ctypes.byref(r))
        if st == RR_ERR_NOT_READY:
            return None
        check(st)
        return r

    def release(self, ticket: int):
        check(lib().rr_serve_release(self.h, int(ticket)))

    def completions(self) -> list:
        """Tickets completed since the last call (oldest first)."""
        out = []
        n = ctypes.c_int()
        while True:
            check(lib().rr_serve_completions(self.h, self._cq, len(self._cq), ctypes.byref(n)))
            out.extend(self._cq[:n.value])
            if n.value < len(self._cq):
                return out

    def fail_next_batch(self):
        check(lib().rr_serve_fail_next_batch(self.h))

    def stats(self) -> dict:
        s = ServeStats()
        check(lib().rr_serve_get_stats(self.h, ctypes.byref(s)))
        return {n: getattr(s, n) for n, _ in ServeStats._fields_}

    def close(self):
        if self.h:
            check(lib().rr_serve_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
