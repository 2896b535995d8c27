"""Thin ctypes binding of the C ABI in ``include/stencil.h``.

Argument marshalling only: every step of the sweep runs in the HIP library.
PyTorch provides device memory and streams (``tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``).  If ``libstencil.so`` is not
built, loading raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# STENCIL_LIBRARY names another build of the same library (the host-side
# sanitizer build of the CPU tests); the default is the in-tree libstencil.so.
LIB_PATH = os.environ.get("STENCIL_LIBRARY") or os.path.join(_HERE, "libstencil.so")

# enums (mirror include/stencil.h)
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, EALIAS, EINTERNAL, ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_SCRATCH_BYTES = 32768  # STENCIL_NOALLOC_SCRATCH_BYTES
STAR, BOX, GENERAL = 0, 1, 2
BC_ZERO, BC_PERIODIC = 0, 1
F32, F64 = 0, 1
PATH_AUTO, PATH_GATHER, PATH_MFMA, PATH_MFMA_BF16X3, PATH_MFMA_F16X3 = 0, 1, 2, 3, 4
LINES_AUTO, LINES_PARALLEL, LINES_ORTHOGONAL, LINES_HYBRID = 0, 1, 2, 3

PATH_NAMES = {PATH_AUTO: "auto", PATH_GATHER: "gather", PATH_MFMA: "mfma",
              PATH_MFMA_BF16X3: "mfma_bf16x3", PATH_MFMA_F16X3: "mfma_f16x3"}


class StencilError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("radius", ctypes.c_int32), ("dims", ctypes.c_int64 * 3),
        ("shape", ctypes.c_int32), ("boundary", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("path", ctypes.c_int32), ("lines", ctypes.c_int32), ("block_n", ctypes.c_int32),
        ("chunk", ctypes.c_int32), ("time_block", ctypes.c_int32),
        ("reg_rows", ctypes.c_int32), ("tile_width", ctypes.c_int32),
        ("coeffs", ctypes.POINTER(ctypes.c_double)),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int32), ("lines", ctypes.c_int32),
        ("ndim", ctypes.c_int32), ("radius", ctypes.c_int32), ("shape", ctypes.c_int32),
        ("boundary", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("taps", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
        ("block_n", ctypes.c_int32), ("mfma_lines", ctypes.c_int32), ("valu_lines", ctypes.c_int32),
        ("k_rows", ctypes.c_int32), ("rank1_per_block", ctypes.c_int64),
        ("useful_flops_per_point", ctypes.c_double), ("executed_flops_per_point", ctypes.c_double),
        ("bytes_per_point", ctypes.c_int32), ("time_block", ctypes.c_int32),
        ("pad0", ctypes.c_int32), ("operand_bytes", ctypes.c_int64),
        ("reg_rows", ctypes.c_int32), ("tile_width", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = [
    "stencil_version", "stencil_status_string", "stencil_desc_check", "stencil_plan_describe",
    "stencil_line_band", "stencil_line_cover", "stencil_plan", "stencil_plan_info", "stencil_plan_destroy",
    "stencil_apply", "stencil_run_steps", "stencil_error_norms",
    "stencil_batch_create", "stencil_batch_run_steps", "stencil_batch_info", "stencil_batch_destroy",
    "stencil_autotune",
    "stencil_server_create", "stencil_server_stream", "stencil_server_submit", "stencil_server_tick",
    "stencil_server_poll", "stencil_server_destroy", "stencil_run_steps_noalloc", "stencil_server_cancel",
]


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32),
                ("max_inflight_ticks", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("tick", ctypes.c_int64), ("arena_in_use", ctypes.c_int64), ("active", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("groups", ctypes.c_int32), ("retired", ctypes.c_int32)]

TUNE_ALLOW_SPLIT, TUNE_FORCE = 1, 2


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int32), ("lines", ctypes.c_int32), ("block_n", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("time_block", ctypes.c_int32), ("reg_rows", ctypes.c_int32), ("tile_width", ctypes.c_int32),
        ("status", ctypes.c_int32), ("ms_per_step", ctypes.c_double),
    ]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libstencil.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2310_16298_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    lib.stencil_version.restype = ctypes.c_char_p
    lib.stencil_status_string.argtypes = [ctypes.c_int]
    lib.stencil_status_string.restype = ctypes.c_char_p
    lib.stencil_desc_check.argtypes = [ctypes.POINTER(Desc)]
    lib.stencil_plan_describe.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(PlanInfo)]
    lib.stencil_line_band.argtypes = [dp, i32, i32, i32, i32, dp]
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.stencil_line_cover.argtypes = [dp, i32, ip, ip, ip]
    lib.stencil_plan.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    lib.stencil_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.stencil_plan_destroy.argtypes = [vp]
    lib.stencil_apply.argtypes = [vp, vp, vp, vp]
    lib.stencil_run_steps.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(i32)]
    lib.stencil_error_norms.argtypes = [vp, i32, vp, i64, vp, vp]
    lib.stencil_run_steps_noalloc.argtypes = [ctypes.POINTER(Desc), vp, vp, i64, vp, ctypes.POINTER(i32)]
    lib.stencil_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32,
                                         ctypes.POINTER(vp)]
    lib.stencil_batch_run_steps.argtypes = [vp, i64, vp, ctypes.POINTER(i32)]
    lib.stencil_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.stencil_batch_destroy.argtypes = [vp]
    lib.stencil_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.stencil_server_stream.argtypes = [vp, ctypes.POINTER(vp)]
    lib.stencil_server_submit.argtypes = [vp, ctypes.POINTER(Desc), vp, vp, i64, ctypes.POINTER(i64)]
    lib.stencil_server_tick.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.stencil_server_poll.argtypes = [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32)]
    lib.stencil_server_destroy.argtypes = [vp]
    lib.stencil_server_cancel.argtypes = [vp, i64]
    lib.stencil_autotune.argtypes = [ctypes.POINTER(Desc), ctypes.c_char_p, i32, ctypes.POINTER(Desc),
                                     ctypes.POINTER(ctypes.c_double), vp, ctypes.POINTER(TuneResult), i32,
                                     ctypes.POINTER(i32)]
    for name in EXPORTS[2:]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load_library().stencil_status_string(int(status)).decode()


def version() -> str:
    return load_library().stencil_version().decode()


def _check(status: int, where: str):
    if status != OK:
        raise StencilError(status, where)


def make_desc(dims: Sequence[int], radius: int, shape: int, coeffs, boundary: int = BC_ZERO,
              dtype: int = F32, path: int = PATH_AUTO, lines: int = LINES_AUTO, block_n: int = 0,
              chunk: int = 0, time_block: int = 0, reg_rows: int = 0, tile_width: int = 0):
    """Build a Desc; returns (desc, keepalive) -- keep the array alive while used."""
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    d = Desc()
    d.ndim = len(dims)
    d.radius = int(radius)
    for k in range(3):
        d.dims[k] = int(dims[k]) if k < len(dims) else 1
    d.shape, d.boundary, d.dtype, d.path, d.lines = int(shape), int(boundary), int(dtype), int(path), int(lines)
    d.block_n, d.chunk, d.time_block = int(block_n), int(chunk), int(time_block)
    d.reg_rows, d.tile_width = int(reg_rows), int(tile_width)
    d.coeffs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d, c


def desc_check(dims, radius, shape, coeffs, **kw) -> int:
    d, keep = make_desc(dims, radius, shape, coeffs, **kw)
    return load_library().stencil_desc_check(ctypes.byref(d))


def describe(dims, radius, shape, coeffs, **kw) -> dict:
    """Host-only: the plan choices and operation counts stencil_plan would make."""
    d, keep = make_desc(dims, radius, shape, coeffs, **kw)
    info = PlanInfo()
    _check(load_library().stencil_plan_describe(ctypes.byref(d), ctypes.byref(info)), "stencil_plan_describe")
    return info.as_dict()


def line_band(coeffs, radius: int, n: int, axis: int, index: int) -> np.ndarray:
    """Host-only: banded operand of one 2D coefficient line (see stencil.h)."""
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    k = n + 2 * radius
    out = np.zeros((n, k) if axis == 0 else (k, n), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load_library().stencil_line_band(c.ctypes.data_as(dp), radius, n, axis, index,
                                            out.ctypes.data_as(dp)), "stencil_line_band")
    return out


def line_cover(coeffs, radius: int):
    """Host-only: minimum axis-parallel line cover of a 2D C^g (Section 3.5).
    Returns (row_lines, col_lines): the indices a of lines CLS(a, *) and b of
    lines CLS(*, b) in the cover."""
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    w = 2 * radius + 1
    rows = (ctypes.c_int32 * w)()
    cols = (ctypes.c_int32 * w)()
    cnt = ctypes.c_int32(0)
    _check(load_library().stencil_line_cover(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), radius, rows,
                                             cols, ctypes.byref(cnt)), "stencil_line_cover")
    rl = [k for k in range(w) if rows[k]]
    cl = [k for k in range(w) if cols[k]]
    assert len(rl) + len(cl) == cnt.value
    return rl, cl


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """A stencil plan on the current device.

    ``Plan(dims, radius, shape, coeffs, boundary, dtype, path, lines, block_n,
    chunk, time_block, reg_rows, tile_width)``; grids
    are torch tensors on the plan's device, contiguous, of the plan's dims and
    dtype (float32 / float64).
    """

    def __init__(self, dims, radius, shape, coeffs, boundary=BC_ZERO, dtype=F32,
                 path=PATH_AUTO, lines=LINES_AUTO, block_n=0, chunk=0, time_block=0, reg_rows=0, tile_width=0):
        lib = load_library()
        self.dims = tuple(int(v) for v in dims)
        self.dtype = dtype
        d, keep = make_desc(self.dims, radius, shape, coeffs, boundary=boundary, dtype=dtype,
                            path=path, lines=lines, block_n=block_n, chunk=chunk, time_block=time_block,
                            reg_rows=reg_rows, tile_width=tile_width)
        h = ctypes.c_void_p()
        _check(lib.stencil_plan(ctypes.byref(d), ctypes.byref(h)), "stencil_plan")
        self._h = h
        self._lib = lib
        self.info = self._info()

    def _info(self) -> dict:
        info = PlanInfo()
        _check(self._lib.stencil_plan_info(self._h, ctypes.byref(info)), "stencil_plan_info")
        return info.as_dict()

    @property
    def handle(self) -> int:
        return self._h.value

    def _validate(self, *tensors):
        torch = _torch()
        want = torch.float64 if self.dtype == F64 else torch.float32
        for t in tensors:
            if not t.is_cuda:
                raise ValueError("grid tensors must be on the GPU")
            if t.dtype != want:
                raise ValueError(f"grid dtype {t.dtype} != plan dtype {want}")
            if not t.is_contiguous():
                raise ValueError("grid tensors must be contiguous")
            if tuple(t.shape) != self.dims:
                raise ValueError(f"grid shape {tuple(t.shape)} != plan dims {self.dims}")

    def apply(self, x, out, stream=None):
        """One Jacobi step out = S(x), enqueued on ``stream``."""
        self._validate(x, out)
        _check(self._lib.stencil_apply(self._h, x.data_ptr(), out.data_ptr(), _stream_ptr(stream)),
               "stencil_apply")
        return out

    def run_steps(self, x, tmp, steps: int, stream=None):
        """``steps`` Jacobi steps ping-ponging between x and tmp; returns the
        tensor that holds the final state."""
        self._validate(x, tmp)
        idx = ctypes.c_int32(0)
        _check(self._lib.stencil_run_steps(self._h, x.data_ptr(), tmp.data_ptr(), int(steps),
                                           _stream_ptr(stream), ctypes.byref(idx)), "stencil_run_steps")
        return x if idx.value == 0 else tmp

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.stencil_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_steps_noalloc(x, tmp, steps: int, radius: int, shape: int, coeffs, boundary=BC_ZERO, path=PATH_AUTO,
                      lines=LINES_AUTO, block_n=0, chunk=0, time_block=0, stream=None):
    """``steps`` Jacobi steps of the stencil described by the arguments on the
    grid in ``x`` (ping-ponging with ``tmp``) through
    ``stencil_run_steps_noalloc``: no plan object, no device allocation.
    Returns the tensor that holds the final state."""
    torch = _torch()
    for t in (x, tmp):
        if not (t.is_cuda and t.is_contiguous()) or t.dtype not in (torch.float32, torch.float64):
            raise ValueError("grids must be contiguous float32/float64 GPU tensors")
    if x.shape != tmp.shape or x.dtype != tmp.dtype:
        raise ValueError("x and tmp must have the same shape and dtype")
    dtype = F64 if x.dtype == torch.float64 else F32
    d, keep = make_desc(tuple(x.shape), radius, shape, coeffs, boundary=boundary, dtype=dtype, path=path,
                        lines=lines, block_n=block_n, chunk=chunk, time_block=time_block)
    idx = ctypes.c_int32(0)
    _check(load_library().stencil_run_steps_noalloc(ctypes.byref(d), x.data_ptr(), tmp.data_ptr(), int(steps),
                                                     _stream_ptr(stream), ctypes.byref(idx)),
           "stencil_run_steps_noalloc")
    return x if idx.value == 0 else tmp


def autotune(dims, radius, shape, coeffs, boundary=BC_ZERO, dtype=F32, path=PATH_AUTO, lines=LINES_AUTO,
             block_n=0, chunk=0, cache: Optional[str] = None, allow_split=False, force=False, stream=None,
             capacity=64):
    """Measure candidate plans on the current device (``stencil_autotune``).

    stream=None measures on the device's null stream.  Returns (knobs,
    ms_per_step, results): knobs is a dict of path, lines,
    block_n, chunk and time_block for ``Plan(..., **knobs)``; results lists every measured
    candidate (empty on a cache hit)."""
    lib = load_library()
    d, keep = make_desc(dims, radius, shape, coeffs, boundary=boundary, dtype=dtype, path=path, lines=lines,
                        block_n=block_n, chunk=chunk)
    best = Desc()
    ms = ctypes.c_double(0.0)
    res = (TuneResult * capacity)()
    cnt = ctypes.c_int32(0)
    flags = (TUNE_ALLOW_SPLIT if allow_split else 0) | (TUNE_FORCE if force else 0)
    _check(lib.stencil_autotune(ctypes.byref(d), cache.encode() if cache else None, flags, ctypes.byref(best),
                                ctypes.byref(ms), _stream_ptr(stream) if stream is not None else None, res,
                                capacity, ctypes.byref(cnt)),
           "stencil_autotune")
    knobs = {"path": best.path, "lines": best.lines, "block_n": best.block_n, "chunk": best.chunk,
             "time_block": best.time_block, "reg_rows": best.reg_rows, "tile_width": best.tile_width}
    rows = [{"path": r.path, "lines": r.lines, "block_n": r.block_n, "chunk": r.chunk, "time_block": r.time_block,
             "reg_rows": r.reg_rows, "tile_width": r.tile_width, "ms_per_step": r.ms_per_step, "status": r.status}
            for r in res[:min(cnt.value, capacity)]]
    return knobs, ms.value, rows


class Batch:
    """Grids of uneven sizes advanced together (``stencil_batch_*``).

    ``Batch(plans, bufs0, bufs1)``: plans[i] advances the grid held in the
    torch tensors bufs0[i] / bufs1[i].  The plans and tensors must stay alive
    while the batch is used."""

    def __init__(self, plans, bufs0, bufs1):
        lib = load_library()
        n = len(plans)
        if n != len(bufs0) or n != len(bufs1):
            raise ValueError("plans, bufs0 and bufs1 must have the same length")
        for p, x, y in zip(plans, bufs0, bufs1):
            p._validate(x, y)
        vp = ctypes.c_void_p
        hs = (vp * n)(*[p.handle for p in plans])
        b0 = (vp * n)(*[x.data_ptr() for x in bufs0])
        b1 = (vp * n)(*[y.data_ptr() for y in bufs1])
        h = vp()
        _check(lib.stencil_batch_create(hs, b0, b1, n, ctypes.byref(h)), "stencil_batch_create")
        self._h = h
        self._lib = lib
        self._keep = (list(plans), list(bufs0), list(bufs1))

    def run_steps(self, steps: int, stream=None) -> int:
        """Enqueue ``steps`` steps of every grid; returns the index (0/1) of
        the buffer set holding the final states."""
        idx = ctypes.c_int32(0)
        _check(self._lib.stencil_batch_run_steps(self._h, int(steps), _stream_ptr(stream), ctypes.byref(idx)),
               "stencil_batch_run_steps")
        return idx.value

    def info(self) -> dict:
        g, it, bl = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(self._lib.stencil_batch_info(self._h, ctypes.byref(g), ctypes.byref(it), ctypes.byref(bl)),
               "stencil_batch_info")
        return {"groups": g.value, "items": it.value, "blocks": bl.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.stencil_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop with continuous batching (``stencil_server_*``).

    ``Server(arena_bytes, max_active=0, max_inflight_ticks=0)``; requests are
    submitted with their input and output tensors (kept alive here until the
    request is polled), advanced by ``tick()`` and reported by ``poll()``."""

    def __init__(self, arena_bytes: int, max_active: int = 0, max_inflight_ticks: int = 0):
        lib = load_library()
        cfg = ServerConfig(int(arena_bytes), int(max_active), int(max_inflight_ticks))
        h = ctypes.c_void_p()
        _check(lib.stencil_server_create(ctypes.byref(cfg), ctypes.byref(h)), "stencil_server_create")
        self._h = h
        self._lib = lib
        self._live = {}
        self._cancelled = []  # tensors of cancelled requests, kept until close()
        sp = ctypes.c_void_p()
        _check(lib.stencil_server_stream(h, ctypes.byref(sp)), "stencil_server_stream")
        self.stream_handle = sp.value

    def stream(self):
        """The server's stream as a torch stream object."""
        return _torch().cuda.ExternalStream(self.stream_handle)

    def submit(self, x, out, steps: int, radius: int, shape: int, coeffs, boundary=BC_ZERO, path=PATH_AUTO,
               lines=LINES_AUTO, block_n=0, chunk=0) -> int:
        torch = _torch()
        if not (x.is_cuda and out.is_cuda and x.is_contiguous() and out.is_contiguous()):
            raise ValueError("input and output must be contiguous GPU tensors")
        if x.shape != out.shape or x.dtype != out.dtype or x.dtype not in (torch.float32, torch.float64):
            raise ValueError("input and output must have the same shape and a float32/float64 dtype")
        dtype = F64 if x.dtype == torch.float64 else F32
        d, keep = make_desc(tuple(x.shape), radius, shape, coeffs, boundary=boundary, dtype=dtype, path=path,
                            lines=lines, block_n=block_n, chunk=chunk)
        rid = ctypes.c_int64(0)
        _check(self._lib.stencil_server_submit(self._h, ctypes.byref(d), x.data_ptr(), out.data_ptr(), int(steps),
                                               ctypes.byref(rid)), "stencil_server_submit")
        self._live[rid.value] = (x, out)
        return rid.value

    def tick(self) -> dict:
        stats = ServerStats()
        _check(self._lib.stencil_server_tick(self._h, ctypes.byref(stats)), "stencil_server_tick")
        return {name: getattr(stats, name) for name, _ in ServerStats._fields_}

    def cancel(self, rid: int):
        """Withdraw a queued or resident request (``stencil_server_cancel``);
        its tensors are released here once the server's stream has passed
        the work already enqueued for it."""
        _check(self._lib.stencil_server_cancel(self._h, int(rid)), "stencil_server_cancel")
        entry = self._live.pop(rid, None)
        if entry is not None:
            self._cancelled.append(entry)

    def poll(self, capacity: int = 4096):
        ids = (ctypes.c_int64 * capacity)()
        cnt = ctypes.c_int32(0)
        _check(self._lib.stencil_server_poll(self._h, ids, capacity, ctypes.byref(cnt)), "stencil_server_poll")
        done = [ids[k] for k in range(cnt.value)]
        for rid in done:
            self._live.pop(rid, None)
        return done

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.stencil_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._live.clear()
            self._cancelled.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def error_norms(a, ref, stream=None):
    """(sum (a-ref)^2, sum ref^2, max |a-ref|) computed on the GPU; ref float64."""
    torch = _torch()
    out = torch.empty(3, dtype=torch.float64, device=a.device)
    dt = F64 if a.dtype == torch.float64 else F32
    _check(load_library().stencil_error_norms(a.data_ptr(), dt, ref.data_ptr(), a.numel(), out.data_ptr(),
                                              _stream_ptr(stream)), "stencil_error_norms")
    return out
