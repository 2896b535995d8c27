"""CPU FP64 oracle for the stencil sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports, calls, links or executes anything here, and
this package imports nothing from the product.

The arithmetic lives in ``stencil_oracle.c`` (plain C, FP64, fixed tap order,
built with ``-ffp-contract=off``): the gather-form stencil of the paper's
Eq. (1) generalised to order r and 2D/3D, repeated as Jacobi steps
(Section 2.2).  This module only builds and marshals.

Parity status of each function (pins live in ``tests/test_oracle_pins.py``):

* ``run`` / ``step`` -- pinned: Eq. (1) printed term list (golden fixture),
  scipy.ndimage.correlate, dense-operator brute force, independent scatter
  form of Eq. (3)-(5), FFT symbol (periodic), sine eigenmodes (zero halo),
  constant fields, exact polynomial reproduction.
* ``window`` -- pinned against ``run`` on grids small enough to run whole.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SHAPE_STAR = 0
SHAPE_BOX = 1
BC_ZERO = 0
BC_PERIODIC = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = [
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-frounding-math",
            _SRC, "-o", tmp,
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_step.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, dp, dp, dp]
        lib.oracle_step.restype = ctypes.c_int
        lib.oracle_run.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, dp, dp, dp, ctypes.c_int64]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> int:
    """Set the OpenMP team size; returns the size in effect."""
    return int(_load().oracle_set_threads(int(n)))


def run(a0: np.ndarray, coeffs: np.ndarray, radius: int, shape: int, bc: int,
        steps: int) -> np.ndarray:
    """Final state after ``steps`` Jacobi steps of the gather stencil.

    ``a0``: 2D or 3D array (any real dtype; widened to FP64).
    ``coeffs``: dense (2r+1)^d gather coefficients C^g (widened to FP64).
    Star shapes use only the on-axis taps of ``coeffs``.
    """
    lib = _load()
    a = np.ascontiguousarray(a0, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    ndim = a.ndim
    w = 2 * radius + 1
    if c.shape != (w,) * ndim:
        raise ValueError(f"coeffs shape {c.shape} != {(w,) * ndim}")
    dims = (ctypes.c_int64 * 3)(*(list(a.shape) + [1] * (3 - ndim)))
    out = np.empty_like(a)
    rc = lib.oracle_run(ndim, dims, radius, shape, bc, _dp(c), _dp(a), _dp(out), int(steps))
    if rc != 0:
        raise RuntimeError(f"oracle_run failed ({rc})")
    return out


def step(a: np.ndarray, coeffs: np.ndarray, radius: int, shape: int, bc: int) -> np.ndarray:
    """One Jacobi step (same contract as ``run`` with steps=1)."""
    return run(a, coeffs, radius, shape, bc, 1)


def window(a0: np.ndarray, coeffs: np.ndarray, radius: int, shape: int, bc: int,
           steps: int, lo: Sequence[int], size: Sequence[int]) -> np.ndarray:
    """Final state on the window [lo, lo+size) of a large grid, computed from
    the input window dilated by r*steps (the light cone of the window).

    Periodic grids take the dilated window with wrapped indices; zero-halo
    grids clip it at the grid faces, where the clipped edge is the true face.
    Either way the sub-problem is solved with a zero halo, which is exact for
    points at distance >= r*steps from every cut that is not a true face.
    """
    a0 = np.asarray(a0)
    ndim = a0.ndim
    halo = radius * steps
    idx = []
    offs = []
    for d in range(ndim):
        n = a0.shape[d]
        if bc == BC_PERIODIC:
            ids = (np.arange(lo[d] - halo, lo[d] + size[d] + halo) % n)
            offs.append(halo)
        else:
            start = max(lo[d] - halo, 0)
            stop = min(lo[d] + size[d] + halo, n)
            ids = np.arange(start, stop)
            offs.append(lo[d] - start)
        idx.append(ids)
    sub = a0[np.ix_(*idx)]
    res = run(sub, coeffs, radius, shape, BC_ZERO, steps)
    sl = tuple(slice(offs[d], offs[d] + size[d]) for d in range(ndim))
    return res[sl]
