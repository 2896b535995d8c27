"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds no stencil arithmetic: it only draws numbers.

Recipe (all draws in FP64 from numpy's PCG64 ``default_rng(seed)``, then cast
to the run dtype; the oracle consumes the cast values widened to FP64):

* grid values: uniform on [-1, 1);
* coefficients: uniform on [0, 1) on the taps of the shape (box: all
  (2r+1)^d offsets; star: the on-axis offsets), zero elsewhere, divided by
  their FP64 sum so they sum to 1 before the cast;
* the 2D five-point diffusion coefficients: centre 1/2, four neighbours 1/8
  (exact in every dtype);
* integer fields and integer coefficients for exactness tests.
"""
from __future__ import annotations

import numpy as np

STAR = 0
BOX = 1


def tap_mask(ndim: int, radius: int, shape: int) -> np.ndarray:
    """Boolean (2r+1)^d mask of the taps a shape uses."""
    w = 2 * radius + 1
    grids = np.meshgrid(*([np.arange(w) - radius] * ndim), indexing="ij")
    if shape == BOX:
        return np.ones((w,) * ndim, dtype=bool)
    nonzero = sum((g != 0).astype(int) for g in grids)
    return nonzero <= 1


def grid(dims, seed: int, dtype=np.float32) -> np.ndarray:
    """Grid values uniform on [-1, 1), drawn in FP64, cast to ``dtype``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=tuple(dims)).astype(dtype)


def coefficients(ndim: int, radius: int, shape: int, seed: int,
                 dtype=np.float32) -> np.ndarray:
    """Normalised positive coefficients on the shape's taps, cast to dtype."""
    rng = np.random.default_rng(seed)
    w = 2 * radius + 1
    mask = tap_mask(ndim, radius, shape)
    c = rng.uniform(0.0, 1.0, size=(w,) * ndim)
    c = np.where(mask, c, 0.0)
    c = c / c.sum()
    return c.astype(dtype)


def diffusion_5pt(dtype=np.float64) -> np.ndarray:
    """2D five-point coefficients: centre 1/2, four neighbours 1/8."""
    c = np.zeros((3, 3), dtype=np.float64)
    c[1, 1] = 0.5
    c[0, 1] = c[2, 1] = c[1, 0] = c[1, 2] = 0.125
    return c.astype(dtype)


def int_grid(dims, seed: int, lo: int = -8, hi: int = 8, dtype=np.float32) -> np.ndarray:
    """Integer-valued grid, uniform on {lo..hi}."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=tuple(dims)).astype(dtype)


def int_coefficients(ndim: int, radius: int, shape: int, seed: int,
                     lo: int = -2, hi: int = 2, dtype=np.float32) -> np.ndarray:
    """Integer coefficients on the shape's taps, uniform on {lo..hi}."""
    rng = np.random.default_rng(seed)
    w = 2 * radius + 1
    mask = tap_mask(ndim, radius, shape)
    c = rng.integers(lo, hi + 1, size=(w,) * ndim).astype(np.float64)
    return np.where(mask, c, 0.0).astype(dtype)


def shift_coefficients(ndim: int, radius: int, offset) -> np.ndarray:
    """A single 1 at gather offset ``offset`` (a pure-shift stencil)."""
    w = 2 * radius + 1
    c = np.zeros((w,) * ndim, dtype=np.float64)
    c[tuple(int(o) + radius for o in offset)] = 1.0
    return c
