"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random fields and ROI regions.  It holds none of the
decomposition, quantization or coding arithmetic, so both the library's
tests and the CPU reference can take their inputs from it.

The paper evaluates on public simulation outputs (Sec. V-A, Table I) that
are not available here; these generators stand in for them:

* ``gaussian_random_field``: white noise filtered in Fourier space so the
  per-mode power falls as k^-beta, normalised to mean 0 and std 1.
* ``bumps_and_modes``: 8 Gaussian bumps + 3 sine modes + N(0, 1e-3) noise.
* ``turbulence_with_front``: a k^-5/3 shell-spectrum field (per-mode
  beta = 11/3) plus a sharp tanh front.
* ROI helpers: non-overlapping boxes, gradient-percentile voxel masks.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import scipy.fft as sfft


def _workers() -> int:
    import os
    return max(1, min(16, os.cpu_count() or 1))


def gaussian_random_field(shape: Sequence[int], beta: float, seed: int,
                          dtype=np.float32) -> np.ndarray:
    """Field whose per-mode power is proportional to k^-beta (k in cycles per box)."""
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape, dtype=np.float64)
    spec = sfft.rfftn(white, workers=_workers())
    del white
    kz = sfft.fftfreq(shape[0]) * shape[0]
    ky = sfft.fftfreq(shape[1]) * shape[1]
    kx = sfft.rfftfreq(shape[2]) * shape[2]
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    spec *= k2 ** (-beta / 4.0)
    spec[0, 0, 0] = 0.0
    del k2
    f = sfft.irfftn(spec, s=shape, workers=_workers())
    del spec
    f -= f.mean()
    f /= f.std()
    return f.astype(dtype)


def bumps_and_modes(n: int = 65, seed: int = 1, dtype=np.float32) -> np.ndarray:
    """Sum of 8 Gaussian bumps, 3 sine modes and N(0, 1e-3) noise on [0,1]^3."""
    rng = np.random.default_rng(seed)
    r = np.arange(n) / (n - 1)
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    f = np.zeros((n, n, n))
    for _ in range(8):
        c = rng.uniform(0, 1, 3)
        s = rng.uniform(0.05, 0.2)
        a = rng.uniform(-1, 1)
        f += a * np.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2) / (2 * s * s))
    for _ in range(3):
        k = rng.integers(1, 5, 3)
        ph = rng.uniform(0, 2 * np.pi)
        f += 0.3 * np.sin(2 * np.pi * (k[0] * z + k[1] * y + k[2] * x) + ph)
    f += rng.normal(0.0, 1e-3, f.shape)
    return f.astype(dtype)


def turbulence_with_front(shape: Sequence[int], seed: int = 3, dtype=np.float64) -> np.ndarray:
    """k^-5/3 shell-spectrum field (per-mode beta 11/3) plus 2 tanh(n.(r - r0)/delta)."""
    f = gaussian_random_field(shape, 11.0 / 3.0, seed, np.float64)
    rng = np.random.default_rng(seed + 7919)
    nv = rng.standard_normal(3)
    nv /= np.linalg.norm(nv)
    c = [(s - 1) / 2.0 for s in shape]
    iz = (np.arange(shape[0]) - c[0]) * nv[0]
    iy = (np.arange(shape[1]) - c[1]) * nv[1]
    ix = (np.arange(shape[2]) - c[2]) * nv[2]
    f += 2.0 * np.tanh((iz[:, None, None] + iy[None, :, None] + ix[None, None, :]) / 2.0)
    return f.astype(dtype)


def disjoint_boxes(shape: Sequence[int], edge: int, count: int, seed: int) -> List[Tuple[int, ...]]:
    """``count`` axis-aligned cubes of side ``edge`` at random origins, redrawn until disjoint."""
    rng = np.random.default_rng(seed)
    boxes: List[Tuple[int, ...]] = []
    while len(boxes) < count:
        o = [int(rng.integers(0, s - edge + 1)) for s in shape]
        cand = (o[0], o[1], o[2], o[0] + edge, o[1] + edge, o[2] + edge)
        if all(any(cand[a + 3] <= bx[a] or bx[a + 3] <= cand[a] for a in range(3)) for bx in boxes):
            boxes.append(cand)
    return boxes


def gradient_percentile_mask(field: np.ndarray, pct: float = 95.0) -> np.ndarray:
    """True where |grad field| exceeds its ``pct`` percentile."""
    g = np.gradient(np.asarray(field, np.float64))
    mag = np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    return mag > np.percentile(mag, pct)


def batched_shapes(count: int = 256, seed: int = 4) -> List[Tuple[int, int, int]]:
    """Per-field dims drawn i.i.d. from {33, 65, 129, 257}."""
    rng = np.random.default_rng(seed)
    choice = np.array([33, 65, 129, 257])
    return [tuple(int(v) for v in rng.choice(choice, 3)) for _ in range(count)]


def batched_roi_box(shape: Sequence[int], seed: int) -> Tuple[int, ...]:
    """One box of edge (d-1)/4+1 per axis at a seeded origin."""
    rng = np.random.default_rng(seed)
    e = [(d - 1) // 4 + 1 for d in shape]
    o = [int(rng.integers(0, d - ed + 1)) for d, ed in zip(shape, e)]
    return (o[0], o[1], o[2], o[0] + e[0], o[1] + e[1], o[2] + e[2])


# Workload recipes ---------------------------------------------------------

def workload_small(seed: int = 1):
    """65^3 FP32 bumps + modes, uniform REL 1e-3, pure global hierarchy."""
    return bumps_and_modes(65, seed)


def workload_roi(n: int = 512, seed: int = 2):
    """n^3 FP32 k^-3 field and two disjoint 64^3 ROI boxes (n/8 boxes for small n)."""
    x = gaussian_random_field((n, n, n), 3.0, seed, np.float32)
    edge = 64 if n >= 128 else max(4, n // 8)
    boxes = disjoint_boxes((n, n, n), edge, 2, seed + 101)
    return x, boxes
