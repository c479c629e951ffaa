"""Grid diffusion oracle (fp64 numpy) -- TEST INFRASTRUCTURE ONLY: the
tests, the smoke check and the benchmark's CPU-baseline leg use it; the GPU
library never imports it.

One step of the diffusion of Section II-C (virus and inflammatory signal
spread from each grid point to its neighbours): every point keeps (1 - D)
of its value and receives D/8 of each of its 8 neighbours'; points outside
the grid contribute 0, which is what the zero border of Section VI-D's
padded grid gives.
"""
from __future__ import annotations

import numpy as np


def diffuse(c: np.ndarray, D: float, steps: int = 1) -> np.ndarray:
    """`steps` diffusion steps of the 2-D grid c (rows = y, columns = x)."""
    c = np.asarray(c, dtype=np.float64)
    for _ in range(steps):
        p = np.pad(c, 1)
        ny, nx = c.shape
        nbrs = np.zeros_like(c)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dy or dx:
                    nbrs += p[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        c = (1.0 - D) * c + (D / 8.0) * nbrs
    return c


def diffuse_loops(c: np.ndarray, D: float) -> np.ndarray:
    """One step written point by point with explicit bounds checks (small
    grids only)."""
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    out = np.empty_like(c)
    for y in range(ny):
        for x in range(nx):
            s = 0.0
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dy or dx) and 0 <= y + dy < ny and 0 <= x + dx < nx:
                        s += c[y + dy, x + dx]
            out[y, x] = (1.0 - D) * c[y, x] + D / 8.0 * s
    return out
