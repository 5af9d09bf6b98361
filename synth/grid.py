"""Uniform cell-centred grids on the domain [-1, 1]^3.

A level of resolution ``n`` has points ``x_i = -1 + (2 i + 1) / n`` on each
axis.  The coordinate is computed in float64 and stored once as float32; that
float32 table is the single definition of the grid shared by every consumer.
For ``n`` a power of two every coordinate is an exact dyadic rational.

Points of a level are linearised with x fastest: ``idx = (k * n + j) * n + i``
for the point ``(axis[i], axis[j], axis[k])``.
"""

import numpy as np


def axis_coords(n: int) -> np.ndarray:
    """float32 coordinates of the ``n`` cell centres of one axis."""
    if n <= 0:
        raise ValueError("grid resolution must be positive")
    i = np.arange(n, dtype=np.float64)
    return (-1.0 + (2.0 * i + 1.0) / n).astype(np.float32)


def grid_points(axis: np.ndarray) -> np.ndarray:
    """All ``n^3`` points of a level as an ``(n^3, 3)`` float64 array (x fastest)."""
    a = np.asarray(axis, dtype=np.float64)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
