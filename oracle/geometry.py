"""Array element coordinates (paper Sec. II-A, antenna scheme).

The ULA sits on the y axis, centred at the origin, with uniform spacing delta
(the paper uses delta = lambda/2).  "Centred" is read as element n at
y_n = (n - (N-1)/2) * delta, n = 0..N-1, which makes eq. (4) the midpoint rule
over [-N*delta/2, N*delta/2].  The UPA (not treated by the paper, which defers
rectangular arrays to future work) is the same construction in the y-z plane:
element (a, b) at (0, (a-(n_y-1)/2) delta, (b-(n_z-1)/2) delta).

Pinned by: mirror invariance and the far-field Dirichlet-kernel limit of the
exact Gram (tests/test_oracle_channel.py).
"""
from __future__ import annotations

import numpy as np

from workloads import GEOM_ULA, GEOM_UPA, ArraySpec


def element_positions(arr: ArraySpec) -> np.ndarray:
    """[N, 3] float64 element coordinates, flat index n = a * n_z + b."""
    ny, nz = int(arr.n_y), int(arr.n_z)
    ya = (np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0) * arr.spacing
    if arr.geometry == GEOM_ULA:
        assert nz == 1
        return np.stack([np.zeros(ny), ya, np.zeros(ny)], axis=-1)
    assert arr.geometry == GEOM_UPA
    zb = (np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0) * arr.spacing
    yy, zz = np.meshgrid(ya, zb, indexing="ij")
    return np.stack([np.zeros(ny * nz), yy.ravel(), zz.ravel()], axis=-1)


def perpendicular_distance(arr: ArraySpec, users: np.ndarray) -> np.ndarray:
    """Distance of each user from the array's line (ULA) or plane (UPA).

    For a ULA the channel is invariant to rotating the user about the array
    axis (Sec. II-A), so a 3-D user at (x, y, z) acts as a 2-D user at
    (sqrt(x^2 + z^2), y).  For a UPA in the x = 0 plane it is |x|.
    """
    users = np.asarray(users, np.float64)
    if arr.geometry == GEOM_ULA:
        return np.hypot(users[:, 0], users[:, 2])
    return np.abs(users[:, 0])
