"""Oracle of the point-cloud pre-processing step (test infrastructure only:
loaded by tests/ alone).

The paper obtains the obstacle set from the local point cloud by keeping the
points inside a task-relevant height band and downsampling them to a fixed
budget N (Section "Problem Statement"); it does not name the downsampling
method.  Reading taken (one representative per occupied voxel, nearest first):

1. a point is kept if all three coordinates are finite, z_min <= z <= z_max
   and its squared planar range to the robot, (x - cx)^2 + (y - cy)^2
   evaluated in single precision, is <= r_max^2;
2. its voxel is (floor(x / v), floor(y / v)) of single-precision quotients;
3. each occupied voxel is represented by its kept point of lowest index;
4. if more than N voxels are occupied, the N representatives of smallest
   (squared range, index) are kept;
5. the kept representatives are written in ascending input order; the
   remaining slots up to N are invalid (mask 0).

Plain numpy; the single-precision steps are the ones the decisions depend on,
taken in the same precision as the device."""
from __future__ import annotations

import numpy as np


def downsample(xyz, center, z_min, z_max, r_max, voxel, n_out):
    """Returns (x[n_out], y[n_out], valid[n_out] uint8, n_kept)."""
    p = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    cx, cy = np.float32(center[0]), np.float32(center[1])
    dx, dy = x - cx, y - cy
    r2 = dx * dx + dy * dy                          # float32, no contraction
    rmax2 = np.float32(r_max) * np.float32(r_max)
    with np.errstate(invalid="ignore"):
        ok = (np.isfinite(p).all(axis=1) & (z >= np.float32(z_min)) & (z <= np.float32(z_max))
              & (r2 <= rmax2))
    v = np.float32(voxel)
    rep = {}
    for i in np.flatnonzero(ok):                    # ascending index: first seen is the lowest
        cell = (int(np.floor(x[i] / v)), int(np.floor(y[i] / v)))
        if cell not in rep:
            rep[cell] = int(i)
    reps = sorted(rep.values())
    if len(reps) > n_out:
        order = sorted(reps, key=lambda i: (float(r2[i]), i))
        reps = sorted(order[:n_out])
    ox = np.zeros(n_out, np.float32)
    oy = np.zeros(n_out, np.float32)
    valid = np.zeros(n_out, np.uint8)
    k = len(reps)
    ox[:k], oy[:k], valid[:k] = x[reps], y[reps], 1
    return ox, oy, valid, k
