"""Pins for the point-cloud pre-processing oracle (CPU only): hand-placed
points (band, range, voxel representatives, budget with range ties, order),
and an independent formulation of the same rule (numpy unique on voxel keys
and a lexicographic sort) on random clouds."""
import numpy as np
import pytest

from oracle import cloud


def _run(pts, n_out, center=(0.0, 0.0), z=(-1.0, 1.0), r_max=10.0, voxel=1.0):
    return cloud.downsample(np.asarray(pts, np.float32), center, z[0], z[1], r_max, voxel, n_out)


def test_hand_placed_points():
    pts = [(0.2, 0.2, 0.0),    # 0: voxel (0, 0)
           (0.7, 0.1, 0.0),    # 1: same voxel, higher index -> dropped
           (1.5, 0.5, 5.0),    # 2: above the band
           (1.5, 0.5, 0.0),    # 3: voxel (1, 0)
           (-0.5, 0.5, -1.0),  # 4: on the band's edge (kept), voxel (-1, 0)
           (30.0, 0.0, 0.0),   # 5: beyond r_max
           (np.nan, 1.0, 0.0), # 6: non-finite
           (0.1, 0.9, 0.5)]    # 7: voxel (0, 0) again
    x, y, v, k = _run(pts, 6)
    assert k == 3
    np.testing.assert_array_equal(v, [1, 1, 1, 0, 0, 0])
    np.testing.assert_array_equal(x[:3], np.float32([0.2, 1.5, -0.5]))
    np.testing.assert_array_equal(y[:3], np.float32([0.2, 0.5, 0.5]))
    assert np.all(x[3:] == 0) and np.all(y[3:] == 0)


def test_budget_keeps_nearest_then_lowest_index_in_input_order():
    # distinct voxels; squared ranges 16, 1, 4, 1, 9 (two ties at 1)
    pts = [(4, 0, 0), (0, 1, 0), (2, 0, 0), (-1, 0, 0), (0, -3, 0)]
    x, y, v, k = _run(pts, 2, voxel=0.5)
    assert k == 2 and list(v) == [1, 1]
    np.testing.assert_array_equal(np.c_[x, y], np.float32([[0, 1], [-1, 0]]))
    x, y, v, k = _run(pts, 3, voxel=0.5)
    np.testing.assert_array_equal(np.c_[x, y], np.float32([[0, 1], [2, 0], [-1, 0]]))
    # the tie at range 1 is broken by index: budget 1 keeps point 1
    x, y, v, k = _run(pts, 1, voxel=0.5)
    np.testing.assert_array_equal(np.c_[x, y], np.float32([[0, 1]]))


def test_range_is_taken_from_the_robot_and_inclusive():
    pts = [(3.0, 4.0, 0.0), (3.0, 4.1, 0.0)]
    _, _, v, k = _run(pts, 4, center=(0.0, 0.0), r_max=5.0, voxel=0.05)
    assert k == 1
    _, _, v, k = _run(pts, 4, center=(3.0, 4.0), r_max=0.2, voxel=0.05)
    assert k == 2


def test_empty_and_zero_budget():
    x, y, v, k = _run(np.zeros((0, 3)), 4)
    assert k == 0 and not v.any()
    x, y, v, k = _run([(0.0, 0.0, 0.0)], 0)
    assert k == 0 and x.size == 0


def _independent(p, center, z_min, z_max, r_max, voxel, n_out):
    p = np.asarray(p, np.float32)
    dx, dy = p[:, 0] - np.float32(center[0]), p[:, 1] - np.float32(center[1])
    r2 = dx * dx + dy * dy
    with np.errstate(invalid="ignore"):
        ok = (np.isfinite(p).all(1) & (p[:, 2] >= np.float32(z_min)) & (p[:, 2] <= np.float32(z_max))
              & (r2 <= np.float32(r_max) * np.float32(r_max)))
    idx = np.flatnonzero(ok)
    cells = np.stack([np.floor(p[idx, 0] / np.float32(voxel)),
                      np.floor(p[idx, 1] / np.float32(voxel))], 1).astype(np.int64)
    _, first = np.unique(cells, axis=0, return_index=True)   # first occurrence = lowest index
    reps = idx[first]
    order = np.lexsort((reps, r2[reps]))                      # by range, then index
    return np.sort(reps[order[:n_out]])


@pytest.mark.parametrize("seed", range(5))
def test_matches_independent_formulation(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 3000))
    p = rng.uniform(-6, 6, (m, 3)).astype(np.float32)
    dup = rng.integers(0, m, m // 5)
    p[dup] = p[rng.integers(0, m, dup.size)]          # repeated points
    p[rng.random(m) < 0.01, 0] = np.nan
    center = tuple(rng.uniform(-1, 1, 2))
    n_out = int(rng.integers(0, 600))
    args = (center, -2.0, 2.5, 5.0, float(rng.choice([0.05, 0.2, 0.5])), n_out)
    x, y, v, k = cloud.downsample(p, *args)
    want = _independent(p, *args)
    assert k == want.size
    np.testing.assert_array_equal(x[:k], p[want, 0])
    np.testing.assert_array_equal(y[:k], p[want, 1])
    assert v[:k].all() and not v[k:].any()
