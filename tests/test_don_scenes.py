"""The narrow-passage scenes of the DoN sweeps (CPU only): where the explicit
footprint and its convex hull can pass, decided without the controller by a
search of the configuration space.  A configuration (x, y, theta) on a grid
is free when the oracle's signed distance of the footprint there, against
the scene's obstacle points, is at least the clearance the controller keeps;
the passage is feasible when free cells connect the start side to the goal
side (6-neighbour search, theta periodic).  Expected (the claim the sweeps
measure): both footprints pass at the looser settings, only the exact one at
the tightest."""
import math
from collections import deque

import numpy as np
import pytest

from paper_2605_29663_amd import don_sweep as ds
from paper_2605_29663_amd.closed_loop import convex_hull


def _free(orc, V, ox, oy, xs, ys, ths, clearance):
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    out = np.zeros((len(xs), len(ys), len(ths)), bool)
    for k, th in enumerate(ths):
        P = np.stack([X.ravel(), Y.ravel(), np.full(X.size, math.cos(th)),
                      np.full(X.size, math.sin(th))], 1).astype(np.float32)
        out[:, :, k] = (orc.dmin(P, None, ox, oy, kind=0, geom=V) >= clearance).reshape(X.shape)
    return out


def _connected(free):
    nx, ny, nt = free.shape
    seen = np.zeros_like(free)
    q = deque()
    for j, k in zip(*np.nonzero(free[0])):
        seen[0, j, k] = True
        q.append((0, j, k))
    while q:
        i, j, k = q.popleft()
        if i == nx - 1:
            return True
        for a, b, c in ((i + 1, j, k), (i - 1, j, k), (i, j + 1, k), (i, j - 1, k),
                        (i, j, (k + 1) % nt), (i, j, (k - 1) % nt)):
            if 0 <= a < nx and 0 <= b < ny and free[a, b, c] and not seen[a, b, c]:
                seen[a, b, c] = True
                q.append((a, b, c))
    return False


@pytest.mark.parametrize("don,exact_ok,hull_ok", [(0.9, True, True), (1.0, True, False)])
def test_corridor_gate_feasibility(orc, don, exact_ok, hull_ok):
    ox, oy = ds.corridor_scene(don, seed=1)
    xg = ds.CORRIDOR["gates"][0]
    xs = np.arange(xg - 1.4, xg + 1.9, 0.02)
    ys = np.arange(-1.2, 1.2001, 0.02)
    ths = np.radians(np.arange(0, 360, 5))
    clr = ds.corridor_params()["d_safe"]
    assert _connected(_free(orc, ds.FOOTPRINT_T, ox, oy, xs, ys, ths, clr)) == exact_ok
    assert _connected(_free(orc, convex_hull(ds.FOOTPRINT_T), ox, oy, xs, ys, ths, clr)) == hull_ok


@pytest.mark.parametrize("width,exact_ok,hull_ok", [(2.0, True, True), (1.9, True, False)])
def test_gap_feasibility(orc, width, exact_ok, hull_ok):
    ox, oy = ds.gap_scene(width, seed=1)
    xw = ds.GAP["wall_x"]
    xs = np.arange(xw - 2.4, xw + 2.4, 0.04)
    ys = np.arange(-2.4, 2.4001, 0.04)
    ths = np.radians(np.arange(0, 360, 5))
    clr = ds.gap_params()["d_safe"]
    assert _connected(_free(orc, ds.FOOTPRINT_L, ox, oy, xs, ys, ths, clr)) == exact_ok
    assert _connected(_free(orc, convex_hull(ds.FOOTPRINT_L), ox, oy, xs, ys, ths, clr)) == hull_ok


def test_don_definitions():
    # the T's width across its direction of travel, and the L's overall width
    assert np.ptp(ds.FOOTPRINT_T[:, 1]) == pytest.approx(ds.T_WIDTH)
    assert np.ptp(ds.FOOTPRINT_L[:, 1]) == pytest.approx(ds.L_WIDTH)
    # the convex hull of the L: minimum width across directions 2.4 / sqrt(2)
    H = convex_hull(ds.FOOTPRINT_L)
    widths = [np.ptp(H @ np.array([math.cos(a), math.sin(a)])) for a in np.radians(np.arange(0, 180, 0.5))]
    assert min(widths) == pytest.approx(2.4 / math.sqrt(2.0), abs=1e-3)
