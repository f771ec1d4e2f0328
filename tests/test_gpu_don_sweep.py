"""Closed-loop narrow passages (the paper's clearance-limited navigation
claim, synthetic scenes of paper_2605_29663_amd.don_sweep): at the tightest
setting of each sweep the controller planning with the exact footprint gets
through, the same controller planning with the footprint's convex hull stops
in front of the passage without contact.  Episodes are deterministic (seeded
noise, bit-identical steps), so one seed per arm pins the outcome."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ds():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29663_amd import don_sweep
    return don_sweep


def _check(ds, case, exact_fp, setting, seed, stop_before):
    from paper_2605_29663_amd.closed_loop import convex_hull
    exact = ds.run_episode(case, exact_fp, setting, seed)
    hull = ds.run_episode(case, convex_hull(exact_fp), setting, seed)
    assert exact["success"] and exact["min_clearance"] >= 0.0, exact
    assert not hull["success"] and hull["min_clearance"] >= 0.0, hull
    assert hull["final_x"] < stop_before, hull


def test_corridor_don_1_exact_passes_hull_stops(ds):
    _check(ds, "corridor", ds.FOOTPRINT_T, 1.0, ds.SWEEP_SEED0 + 1,
           ds.CORRIDOR["gates"][0] + ds.CORRIDOR["post_gap"])


def test_gap_1p9_exact_passes_hull_stops(ds):
    _check(ds, "gap", ds.FOOTPRINT_L, 1.9, ds.SWEEP_SEED0 + 1, ds.GAP["wall_x"])
