"""Closed-loop docking (the paper's footprint claim, Experiment 2, synthetic):
with the explicit fork-shaped footprint plain MPPI docks around the post
without contact; with the footprint's convex hull the docked pose is in
collision, so the same controller stops short."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29663_amd import closed_loop
    return closed_loop


def test_exact_footprint_docks_hull_does_not(cl):
    exact = cl.run_episode(cl.FOOTPRINT_FORK, 100, steps=150)
    hull = cl.run_episode(cl.convex_hull(cl.FOOTPRINT_FORK), 100, steps=150)
    assert exact["success"] and exact["min_clearance"] > 0.0, exact
    assert not hull["success"] and hull["final_error"] > 0.4, hull
    assert hull["min_clearance"] > 0.0      # stopping short, not colliding
