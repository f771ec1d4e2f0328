"""sdf_min_poses_noalloc (the entry point for callers that cannot allocate
device memory) against sdf_min_poses, through the C ABI: two calls in a row,
the second on a smaller input, with and without the argmin, polygon and
rectangle cover, static and moving points; the capacity limit; no device
memory taken by the call."""
import numpy as np
import pytest

from paper_2605_29663_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29663_amd as p
    p.load()
    return p


def _poses(rng, K, T, spread=3.0):
    th = rng.uniform(-np.pi, np.pi, (K, T))
    return np.stack([rng.uniform(-spread, spread, (K, T)), rng.uniform(-spread, spread, (K, T)),
                     np.cos(th), np.sin(th)], -1).astype(np.float32)


def _both(pkg, ctx, poses_np, kind, state_offset, dt, argmin):
    import torch
    poses = torch.tensor(poses_np, device="cuda")
    ref = ctx.sdf_min_poses(poses, dt=dt, state_offset=state_offset, kind=kind, argmin=argmin)
    K, T = poses_np.shape[:2]
    d = torch.full((K, T), float("nan"), device="cuda")
    am = torch.full((K, T), -7, dtype=torch.int32, device="cuda") if argmin else None
    ctx.sdf_min_poses_noalloc(poses, d, am, dt=dt, state_offset=state_offset, kind=kind)
    torch.cuda.synchronize()
    if argmin:
        d_ref, am_ref = ref
        assert np.array_equal(am.cpu().numpy(), am_ref.cpu().numpy())
    else:
        d_ref = ref
    assert np.array_equal(d.cpu().numpy(), d_ref.cpu().numpy())
    return d.cpu().numpy()


@pytest.mark.parametrize("kind,moving,argmin", [(0, False, False), (0, True, True),
                                                (1, False, True), (1, True, False)])
def test_noalloc_matches_sdf_min_poses(pkg, kind, moving, argmin):
    rng = np.random.default_rng(10 * kind + 2 * moving + argmin)
    ctx = pkg.Context(0)
    try:
        N = 3001
        ox, oy = rng.uniform(-5, 5, N).astype(np.float32), rng.uniform(-5, 5, N).astype(np.float32)
        vx = vy = None
        if moving:
            vx, vy = rng.uniform(-1, 1, N).astype(np.float32), rng.uniform(-1, 1, N).astype(np.float32)
        valid = (rng.uniform(size=N) < 0.8).astype(np.uint8)
        ctx.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_TOWED16)
        ctx.set_footprint(pkg.RECTS, scenes.RECTS_4)
        ctx.set_points(ox, oy, vx, vy, valid)
        # first call larger than the second: the second must not see the first's keys
        big = _both(pkg, ctx, _poses(rng, 300, 41), kind, 1, 0.05, argmin)
        small = _both(pkg, ctx, _poses(rng, 7, 5), kind, 0, 0.1, argmin)
        assert np.all(np.isfinite(big)) and np.all(np.isfinite(small))
    finally:
        ctx.close()


def test_noalloc_capacity_and_no_allocation(pkg):
    import torch
    ctx = pkg.Context(0)
    try:
        rng = np.random.default_rng(3)
        ctx.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_L8)
        ctx.set_points(rng.uniform(-4, 4, 500).astype(np.float32),
                       rng.uniform(-4, 4, 500).astype(np.float32))
        cap = 1 << 19                                      # MPPI_NOALLOC_MAX_POSES
        K, T = cap // 64, 64                               # exactly the capacity
        poses = torch.tensor(_poses(rng, K, T), device="cuda")
        d = torch.empty((K, T), device="cuda")
        am = torch.empty((K, T), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.sdf_min_poses_noalloc(poses, d, am)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        # the keys of 2^19 poses would take 4 MiB if the call allocated them
        assert free0 - free1 < (1 << 20)
        ref_d, ref_am = ctx.sdf_min_poses(poses, argmin=True)
        assert torch.equal(d, ref_d) and torch.equal(am, ref_am)
        over = torch.tensor(_poses(rng, K + 1, T), device="cuda")
        with pytest.raises(pkg.MppiError) as e:
            ctx.sdf_min_poses_noalloc(over, torch.empty((K + 1, T), device="cuda"))
        assert e.value.code == pkg.MPPI_E_CAPACITY
        # an empty call is a no-op
        ctx.sdf_min_poses_noalloc(torch.empty((0, T, 4), device="cuda"),
                                  torch.empty((0, T), device="cuda"))
    finally:
        ctx.close()
