"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (the contract of the method): signed distances within 1e-5 m
absolute; signs identical except where the oracle's |d| < 1e-6 m; sampled
noise and rollouts bit-identical; augmented costs within 1e-5 relative (FP32
sum of at most 128 terms); weights and updated controls within 1e-5.
"""
import math

import numpy as np
import pytest

from paper_2605_29663_amd import scenes
from rowcheck import SIGN_BAND, TOL_D, assert_sdf_close, check_step_rows as _check_step_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29663_amd as p
    p.load()
    return p


@pytest.fixture(scope="module")
def ctx(pkg):
    c = pkg.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


# ------------------------------------------------------------- point-wise SDF

def _near_boundary_points(V, rng, n):
    E = np.roll(V, -1, axis=0) - V
    b = rng.integers(0, len(V), n)
    t = rng.uniform(0, 1, n)
    nrm = np.stack([E[b, 1], -E[b, 0]], 1) / np.linalg.norm(E[b], axis=1)[:, None]
    off = rng.choice([-1, 1], n) * 10 ** rng.uniform(-7, -1, n)
    return V[b] + t[:, None] * E[b] + off[:, None] * nrm


POLYS = {"L8": scenes.FOOTPRINT_L8, "towed16": scenes.FOOTPRINT_TOWED16,
         "union20": scenes.RECTS_4_BOUNDARY, "gapL": scenes.FOOTPRINT_GAP_L,
         "tri": np.array([(0.0, 0.0), (1.0, 0.1), (0.3, 0.9)]),
         "star32": scenes.star_polygon(np.random.default_rng(32), 32),
         "star5": scenes.star_polygon(np.random.default_rng(5), 5),
         "star64": scenes.star_polygon(np.random.default_rng(64), 64)}


@pytest.mark.parametrize("name", sorted(POLYS))
def test_sdf_polygon_pointwise(ctx, pkg, orc, name):
    V = POLYS[name]
    rng = np.random.default_rng(sum(map(ord, name)))
    far = rng.uniform(-25, 25, size=(100000, 2))      # the paper's 50 x 50 m query box
    near = rng.uniform(-2, 2, size=(50000, 2))
    edge = _near_boundary_points(V, rng, 30000)
    P = np.concatenate([far, near, edge, V]).astype(np.float32)
    ctx.set_footprint(pkg.POLYGON, V)
    d = _np(ctx.sdf_polygon(P[:, 0].copy(), P[:, 1].copy()))
    assert_sdf_close(d, orc.sdf_polygon(V, P[:, 0], P[:, 1]))


@pytest.mark.parametrize("name", ["L8", "towed16", "gapL", "union20", "star32", "star64"])
def test_sdf_ray_through_vertices(ctx, pkg, orc, name):
    """Query points at exactly the height of a vertex, and one float step above
    and below it: the ray-casting corner case, where the half-open rule must
    count a crossing at a vertex once.  Through the point-wise evaluator and
    through the fused distance pass (poses with identity rotation around a
    single point at the origin, so that each pose's offset to the point is
    the query point exactly and the rotated vertices are the vertices)."""
    V = POLYS[name].astype(np.float32)
    y0 = np.unique(V[:, 1])
    ys = np.unique(np.concatenate([y0, np.nextafter(y0, np.float32(np.inf)),
                                   np.nextafter(y0, np.float32(-np.inf))])).astype(np.float32)
    xs = np.linspace(V[:, 0].min() - 1.0, V[:, 0].max() + 1.0, 97).astype(np.float32)
    xs = np.unique(np.concatenate([xs, V[:, 0]])).astype(np.float32)
    X, Y = np.meshgrid(xs, ys)
    P = np.stack([X.ravel(), Y.ravel()], 1).astype(np.float32)
    ref = orc.sdf_polygon(V.astype(np.float64), P[:, 0].astype(np.float64), P[:, 1].astype(np.float64))
    ctx.set_footprint(pkg.POLYGON, V)
    assert_sdf_close(_np(ctx.sdf_polygon(P[:, 0].copy(), P[:, 1].copy())), ref)
    ctx.set_points(np.zeros(1, np.float32), np.zeros(1, np.float32))
    poses = np.zeros((len(P), 1, 4), np.float32)
    poses[:, 0, 0], poses[:, 0, 1], poses[:, 0, 2] = -P[:, 0], -P[:, 1], 1.0
    assert_sdf_close(_np(ctx.sdf_min_poses(poses))[:, 0], ref)


RECTS = {"rects4": scenes.RECTS_4, "gapL": scenes.RECTS_GAP_L, "one": np.array([(0.3, -0.2, 0.5, 0.25)]),
         "L": scenes.SHAPES_LTF["L"][1], "F": scenes.SHAPES_LTF["F"][1],
         "r32": np.concatenate([np.random.default_rng(1).uniform(-1, 1, (32, 2)),
                                np.random.default_rng(2).uniform(0.05, 0.5, (32, 2))], 1)}


@pytest.mark.parametrize("name", sorted(RECTS))
def test_sdf_rectcover_pointwise(ctx, pkg, orc, name):
    R = RECTS[name]
    rng = np.random.default_rng(len(name))
    P = np.concatenate([rng.uniform(-25, 25, (100000, 2)), rng.uniform(-1.5, 1.5, (80000, 2))])
    P = P.astype(np.float32)
    ctx.set_footprint(pkg.RECTS, R)
    d = _np(ctx.sdf_rectcover(P[:, 0].copy(), P[:, 1].copy()))
    assert_sdf_close(d, orc.sdf_rectcover(R, P[:, 0], P[:, 1]))


def test_sdf_pointwise_empty_and_ragged(ctx, pkg, orc):
    ctx.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_L8)
    assert ctx.sdf_polygon(np.zeros(0, np.float32), np.zeros(0, np.float32)).numel() == 0
    for n in (1, 63, 257):
        P = np.random.default_rng(n).uniform(-2, 2, (n, 2)).astype(np.float32)
        d = _np(ctx.sdf_polygon(P[:, 0].copy(), P[:, 1].copy()))
        assert_sdf_close(d, orc.sdf_polygon(scenes.FOOTPRINT_L8, P[:, 0], P[:, 1]))


# ------------------------------------------------------------- fused d_min

def _random_poses(rng, K, T, spread=2.0):
    th = rng.uniform(-math.pi, math.pi, (K, T))
    P = np.stack([rng.uniform(-spread, spread, (K, T)), rng.uniform(-spread, spread, (K, T)),
                  np.cos(th), np.sin(th)], -1)
    return P.astype(np.float32)


FUSED_POLYS = {"towed16": scenes.FOOTPRINT_TOWED16,
               "star7": scenes.star_polygon(np.random.default_rng(7), 7),
               "star13": scenes.star_polygon(np.random.default_rng(13), 13),
               "star27": scenes.star_polygon(np.random.default_rng(27), 27),
               "star33": scenes.star_polygon(np.random.default_rng(33), 33),
               "star50": scenes.star_polygon(np.random.default_rng(50), 50),
               "star64": scenes.star_polygon(np.random.default_rng(64), 64)}


@pytest.mark.parametrize("kind,moving,masked,poly", [(0, False, False, "towed16"),
                                                     (0, True, True, "towed16"),
                                                     (0, True, True, "star27"),
                                                     (0, False, False, "star27"),
                                                     (0, False, True, "star7"),
                                                     (0, True, False, "star13"),
                                                     (0, True, True, "star33"),
                                                     (0, False, True, "star50"),
                                                     (0, False, False, "star64"),
                                                     (0, True, False, "star64"),
                                                     (1, False, True, None), (1, True, False, None),
                                                     (1, True, True, "r32")])
def test_sdf_min_poses(ctx, pkg, orc, kind, moving, masked, poly):
    """Polygons of odd vertex counts run unpadded (one lane per pose); the
    27-vertex polygon is padded to 28 (a lane pair per pose); above 32
    vertices a lane quad shares a pose (33 -> 36, 50 -> 52 padded, 64 exact)."""
    rng = np.random.default_rng(10 * kind + 2 * moving + masked + 100 * len(poly or ""))
    K, T, N, dt = 100, 7, 2500, 0.1            # 700 poses (ragged vs 64), 3 LDS tiles
    poses = _random_poses(rng, K, T)
    ox, oy = rng.uniform(-4, 4, N).astype(np.float32), rng.uniform(-4, 4, N).astype(np.float32)
    vx = vy = None
    if moving:
        vx, vy = rng.uniform(-1, 1, N).astype(np.float32), rng.uniform(-1, 1, N).astype(np.float32)
    valid = (rng.uniform(size=N) < 0.6).astype(np.uint8) if masked else None
    geom = FUSED_POLYS[poly] if kind == 0 else RECTS[poly] if poly else scenes.RECTS_4
    ctx.set_footprint(kind, geom)
    ctx.set_points(ox, oy, vx, vy, valid)
    d, am = ctx.sdf_min_poses(poses, dt=dt, state_offset=1, kind=kind, argmin=True)
    d, am = _np(d), _np(am)
    tau = ((np.arange(T) + 1) * np.float64(np.float32(dt)))[None].repeat(K, 0).ravel()
    d_o, am_o = orc.dmin(poses.reshape(-1, 4), tau, ox, oy, vx, vy, valid, kind, geom,
                         want_argmin=True)
    assert_sdf_close(d.ravel(), d_o)
    # the oracle's distance at the GPU's argmin point equals the oracle minimum
    am = am.ravel()
    assert np.all((am >= 0) == (am_o >= 0))
    if valid is not None:
        assert np.all(valid[am[am >= 0]] == 1)
    sel = np.flatnonzero(am >= 0)
    for k in sel[:: max(1, len(sel) // 300)]:
        i = am[k]
        d_at = orc.dmin(poses.reshape(-1, 4)[k:k + 1], tau[k:k + 1], ox[i:i + 1], oy[i:i + 1],
                        None if vx is None else vx[i:i + 1], None if vy is None else vy[i:i + 1],
                        None, kind, geom)[0]
        assert abs(d_at - d_o[k]) <= TOL_D


def test_sdf_min_poses_empty_and_all_masked(ctx, pkg):
    ctx.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_L8)
    poses = _random_poses(np.random.default_rng(0), 3, 5)
    ctx.set_points(np.zeros(0, np.float32), np.zeros(0, np.float32))
    d, am = ctx.sdf_min_poses(poses, argmin=True)
    assert np.all(np.isposinf(_np(d))) and np.all(_np(am) == -1)
    x = np.float32([0.1, 0.2, np.nan, 5.0])
    ctx.set_points(x, x, valid=np.uint8([0, 0, 1, 0]))      # the only "valid" one is NaN
    d, am = ctx.sdf_min_poses(poses, argmin=True)
    assert np.all(np.isposinf(_np(d))) and np.all(_np(am) == -1)


@pytest.mark.parametrize("poly", ["star32", "star64"])
def test_sdf_min_poses_large_n_ragged(ctx, pkg, orc, poly):
    """Many chunks and LDS tiles: N = 30001 points, 130 poses, polygon B = 32
    (lane pairs) and B = 64 (lane quads)."""
    rng = np.random.default_rng(7)
    V = POLYS[poly]
    poses = _random_poses(rng, 13, 10, spread=5.0)
    N = 30001
    ox, oy = rng.uniform(-8, 8, N).astype(np.float32), rng.uniform(-8, 8, N).astype(np.float32)
    ctx.set_footprint(pkg.POLYGON, V)
    ctx.set_points(ox, oy)
    d = _np(ctx.sdf_min_poses(poses, dt=0.05, kind=pkg.POLYGON)).ravel()
    assert_sdf_close(d, orc.dmin(poses.reshape(-1, 4), None, ox, oy, kind=0, geom=V))


# ------------------------------------------------------------- rollouts

MODEL_CASES = [("c1", {}), ("c2", {}), ("c3", {}),
               ("c1", dict(model="spin", nu=1, sigma=(0.7,), u_min=(-1.0,), u_max=(1.0,))),
               ("c1", dict(model="parallel", nu=1, sigma=(0.5,), u_min=(-0.6,), u_max=(0.6,))),
               ("c2", dict(state_offset=0))]


@pytest.mark.parametrize("T", [33, 24, 7])
@pytest.mark.parametrize("cfg,over", MODEL_CASES)
def test_rollout_bit_exact(ctx, pkg, orc, cfg, over, T):
    """Every motion model, bit for bit.  T = 33: chunks of 16 steps (two
    straight-line chunks and a one-step tail); T = 24: the whole horizon in
    one 32-step chunk; T = 7: one partial chunk."""
    prm = scenes.params(cfg, K=300, T=T, **over)
    rng = np.random.default_rng(3)
    lo, hi = np.float32(prm["u_min"]), np.float32(prm["u_max"])
    U = (rng.uniform(size=(prm["T"], prm["nu"])) * (hi - lo) * 0.8 + lo * 0.8).astype(np.float32)
    q0 = np.float32([0.3, -1.2, 2.9])
    poses, eps, us = ctx.mppi_rollout(prm, q0, U, seed=0xC0FFEE, step=17)
    p_o, e_o, u_o = orc.rollout_f32(prm, q0, U, 0xC0FFEE, 17)
    np.testing.assert_array_equal(_np(eps), e_o)
    np.testing.assert_array_equal(_np(us), u_o)
    np.testing.assert_array_equal(_np(poses), p_o)


# ------------------------------------------------------------- full step

def _step_case(name, K=None, N=None, T=None):
    prm, sc = scenes.config(name)
    if K:
        prm["K"] = K
    if T:
        prm["T"] = T
    if N:
        keep = slice(0, N)
        sc = {k: (v[keep] if isinstance(v, np.ndarray) and v.ndim == 1 and v.size > 1000 else v)
              for k, v in sc.items()}
    return prm, sc


def _load_scene(ctx, pkg, prm, sc):
    if prm["footprint_kind"] == 0:
        ctx.set_footprint(pkg.POLYGON, sc["polygon"])
    else:
        ctx.set_footprint(pkg.RECTS, sc["rects"])
    ctx.set_points(sc["ox"], sc["oy"], sc.get("ovx"), sc.get("ovy"), sc.get("valid"))


@pytest.mark.parametrize("name,K,N,T,offset", [("c1", None, None, None, 1),
                                               ("c2", 192, 1500, None, 1),
                                               ("c2", 192, 1500, 10, 1),
                                               ("c3", 128, 2100, 24, 1),
                                               ("c2", 192, 1500, None, 0),
                                               ("c3", 128, 2100, 24, 0)])
def test_step_parity_small(ctx, pkg, orc, name, K, N, T, offset):
    """Every row of one step against the oracle.  offset = 0 is the literal
    reading of the paper's cost (the (r, h) term scores the pre-step state
    q_h, moving points at time h dt), with static (c2) and moving (c3)
    points; offset = 1 scores q_{h+1}.  c2 with T = 10 and c3 validate in
    one workgroup over two point tiles (T N B <= 2^18, N > 1024), c1 over
    one."""
    import torch
    prm, sc = _step_case(name, K, N, T)
    prm["state_offset"] = offset
    _load_scene(ctx, pkg, prm, sc)
    rng = np.random.default_rng(11)
    U0 = (0.3 * rng.standard_normal((prm["T"], prm["nu"]))).astype(np.float32)
    U0 = np.clip(U0, np.float32(prm["u_min"]), np.float32(prm["u_max"]))
    q0 = np.float32([0.05, -0.02, 0.03])
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=0x5EED, step=3, diag=True)
    _check_step_rows(orc, prm, sc, q0, U0, 0x5EED, 3, u_star, valid, D, Ut)


def test_step_padding_rollouts_ignore_stale_workspace(ctx, pkg, orc, monkeypatch):
    """K = 100 leaves rollouts [100, 128) as padding of the 64-wide layout.
    Their weight is exp(-inf) = 0, so the update must not read whatever
    their perturbation slots held: with every new workspace filled with NaN
    bytes (EXACT_MPPI_POISON) the step still matches the oracle row by row,
    for the single-scene step and for a batch of two scenes."""
    import torch
    monkeypatch.setenv("EXACT_MPPI_POISON", "1")
    prm, sc = _step_case("c2", 100, 1500, 20)
    c = pkg.Context(0)
    try:
        _load_scene(c, pkg, prm, sc)
        rng = np.random.default_rng(100)
        U0 = np.clip((0.3 * rng.standard_normal((prm["T"], prm["nu"]))).astype(np.float32),
                     np.float32(prm["u_min"]), np.float32(prm["u_max"]))
        q0 = np.float32([0.02, -0.01, 0.01])
        Ut = torch.tensor(U0, device="cuda")
        u_star, valid, D = c.mppi_step(prm, q0, Ut, seed=0x100, step=4, diag=True)
        assert np.all(np.isfinite(_np(D["U_upd"])))
        _check_step_rows(orc, prm, sc, q0, U0, 0x100, 4, u_star, valid, D, Ut)
        prm2 = dict(prm, K=37, T=9)
        b = pkg.Batch([c, c], [prm, prm2])
        try:
            U = b.new_nominals()
            b.nominal(U, 0).copy_(torch.tensor(U0, device="cuda"))
            u_b, v_b = b.mppi_step_batched(np.tile(q0, (2, 1)), U, [0x100, 0x100], [4, 4],
                                           use_graph=False)
            np.testing.assert_array_equal(u_b[0, :2], u_star)
            np.testing.assert_array_equal(_np(b.nominal(U, 0)), _np(Ut))
            for s in range(2):
                assert np.all(np.isfinite(_np(b.scene_diag(s)["U_upd"])))
        finally:
            b.close()
    finally:
        c.close()


def test_step_non_finite_nominal_holds(ctx, pkg, orc):
    """A NaN in the nominal makes the updated nominal NaN there; its rollout
    has NaN poses whose distances never lower the minimum (d_nom = +inf), so
    only the finiteness rule stops it: hold (u* = 0) and reset, as in the
    oracle, every row checked from the GPU's intermediates."""
    import torch
    prm, sc = _step_case("c2", 128, 1200, 16)
    _load_scene(ctx, pkg, prm, sc)
    U0 = np.zeros((prm["T"], prm["nu"]), np.float32)
    U0[5, 0] = np.nan
    q0 = np.zeros(3, np.float32)
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=0xBAD, step=0, diag=True)
    assert not valid and np.all(u_star == 0) and torch.all(Ut == 0)
    assert np.isnan(_np(D["U_upd"])[5, 0]) and np.all(np.isposinf(_np(D["d_nom"])[5:]))
    _check_step_rows(orc, prm, sc, q0, U0, 0xBAD, 0, u_star, valid, D, Ut)


def test_step_parity_max_horizon(ctx, pkg, orc):
    """The longest horizon (T = 128): the rollout kernel's 8 chunks of 16
    steps, the update over 128 steps and the 128-pose validation pass, every
    row against the oracle."""
    import torch
    prm, sc = _step_case("c2", 128, 1200, 128)
    _load_scene(ctx, pkg, prm, sc)
    rng = np.random.default_rng(128)
    U0 = (0.2 * rng.standard_normal((prm["T"], prm["nu"]))).astype(np.float32)
    U0 = np.clip(U0, np.float32(prm["u_min"]), np.float32(prm["u_max"]))
    q0 = np.float32([0.0, 0.01, 0.0])
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=0x7128, step=2, diag=True)
    _check_step_rows(orc, prm, sc, q0, U0, 0x7128, 2, u_star, valid, D, Ut)


def test_step_parity_max_rollouts(ctx, pkg, orc):
    """The largest K (2^20 rollouts) with a short horizon: noise, rollouts,
    costs, weights, update and validation of every rollout against the
    oracle, d_min on 4096 sampled poses."""
    import torch
    prm, sc = _step_case("c1", 1 << 20, None, 4)
    _load_scene(ctx, pkg, prm, sc)
    K, T = prm["K"], prm["T"]
    sample = np.sort(np.random.default_rng(20).choice(K * T, 4096, replace=False))
    U0 = np.tile(np.float32([0.4, 0.1]), (T, 1))
    q0 = np.zeros(3, np.float32)
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=0x20, step=1, diag=True)
    _check_step_rows(orc, prm, sc, q0, U0, 0x20, 1, u_star, valid, D, Ut, sample=sample)


@pytest.mark.parametrize("B", [37, 64])
def test_step_parity_large_polygon(ctx, pkg, orc, B):
    """Whole step with a footprint of 37 (padded to 40) and 64 vertices: the
    distance stage runs a lane quad per pose, the validation pass too."""
    import torch
    prm, sc = _step_case("c2", 160, 1300, 18)
    sc = dict(sc, polygon=scenes.star_polygon(np.random.default_rng(B), B, 0.15, 0.4))
    _load_scene(ctx, pkg, prm, sc)
    rng = np.random.default_rng(B + 1)
    U0 = (0.3 * rng.standard_normal((prm["T"], prm["nu"]))).astype(np.float32)
    U0 = np.clip(U0, np.float32(prm["u_min"]), np.float32(prm["u_max"]))
    q0 = np.float32([0.02, 0.01, -0.03])
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=0xB16, step=5, diag=True)
    _check_step_rows(orc, prm, sc, q0, U0, 0xB16, 5, u_star, valid, D, Ut)


@pytest.mark.parametrize("name,path", [("c2", [(0.0, 0.0), (2.0, 0.3), (2.0, 0.3), (4.0, -1.0)]),
                                       ("c1", [(1.0, 0.5)])])
def test_step_parity_with_guidance(ctx, pkg, orc, name, path):
    """Path-following task term: the GPU's J~ and J_nom against the oracle's
    costs with the same polyline (repeated waypoint and single waypoint)."""
    import torch
    prm, sc = _step_case(name, 128 if name == "c2" else None, 1200 if name == "c2" else None)
    prm = dict(prm, w_path=1.5, path=path)
    _load_scene(ctx, pkg, prm, sc)
    ctx.set_guidance(path)
    try:
        U0 = np.zeros((prm["T"], prm["nu"]), np.float32)
        q0 = np.float32([0.1, 0.05, -0.02])
        Ut = torch.tensor(U0, device="cuda")
        u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=5, step=1, diag=True)
        Jt = _check_step_rows(orc, prm, sc, q0, U0, 5, 1, u_star, valid, D, Ut)
        # the term is really there: without the path the costs differ
        J_plain = orc.costs(dict(prm, path=None), _np(D["poses"])[..., :2], _np(D["u"]),
                            _np(D["d_min"]).astype(np.float64))[2]
        assert np.all(Jt > J_plain)
    finally:
        ctx.set_guidance(None)


def test_guidance_errors(ctx, pkg):
    with pytest.raises(pkg.MppiError):
        ctx.set_guidance(np.zeros((65, 2), np.float32))
    with pytest.raises(pkg.MppiError):
        ctx.set_guidance([(0.0, 0.0), (np.nan, 1.0)])
    ctx.set_guidance(None)


def test_step_matches_oracle_from_scratch_c1(ctx, pkg, orc):
    """End to end on the small unicycle case: the oracle runs the whole cycle
    itself (double-precision SDF, costs, update, validation)."""
    import torch
    prm, sc = scenes.config("c1")
    _load_scene(ctx, pkg, prm, sc)
    U0 = np.zeros((prm["T"], 2), np.float32)
    q0 = np.zeros(3, np.float32)
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, seed=1, step=0, diag=True)
    ref = orc.mppi_step(prm, q0, U0, sc, 1, 0)
    assert_sdf_close(_np(D["d_min"]).ravel(), ref["d"].ravel())
    # rollouts whose d_min sits within 1e-5 of 0 or d_safe may legitimately
    # differ in their penalty branch; none do in this scene
    dd = ref["d"]
    edge = np.any((np.abs(dd) < TOL_D) | (np.abs(dd - prm["d_safe"]) < TOL_D), axis=1)
    np.testing.assert_allclose(_np(D["J"])[~edge], ref["Jt"][~edge], rtol=1e-5)
    np.testing.assert_allclose(_np(D["U_upd"]), ref["U_upd"], atol=1e-5)
    assert valid == ref["valid"]
    np.testing.assert_allclose(u_star, ref["u_star"], atol=1e-5)


def test_step_edge_cases(ctx, pkg, orc):
    import torch
    # K = 1, T = 1, triangle footprint, no points: always valid, U += eps
    prm = scenes.params("c1", K=1, T=1)
    ctx.set_footprint(pkg.POLYGON, POLYS["tri"])
    ctx.set_points(np.zeros(0, np.float32), np.zeros(0, np.float32))
    U0 = np.float32([[0.2, 0.1]])
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, np.zeros(3, np.float32), Ut, 9, 9, diag=True)
    assert valid and np.all(np.isposinf(_np(D["d_min"])))
    assert _np(D["w"])[0] == 1.0
    _, e_o, _ = orc.rollout_f32(prm, np.zeros(3, np.float32), U0, 9, 9)
    np.testing.assert_allclose(u_star, U0[0] + e_o[0, 0], atol=1e-6)
    # a wall of points on the path: validation fails -> hold and reset
    prm = scenes.params("c1", K=64, T=10, sigma=(1e-3, 1e-3), validate=1)
    ctx.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_L8)
    ys = np.linspace(-2, 2, 200).astype(np.float32)
    ctx.set_points(np.full(200, 0.8, np.float32), ys)
    Ut = torch.tensor(np.tile(np.float32([1.0, 0.0]), (10, 1)), device="cuda")
    u_star, valid, _ = ctx.mppi_step(prm, np.zeros(3, np.float32), Ut, 1, 0)
    assert not valid and np.all(u_star == 0) and torch.all(Ut == 0)
    # validate = 0: always execute and shift
    prm["validate"] = 0
    Ut = torch.tensor(np.tile(np.float32([1.0, 0.0]), (10, 1)), device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, np.zeros(3, np.float32), Ut, 1, 0, diag=True)
    assert valid
    np.testing.assert_array_equal(u_star, _np(D["U_upd"])[0])


def test_step_errors(ctx, pkg):
    import torch
    prm = scenes.params("c1")
    Ut = torch.zeros((prm["T"], 2), device="cuda")
    c2 = pkg.Context(0)
    with pytest.raises(pkg.MppiError) as e:
        c2.mppi_step(prm, np.zeros(3), Ut, 1, 0)
    assert e.value.code == pkg.MPPI_E_NO_FOOTPRINT
    c2.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_L8)
    for bad in (dict(K=0), dict(K=(1 << 20) + 1), dict(T=129), dict(nu=3), dict(lambda_=0.0)):
        with pytest.raises(pkg.MppiError):
            c2.mppi_step(dict(prm, **bad), np.zeros(3), Ut, 1, 0)
    with pytest.raises(pkg.MppiError) as e:
        c2.set_footprint(pkg.POLYGON, [(0, 0), (1, 1), (1, 0), (0, 1)])
    assert e.value.code == pkg.MPPI_E_FOOTPRINT
    c2.close()


def test_step_deterministic(ctx, pkg):
    import torch
    prm, sc = _step_case("c3", K=256, N=3000, T=20)
    _load_scene(ctx, pkg, prm, sc)
    outs = []
    for _ in range(3):
        Ut = torch.zeros((prm["T"], prm["nu"]), device="cuda")
        u, v, D = ctx.mppi_step(prm, np.zeros(3, np.float32), Ut, 5, 5, diag=True)
        outs.append((u, v, {k: _np(t) for k, t in D.items()}, _np(Ut)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[1] == outs[0][1]
        for k in o[2]:
            assert np.array_equal(o[2][k], outs[0][2][k], equal_nan=True), k
        assert np.array_equal(o[3], outs[0][3])


@pytest.mark.parametrize("poly", [None, "star64"])
def test_step_bitwise_identical_across_tiles(ctx, pkg, poly):
    """Every tile shape (and the autotuner's pick) gives bit-identical outputs,
    with the 16-vertex footprint (one lane per pose) and a 64-vertex one (a
    lane quad per pose)."""
    import torch
    prm, sc = _step_case("c2", K=256, N=2000, T=16)
    if poly:
        sc = dict(sc, polygon=0.4 * POLYS[poly])
    _load_scene(ctx, pkg, prm, sc)
    ref = None
    shapes = [(0, 0), (64, 1), (64, 7), (128, 3), (256, 2), (256, 31)]
    try:
        for blk, nc in shapes:
            ctx.mppi_set_tiles(blk, nc)
            Ut = torch.zeros((prm["T"], prm["nu"]), device="cuda")
            u, v, D = ctx.mppi_step(prm, np.zeros(3, np.float32), Ut, 3, 1, diag=True)
            out = {k: _np(t) for k, t in D.items()}
            out["U"] = _np(Ut)
            if ref is None:
                ref = out
            for k in out:
                assert np.array_equal(out[k], ref[k], equal_nan=True), (blk, nc, k)
        ctx.mppi_set_tiles(0, 0)
        blk, nc = ctx.mppi_autotune(prm, reps=1)
        assert blk in (64, 128, 256) and nc >= 1
        Ut = torch.zeros((prm["T"], prm["nu"]), device="cuda")
        u, v, D = ctx.mppi_step(prm, np.zeros(3, np.float32), Ut, 3, 1, diag=True)
        assert np.array_equal(_np(D["d_min"]), ref["d_min"])
        assert np.array_equal(_np(Ut), ref["U"])
    finally:
        ctx.mppi_set_tiles(0, 0)


# ------------------------------------------------------------- full sizes

@pytest.mark.parametrize("name", ["c2", "c3"])
def test_step_full_size_sampled(ctx, pkg, orc, name):
    """Full-size configuration in the benchmark's launch shape; d_min checked on
    a random 2 % of the (rollout, step) poses (1638 of 81920 at c2, 4096 of
    204800 at c3), everything else in full."""
    import torch
    prm, sc = scenes.config(name)
    _load_scene(ctx, pkg, prm, sc)
    U0 = np.zeros((prm["T"], prm["nu"]), np.float32)
    q0 = np.zeros(3, np.float32)
    Ut = torch.tensor(U0, device="cuda")
    u_star, valid, D = ctx.mppi_step(prm, q0, Ut, 0x5EED0002, 0, diag=True)
    n_poses = prm["K"] * prm["T"]
    sample = np.random.default_rng(0).choice(n_poses, n_poses // 50, replace=False)
    _check_step_rows(orc, prm, sc, q0, U0, 0x5EED0002, 0, u_star, valid, D, Ut, sample=sample)


def test_sequence_costs(ctx, pkg, orc):
    """Noise-free costs of given control sequences (some outside the control
    box): equal to the J~ of a zero-noise one-rollout step bit for bit, and to
    the oracle's own rollout, distances and costs."""
    import torch
    prm, sc = scenes.config("c2", K=1, T=24)
    sc = dict(sc, ox=sc["ox"][:2000], oy=sc["oy"][:2000])
    _load_scene(ctx, pkg, prm, sc)
    rng = np.random.default_rng(77)
    n, T = 5, prm["T"]
    lo, hi = np.float32(prm["u_min"][:2]), np.float32(prm["u_max"][:2])
    Useq = rng.uniform(1.3 * lo, 1.3 * hi, (n, T, 2)).astype(np.float32)
    q0 = np.float32([0.1, -0.05, 0.02])
    J = _np(ctx.mppi_sequence_costs(prm, q0, torch.tensor(Useq, device="cuda")))
    p0 = dict(prm, K=1, sigma=(0.0, 0.0), validate=0)
    for r in range(n):
        U = torch.tensor(Useq[r], device="cuda")
        _, _, D = ctx.mppi_step(p0, q0, U, 0, 0, diag=("J",))
        assert J[r] == _np(D["J"])[0]
        poses, _, u = orc.rollout_f32(p0, q0, Useq[r], 0, 0)
        d = orc.dmin(poses.reshape(-1, 4), orc.tau_of(p0, T), sc["ox"], sc["oy"], kind=0,
                     geom=sc["polygon"]).reshape(1, T)
        _, _, Jt = orc.costs(p0, poses[..., :2], u, d)
        assert not np.any((np.abs(d) < TOL_D) | (np.abs(d - p0["d_safe"]) < TOL_D))
        np.testing.assert_allclose(J[r], Jt[0], rtol=1e-5)
    with pytest.raises(ValueError):
        ctx.mppi_sequence_costs(prm, q0, torch.zeros((0, T, 2), device="cuda"))
