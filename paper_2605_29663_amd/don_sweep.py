"""Clearance-limited navigation sweeps: explicit footprint against its convex hull.

Synthetic counterparts of the paper's two narrow-passage studies (Section
"Experiment 2: Clearance-Limited Navigation", Tables "Corridor DoN sweep" and
"Omni-directional gap DoN sweep"), run in closed loop with the library's own
MPPI step and the same controller for both footprints:

* corridor: a differential-drive (unicycle) robot with a T-shaped footprint
  (a 1.0 m wide, 0.3 m deep cross bar in front of a 0.4 m wide, 0.9 m long
  stem) drives along a corridor through two "gates", each a pair of 0.1 m
  thick posts standing out of the opposite walls, 0.6 m apart along the
  corridor.  The lateral opening between the tips of a gate's posts is
  W_p = W_r / DoN with W_r = 1.0 m, the robot's width across its direction of
  travel (the paper's Degree of Narrowness).  Up to DoN 0.9 the cross bar
  passes straight; at DoN 1.0 it must pass the first post on one side and the
  second on the other while the first post is beside the narrow stem, which
  the convex hull cannot do.
* gap: an omni-directional robot with the paper's L-shaped footprint (2.0 x
  2.0 m, 0.4 m legs) crosses a 0.1 m thick wall through a gap of width 1.9,
  2.0, 2.2 or 2.4 m (DoN = 2.0 m / gap).  With the 0.12 m clearance used here
  the convex hull (minimum width 1.70 m) needs a gap of 1.94 m; the exact L
  can thread a narrower gap by rotating while it passes.

Both footprints are feasible at every setting except the hull at the
tightest one, which configuration-space searches over (x, y, theta) confirm
(`tests/test_don_scenes.py`).  Each episode: the robot follows u* with the
same Euler model in double precision; success = the robot's reference point
reaches the goal line within the step budget with the exact footprint never
in contact (the robot is the exact shape in both arms).  Reported per cell:
success rate, mean navigation time and mean speed over the successful
episodes.

    python -m paper_2605_29663_amd.don_sweep --episodes 10 --out result.json

This module generates the scenes (geometry only) and orchestrates episodes;
every signed distance, rollout and update runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

import paper_2605_29663_amd as pkg
from paper_2605_29663_amd import scenes
from paper_2605_29663_amd.closed_loop import convex_hull

# T-shaped footprint (CCW, body frame, origin at the stem's middle).
FOOTPRINT_T = np.array([(-0.6, -0.2), (0.3, -0.2), (0.3, -0.5), (0.6, -0.5), (0.6, 0.5),
                        (0.3, 0.5), (0.3, 0.2), (-0.6, 0.2)], dtype=np.float64)
T_WIDTH = 1.0
# The paper's L (2.0 x 2.0 m, 0.4 m legs), origin at its bounding-box centre.
FOOTPRINT_L = scenes.FOOTPRINT_GAP_L - 1.0
L_WIDTH = 2.0

CORRIDOR_DON = (0.6, 0.7, 0.8, 0.9, 1.0)
GAP_WIDTHS = (2.4, 2.2, 2.0, 1.9)

SPACING = 0.04        # obstacle point spacing along every edge (m)
SWEEP_SEED0 = 500     # episode e of every cell uses seed SWEEP_SEED0 + e
JITTER = 0.005        # per-point position noise (m)


def _segment(a, b, h=SPACING):
    n = max(2, int(math.ceil(math.dist(a, b) / h)) + 1)
    t = np.linspace(0.0, 1.0, n)[:, None]
    return np.asarray(a, float) * (1.0 - t) + np.asarray(b, float) * t


def _box(x0, x1, y0, y1):
    return [_segment((x0, y0), (x1, y0)), _segment((x1, y0), (x1, y1)),
            _segment((x1, y1), (x0, y1)), _segment((x0, y1), (x0, y0))]


def _points(parts, rng):
    p = np.concatenate(parts)
    p = p + rng.normal(0.0, JITTER, p.shape)
    return p[:, 0].astype(np.float32), p[:, 1].astype(np.float32)


# ------------------------------------------------------------- corridor (T)
CORRIDOR = dict(length=10.0, half_width=1.2, gates=(3.5, 6.5), post_gap=0.6, post_t=0.1,
                start=(0.0, 0.0, 0.0), goal_x=9.0)


def corridor_scene(don, seed, flip=None):
    """Obstacle points of the corridor at degree of narrowness `don`.  Gate g
    has a post from one wall (tip at +W_p/2) and, post_gap further, a post
    from the other wall (tip at -W_p/2); the first post's side alternates."""
    c = CORRIDOR
    rng = np.random.default_rng(seed)
    wp = T_WIDTH / don
    H, t = c["half_width"], c["post_t"]
    parts = [_segment((-1.0, H), (c["length"], H)), _segment((-1.0, -H), (c["length"], -H))]
    for g, xg in enumerate(c["gates"]):
        s = (1.0 if g % 2 == 0 else -1.0) if flip is None else flip
        for k, x in enumerate((xg, xg + c["post_gap"])):
            side = s if k == 0 else -s
            tip = side * wp / 2.0
            parts += _box(x - t / 2, x + t / 2, min(tip, side * H), max(tip, side * H))
    return _points(parts, rng)


def corridor_params(K=1024, T=50):
    return dict(scenes.COST_DEFAULTS, K=K, T=T, nu=2, model="unicycle", footprint_kind=0,
                dt=0.1, sigma=(0.6, 1.0), u_min=(-1.0, -1.0), u_max=(2.0, 1.0),
                goal=(CORRIDOR["goal_x"] + 1.0, 0.0), w_goal=1.0, w_path=2.0, d_safe=0.05)


# ------------------------------------------------------------- wall gap (L)
GAP = dict(wall_x=3.0, wall_t=0.1, wall_half=4.0, start=(0.0, 0.0, 0.0), goal_x=6.0)


def gap_scene(width, seed):
    """Obstacle points of a 0.1 m thick wall across the robot's way with a
    centred gap of `width`."""
    g = GAP
    rng = np.random.default_rng(seed)
    x0, x1, a, H = g["wall_x"] - g["wall_t"] / 2, g["wall_x"] + g["wall_t"] / 2, width / 2, g["wall_half"]
    parts = _box(x0, x1, a, H) + _box(x0, x1, -H, -a)
    return _points(parts, rng)


def gap_params(K=4096, T=50):
    return dict(scenes.COST_DEFAULTS, K=K, T=T, nu=3, model="omni", footprint_kind=0, dt=0.1,
                sigma=(0.6, 0.6, 1.2), u_min=(-1.5, -1.0, -1.5), u_max=(1.5, 1.0, 1.5),
                goal=(GAP["goal_x"] + 1.0, 0.0), w_goal=1.0, w_path=2.0, d_safe=0.12)


# ------------------------------------------------------------- episodes
def _propagate(model, q, u, dt):
    x, y, th = q
    if model == "unicycle":
        v, w = float(u[0]), float(u[1])
        return (x + v * math.cos(th) * dt, y + v * math.sin(th) * dt, th + w * dt)
    vx, vy, w = float(u[0]), float(u[1]), float(u[2])
    c, s = math.cos(th), math.sin(th)
    return (x + (vx * c - vy * s) * dt, y + (vx * s + vy * c) * dt, th + w * dt)


def run_episode(case, planner_fp, setting, seed, steps=None, K=None, T=50):
    """One closed-loop episode.  case: "corridor" (setting = DoN) or "gap"
    (setting = gap width); planner_fp: the footprint the controller plans
    with (exact or its convex hull).  Contact is checked with the exact
    footprint.  K defaults to 1024 samples in the corridor and 4096 at the
    wall gap, whose rotate-while-passing manoeuvre is rarely sampled with
    fewer.  Returns success, steps, time, path length, mean speed and the
    minimum clearance."""
    if case == "corridor":
        ox, oy = corridor_scene(setting, seed)
        prm, exact, cfg = corridor_params(K or 1024, T), FOOTPRINT_T, CORRIDOR
        steps = steps or 400
    else:
        ox, oy = gap_scene(setting, seed)
        prm, exact, cfg = gap_params(K or 4096, T), FOOTPRINT_L, GAP
        steps = steps or 400
    rng = np.random.default_rng(seed)
    q = (cfg["start"][0], cfg["start"][1] + rng.uniform(-0.05, 0.05),
         cfg["start"][2] + rng.uniform(-0.05, 0.05))
    plan = pkg.Context(0)
    plan.set_footprint(pkg.POLYGON, planner_fp)
    plan.set_points(ox, oy)
    plan.set_guidance([(-1.0, 0.0), (cfg["goal_x"] + 1.0, 0.0)])
    check = pkg.Context(0)
    check.set_footprint(pkg.POLYGON, exact)
    check.set_points(ox, oy)
    U = torch.zeros((T, prm["nu"]), device="cuda")
    min_clear, path, reached = math.inf, 0.0, None
    try:
        for t in range(steps):
            u, _, _ = plan.mppi_step(prm, np.float32(q), U, seed, t)
            q_new = _propagate(prm["model"], q, u, prm["dt"])
            path += math.hypot(q_new[0] - q[0], q_new[1] - q[1])
            q = q_new
            pose = torch.tensor([[[q[0], q[1], math.cos(q[2]), math.sin(q[2])]]], dtype=torch.float32)
            min_clear = min(min_clear, float(check.sdf_min_poses(pose, state_offset=0)[0, 0]))
            if min_clear < 0.0:
                break
            if q[0] >= cfg["goal_x"]:
                reached = t + 1
                break
    finally:
        plan.close()
        check.close()
    ok = reached is not None and min_clear >= 0.0
    time_s = reached * prm["dt"] if ok else None
    return dict(success=bool(ok), steps=reached, time_s=time_s, path_m=path,
                speed=(path / time_s) if ok else None, min_clearance=min_clear,
                final_x=q[0])


def sweep(case, episodes=10, seed0=SWEEP_SEED0, log=print, **kw):
    settings = CORRIDOR_DON if case == "corridor" else GAP_WIDTHS
    exact = FOOTPRINT_T if case == "corridor" else FOOTPRINT_L
    rows = []
    for st in settings:
        row = dict(setting=st, don=(st if case == "corridor" else L_WIDTH / st))
        for arm, fp in (("exact", exact), ("convex_hull", convex_hull(exact))):
            eps = [run_episode(case, fp, st, seed0 + e, **kw) for e in range(episodes)]
            ok = [e for e in eps if e["success"]]
            row[arm] = dict(success_rate=len(ok) / len(eps),
                            mean_time_s=float(np.mean([e["time_s"] for e in ok])) if ok else None,
                            mean_speed=float(np.mean([e["speed"] for e in ok])) if ok else None,
                            collisions=sum(1 for e in eps if e["min_clearance"] < 0.0),
                            episodes=eps)
            log(f"{case} {st}: {arm} success {len(ok)}/{len(eps)} "
                f"time {row[arm]['mean_time_s']} speed {row[arm]['mean_speed']}")
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--episodes", type=int, default=10)
    ap.add_argument("--cases", default="corridor,gap")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    t0 = time.time()
    res = {}
    for case in args.cases.split(","):
        res[case] = sweep(case, args.episodes, log=lambda m: print(m, flush=True))
    res["seconds"] = time.time() - t0
    table = {case: [(r["don"], r["exact"]["success_rate"], r["exact"]["mean_time_s"],
                     r["convex_hull"]["success_rate"], r["convex_hull"]["mean_time_s"])
                    for r in rows] for case, rows in res.items() if case != "seconds"}
    print(json.dumps({"don_exact_hull": table}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
