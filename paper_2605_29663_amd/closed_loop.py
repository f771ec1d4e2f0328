"""Closed-loop docking benchmark: explicit footprint against its convex hull.

The paper's claim (Section "Experiments and Results", Experiment 2): an
explicit non-convex footprint keeps feasible motions that a convex proxy
removes.  Synthetic reproduction with the library's own step: a
differential-drive robot with a fork-shaped (U) footprint must drive its
forks around a post (a circle of obstacle points in front of a wall).  At
the goal the post sits in the footprint's concavity, so the goal is
collision-free for the exact footprint and in collision for its convex hull.
Each episode runs plain MPPI in closed loop (the robot follows u* with the
same Euler model in double precision), guided by a straight waypoint line.

    python -m paper_2605_29663_amd.closed_loop --episodes 8 --out result.json

Every arithmetic step runs in the library's kernels; this module only
orchestrates episodes and checks the executed poses.
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

# U-shaped footprint (CCW, body frame): body x in [-0.5, 0.3], forks
# x in [0.3, 1.1] at |y| in [0.25, 0.4]; the opening between the forks is 0.5 m.
FOOTPRINT_FORK = np.array([(-0.5, -0.4), (1.1, -0.4), (1.1, -0.25), (0.3, -0.25), (0.3, 0.25),
                           (1.1, 0.25), (1.1, 0.4), (-0.5, 0.4)], dtype=np.float64)
POST = (4.0, 0.0)          # post centre (planning frame)
POST_R = 0.12              # post radius
DOCK_DEPTH = 0.75          # post centre in the robot frame when docked
GOAL = (POST[0] - DOCK_DEPTH, POST[1])


def convex_hull(poly):
    """Counter-clockwise convex hull (Andrew's monotone chain)."""
    pts = sorted(map(tuple, np.asarray(poly, dtype=np.float64)))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return np.array(lower[:-1] + upper[:-1])


def dock_scene(seed, n_post=48, wall=True):
    """Obstacle points: the post, a wall 0.6 m behind it, small jitter."""
    rng = np.random.default_rng(seed)
    a = np.linspace(0.0, 2.0 * math.pi, n_post, endpoint=False)
    px = POST[0] + POST_R * np.cos(a)
    py = POST[1] + POST_R * np.sin(a)
    pts = [np.stack([px, py], 1)]
    if wall:
        wy = np.linspace(-2.0, 2.0, 81)
        pts.append(np.stack([np.full_like(wy, POST[0] + 0.75), wy], 1))
    p = np.concatenate(pts) + rng.normal(0.0, 0.005, (sum(len(q) for q in pts), 2))
    return p.astype(np.float32)


def params(K=1024, T=30):
    return dict(scenes.COST_DEFAULTS, K=K, T=T, nu=2, model="unicycle", footprint_kind=0,
                dt=0.1, sigma=(0.3, 0.4), u_min=(-0.6, -0.8), u_max=(0.6, 0.8), goal=GOAL,
                w_goal=1.0, w_path=2.0, d_safe=0.02)


def run_episode(footprint, seed, steps=250, K=1024, T=30, tol=0.08):
    """One closed-loop episode; returns a dict of outcome measures."""
    pts = dock_scene(seed)
    prm = params(K, T)
    ctx = pkg.Context(0)
    ctx.set_footprint(pkg.POLYGON, footprint)
    ctx.set_points(pts[:, 0], pts[:, 1])
    ctx.set_guidance([(-1.0, 0.0), GOAL])
    ctx.mppi_set_graph(True)
    rng = np.random.default_rng(seed)
    q = np.array([0.0, rng.uniform(-0.15, 0.15), rng.uniform(-0.2, 0.2)])
    U = torch.zeros((T, 2), device="cuda")
    min_clear = math.inf
    reached_at = None
    holds = 0
    for t in range(steps):
        u, valid, _ = ctx.mppi_step(prm, q.astype(np.float32), U, seed, t)
        holds += 0 if valid else 1
        v, w = float(u[0]), float(u[1])
        q = np.array([q[0] + v * math.cos(q[2]) * prm["dt"], q[1] + v * math.sin(q[2]) * prm["dt"],
                      q[2] + w * prm["dt"]])
        pose = torch.tensor([[[q[0], q[1], math.cos(q[2]), math.sin(q[2])]]], dtype=torch.float32)
        d = float(ctx.sdf_min_poses(pose, state_offset=0)[0, 0])
        min_clear = min(min_clear, d)
        if math.hypot(q[0] - GOAL[0], q[1] - GOAL[1]) < tol and reached_at is None:
            reached_at = t + 1
            break
    ctx.close()
    err = math.hypot(q[0] - GOAL[0], q[1] - GOAL[1])
    return dict(success=bool(reached_at is not None and min_clear >= 0.0), steps=reached_at,
                final_error=err, min_clearance=min_clear, holds=holds)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--episodes", type=int, default=8)
    ap.add_argument("--steps", type=int, default=250)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    t0 = time.time()
    res = {}
    for name, fp in (("exact", FOOTPRINT_FORK), ("convex_hull", convex_hull(FOOTPRINT_FORK))):
        eps = []
        for e in range(args.episodes):
            eps.append(run_episode(fp, 100 + e, steps=args.steps))
            print(f"{name} episode {e}: {eps[-1]}", flush=True)
        res[name] = dict(episodes=eps, success_rate=float(np.mean([x["success"] for x in eps])),
                         mean_final_error=float(np.mean([x["final_error"] for x in eps])))
    res["seconds"] = time.time() - t0
    summary = {k: (v["success_rate"], v["mean_final_error"]) for k, v in res.items() if k != "seconds"}
    print(json.dumps({"success_rate_and_final_error": summary}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
