#!/usr/bin/env python3
"""Benchmark of one MPPI control step with exact footprint signed distance.

A step is one pass of Algorithm 1 (sampling, rollouts, rollout-frame
transform, exact polygon signed distance, masked min over points, costs,
softmax update, nominal re-rollout and validation).  The default workload is
the largest single-GPU one: 64 independent scenes of uneven size (K 512..4096
rollouts, T 20..60 steps, N 1e3..3e4 points, 4..32-vertex star-shaped
footprints, unicycle / Ackermann) in one batched step replayed from a
captured hipGraph.  --config c1 | c2 | c3 run the single-scene workloads
(unicycle open field, Ackermann corridor, omni rectangle cover with moving
points).  FP32 on the GPU.

Prints ONE JSON line.  `value` is SDF evaluations per second of the whole step
(point-edge pairs of the sampled rollouts plus the validation pass, divided by
the step's wall time); `ms_per_step` is the step latency.  `roofline` reports
the dominant kernel (fused transform + signed distance + min) against the
VALU issue peak, timed with HIP events recorded on the library's stream
around every launch of that kernel in the timed region.  `cpu_baseline` is the
CPU oracle timed on a bounded sample of the same workload, on all host
threads (`value`, `cores`) and on one thread (`one_thread`), with the host
CPU model.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))

# MI355X FP32 VALU issue ceiling: the published FP32 vector peak (157.3 TFLOP/s)
# counts 2 flops per FMA lane-instruction, i.e. 78.6e12 lane-instructions/s =
# 256 CUs x 128 lanes/clock x 2.4 GHz.
VALU_PEAK_TOPS = 157.3 / 2

# Algorithmic VALU lane-instructions per unit of work, counted by hand from
# the formulas (not read back from the compiled code).  `frac` uses the
# count that assumes packed FP32 pairs (a 2-vector add or fma counts once):
#   11 per (pose, point, primitive): polygon edge w = p - v (1 packed add),
#     w . e' (mul + fma), clamp (med3), r = w - t e (1 packed fma), |r|^2
#     (mul + fma), running min, crossing test (2 compares + 1 fma); box
#     |p - c| - h (1 packed add, 2 abs-sub), max, min, 2 max0, squares (mul +
#     fma), signed square (fma), min;
#   5 per (pose, point): transform 3, sign select 1, min over points 1, and
#     1 more for a moving point (o + v t).
# The library evaluates a polygon edge in another algebraic form of the same
# quantities: the edge is taken from its lower end with a unit direction e
# and length l, the point's coordinates along and across it are
# u = e . (p - a) and v = e x (p - a) (2 fmas each, from the point offset and
# per-edge constants), the clipped projection is med3(u, 0, l), the squared
# distance (u - med3)^2 + v^2 (sub, mul, fma), and the crossing test is the
# sign of v.  With packed FP32 disabled that is
#   10.5 per polygon edge (the above, 2 compares, half of a 3-input min; the
#     parity XOR runs on the scalar unit) and 4 per (pose, point) (offset 2,
#     sign select 1, min over points 1);
#   10 per box and 7 per (pose, point) for the rectangle cover (offset 2,
#     rotation 4, min over points 1);
#   2 more per (pose, point) for a moving point (o + v tau),
# reported as `frac_kernel_count` beside `frac`.
OPS = {0: (11.0, 5.0), 1: (11.0, 5.0)}
OPS_MOVING_EXTRA = 1.0
OPS_KERNEL = {0: (10.5, 4.0), 1: (10.0, 7.0)}
OPS_KERNEL_MOVING_EXTRA = {0: 2.0, 1: 2.0}


def roofline_ops(kind, pairs, pose_points, moving=False, kernel_count=False):
    """VALU lane-instructions of one launch of the distance pass."""
    per_unit, per_pose_point = (OPS_KERNEL if kernel_count else OPS)[kind]
    if moving:
        per_pose_point += OPS_KERNEL_MOVING_EXTRA[kind] if kernel_count else OPS_MOVING_EXTRA
    return pairs * per_unit + pose_points * per_pose_point


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c4",
                    choices=["c1", "c2", "c3", "c4", "hybrid", "cloud", "exp1", "proposal"],
                    help="c4 (default): 64-scene batched step (graph); c1/c2/c3: single-scene step; "
                         "hybrid: three-mode cycle (Algorithm 2); cloud: point-cloud downsampling; "
                         "exp1: point-wise polygon vs rectangle-cover evaluator (L, T, F shapes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="re-tune the tile shapes instead of using the shipped table")
    ap.add_argument("--cpu-reps", type=int, default=4,
                    help="whole oracle steps timed for the CPU baseline (c1..c3); scenes of "
                         "the batch timed for it (c4, twice this many)")
    ap.add_argument("--graph", action="store_true",
                    help="time steps replayed from a captured graph of a one-scene batch "
                         "(autotuned persistent distance kernel, timed on as many eager steps "
                         "of the same batch right after)")
    ap.add_argument("--polygon-vertices", type=int, default=0,
                    help="c1/c2: replace the footprint by a seeded star-shaped polygon of this "
                         "many vertices (3..64; radii 0.15..0.4 m)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (5 times), "
                         "the reference kernel for scaling the HBM byte counters")
    return ap.parse_args()


def padded_count(kind, count):
    """Primitive count the fused kernel is instantiated for (padding is exact)."""
    if kind == 0:
        if count <= 16:
            return max(3, count)
        return (count + 1) // 2 * 2 if count <= 32 else (count + 3) // 4 * 4
    return next(b for b in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32) if count <= b)


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2605_29663_amd", "csrc", f)
                  for f in ("kernels_sdf.hip", "kernels_batch.hip", "sdf_device.hpp", "kernels.hpp")]


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_record(workload):
    """HBM bytes per launch measured by rocprofv3 counters, if they were taken on
    the current source of the distance kernels (sha256 recorded with the numbers)."""
    path = os.path.join(ROOT, "profiles", f"dmin_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256") != kernel_sha256():
        return None
    return rec.get("bytes_per_launch")


def copy_probe(mib):
    """A plain copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * 2 ** 20 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "launches": 5}))


def run_hybrid(args):
    """Hybrid-mode cycle: dual-Ackermann, parallel and spin families of K = 1024
    each on the corridor scene (N = 8192, 6-vertex footprint), graph replay."""
    import numpy as np
    import torch
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import scenes

    sc = scenes.scene_c2()
    modes = scenes.hybrid_modes(K=1024, T=40, goal=tuple(float(g) for g in sc["goal"]))
    ctx = pkg.Context(0)
    ctx.set_footprint(pkg.POLYGON, scenes.FOOTPRINT_RANGER6)
    ctx.set_points(sc["ox"], sc["oy"])
    h = pkg.Hybrid(ctx, modes)
    work = h.autotune(reps=2)
    U = h.new_nominals()
    hp = dict(lambda_switch=2.0, cool_max=5, v_min=0.1, w_min=0.2, noise_v=0.01, noise_w=0.02)
    state = (0, 0)
    q = np.zeros(3, np.float32)
    for i in range(args.warmup):
        r = h.step(q, U, 7, i, hp, *state)
        state = (r["mode"], r["tau_cool"])
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        r = h.step(q, U, 7, args.warmup + i, hp, *state)
        state = (r["mode"], r["tau_cool"])
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    N, B, T = sc["ox"].size, len(scenes.FOOTPRINT_RANGER6), 40
    pairs = sum(m["K"] * T * N * B + T * N * B for m in modes)
    print(json.dumps({
        "metric": "hybrid-mode cycle latency and SDF evals/s", "value": pairs / (ms / 1e3),
        "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                          "p95": float(np.percentile(lat, 95) * 1e3)},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded scene generator)", "execution": "hipGraph replay",
        "config": {"workload": "hybrid modes (dual-Ackermann, parallel, spin) on the corridor",
                   "modes": 3, "K_per_mode": 1024, "T": T, "N": N, "B": B,
                   "pairs_per_item": work}}))
    h.close()


def run_proposal(args):
    """Learned proposal against plain MPPI on held-out corridor scenes (the
    proposal's training workload): latency of one plain K = 4096 step, one
    plain K = 1024 step and one learned cycle (features, the network's mean,
    the fallback test on the two noise-free costs, the K = 1024 step), and the
    network's training step (batch 1024, forward + backward + Adam on the
    matrix cores).  The cost side of the comparison is the held-out
    evaluation in profiles/proposal_c2_eval.json."""
    import numpy as np
    import torch
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import learn

    net = pkg.Proposal(40, 2, hidden=256, max_batch=1024)
    net.load(os.path.join(ROOT, "paper_2605_29663_amd", "proposal_c2.bin"))
    scs = [learn.corridor_scene(learn.HELDOUT_SEED0 + s) for s in range(4)]
    ctxs = [learn.make_context(sc) for sc in scs]
    q = np.zeros(3, np.float32)
    T = 40

    def time_calls(fn, n):
        for i in range(max(1, args.warmup)):
            fn(i)
        torch.cuda.synchronize()
        lat = []
        for i in range(n):
            ts = time.perf_counter()
            fn(10 ** 4 + i)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
        return float(np.mean(lat) * 1e3), float(np.percentile(lat, 50) * 1e3)

    res = {}
    for name, K in (("plain_k4096", 4096), ("plain_k1024", 1024)):
        ms = []
        for sc, c in zip(scs, ctxs):
            prm = learn.scene_params(sc, K)
            U = torch.zeros((T, 2), device="cuda")
            ms.append(time_calls(lambda i: c.mppi_step(prm, q, U, 7, i), args.steps))
        res[name] = (float(np.mean([m[0] for m in ms])), float(np.mean([m[1] for m in ms])))
    ms = []
    fallbacks = 0
    for sc, c in zip(scs, ctxs):
        prm = learn.scene_params(sc, 1024)
        U = torch.zeros((T, 2), device="cuda")

        def cycle(i):
            nonlocal fallbacks
            _, _, _, fb = learn.learned_update(net, c, prm, q, U, 7, 1024, step=i, diag=False)
            fallbacks += int(fb)
        ms.append(time_calls(cycle, args.steps))
    res["learned_k1024"] = (float(np.mean([m[0] for m in ms])), float(np.mean([m[1] for m in ms])))

    # training step: batch 1024 of features and targets
    rng = np.random.default_rng(3)
    feat = torch.tensor(rng.uniform(0, 1, (1024, net.in_dim)).astype(np.float32), device="cuda")
    tgt = torch.tensor(rng.normal(0, 1, (1024, net.out_dim)).astype(np.float32), device="cuda")
    for i in range(5):
        net.train_step(feat, tgt, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    n_train = max(20, args.steps)
    t0 = time.perf_counter()
    for i in range(n_train):
        net.train_step(feat, tgt, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3 / n_train
    H, I, O, M = 256, net.in_dim, net.out_dim, 1024
    mac_fwd = M * (I * H + H * H + H * O)
    # backward: dW of all three layers, dX of the two upper layers
    mac_bwd = M * (I * H + H * H + H * O) + M * (H * H + H * O)
    train_tflops = 2.0 * (mac_fwd + mac_bwd) / (train_ms / 1e3) / 1e12
    ev = json.load(open(os.path.join(ROOT, "profiles", "proposal_c2_eval.json")))
    print(json.dumps({
        "metric": "learned-proposal cycle latency (K=1024 + network) vs plain MPPI K=4096",
        "value": res["learned_k1024"][0], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["learned_k1024"][0],
        "latency_ms": {"p50": res["learned_k1024"][1]},
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (network), f32",
        "data": "synthetic (seeded held-out corridor scenes)",
        "config": {"workload": "learned proposal on corridor scenes", "T": T,
                   "scenes": len(scs), "N": int(np.mean([sc["ox"].size for sc in scs]))},
        "plain_k4096_ms": res["plain_k4096"][0], "plain_k1024_ms": res["plain_k1024"][0],
        "speedup_vs_plain_k4096": res["plain_k4096"][0] / res["learned_k1024"][0],
        "fallbacks": fallbacks,
        "held_out_cost_ratio_learned_k1024_over_plain_k4096": ev["learned_small_over_plain_big"],
        "mlp_train_step": {"batch": M, "ms": train_ms, "achieved": train_tflops,
                           "peak": 2500.0, "unit": "TFLOP/s (bf16 MFMA)",
                           "frac": train_tflops / 2500.0, "bound": "mfma (latency-bound at this size)"},
    }))
    net.close()
    for c in ctxs:
        c.close()


def run_cloud(args):
    """Point-cloud pre-processing: 2^20 points -> 8192 slots."""
    import numpy as np
    import torch
    import paper_2605_29663_amd as pkg

    rng = np.random.default_rng(5)
    m, n_out = 1 << 20, 8192
    p = np.concatenate([rng.uniform(-12, 12, (m, 2)), rng.uniform(-0.5, 2.5, (m, 1))], 1)
    xyz = torch.tensor(p.astype(np.float32), device="cuda")
    ctx = pkg.Context(0)
    for i in range(args.warmup):
        ctx.cloud_downsample(xyz, (0.0, 0.0), 0.0, 1.8, 10.0, 0.1, n_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, _, _, k = ctx.cloud_downsample(xyz, (0.0, 0.0), 0.0, 1.8, 10.0, 0.1, n_out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    algo = 12.0 * m + 9.0 * n_out          # read xyz, write x, y, valid
    print(json.dumps({
        "metric": "point-cloud downsampling throughput", "value": m / (ms / 1e3),
        "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (uniform cloud)",
        "config": {"workload": "height band + voxel downsampling", "points": m, "n_out": n_out,
                   "voxel": 0.1, "r_max": 10.0, "kept": k},
        "roofline": {"bound": "hbm", "achieved": algo / (ms / 1e3) / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": algo / (ms / 1e3) / 1e9 / 8000.0, "traffic": None,
                     "note": "algorithmic bytes only; the pass is a chain of 9 small launches"}}))
    ctx.close()


def run_exp1(args):
    """Point-wise evaluator timing in the shape of the paper's Experiment 1:
    query points uniform in a 50 x 50 m square, 1e2 .. 1e6 per call, the L, T
    and F footprints as polygons and as rectangle covers."""
    import numpy as np
    import torch
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import scenes

    ctx = pkg.Context(0)
    lib = ctx.lib
    stream = torch.cuda.current_stream()
    rows = []
    for name, (poly, rects) in scenes.SHAPES_LTF.items():
        ctx.set_footprint(pkg.POLYGON, poly)
        ctx.set_footprint(pkg.RECTS, rects)
        for n in (100, 1000, 10000, 100000, 1000000):
            rng = np.random.default_rng(n)
            p = torch.tensor(rng.uniform(-25, 25, (2, n)).astype(np.float32), device="cuda")
            out = torch.empty(n, dtype=torch.float32, device="cuda")
            res = {}
            for kind, fn in (("polygon", lib.sdf_polygon), ("rect_cover", lib.sdf_rectcover)):
                args_c = (ctx.h, ctypes.c_void_p(p[0].data_ptr()), ctypes.c_void_p(p[1].data_ptr()),
                          n, ctypes.c_void_p(out.data_ptr()))
                for _ in range(max(3, args.warmup)):
                    fn(*args_c)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = max(20, args.steps)
                e0.record(stream)
                for _ in range(reps):
                    fn(*args_c)
                e1.record(stream)
                torch.cuda.synchronize()
                res[kind] = e0.elapsed_time(e1) * 1e3 / reps      # us per call
            rows.append({"shape": name, "points": n, "B": len(poly), "R": len(rects),
                         "polygon_us": res["polygon"], "rect_cover_us": res["rect_cover"],
                         "polygon_over_rect": res["polygon"] / res["rect_cover"]})
    ref = {r["shape"]: r for r in rows if r["points"] == 100000}
    print(json.dumps({
        "metric": "point-wise signed-distance evaluation time per call", "unit": "us",
        "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
        "data": "synthetic (query points uniform in a 50 x 50 m square)",
        "config": {"workload": "evaluator calls, L/T/F footprints, 1e2..1e6 points"},
        "polygon_over_rect_at_1e5": {k: v["polygon_over_rect"] for k, v in ref.items()},
        "rows": rows}))
    ctx.close()


def run_batched(args):
    """64 uneven scenes in one batched step, replayed from the captured graph."""
    import numpy as np
    import torch
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import scenes

    cases = scenes.batch_scenes(64)
    setup = {}
    tl = time.perf_counter()
    pkg.load()
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    setup["library_load_and_device_init_s"] = time.perf_counter() - tl
    ctxs, t_fp = [], []
    ts = time.perf_counter()
    for prm, sc in cases:
        c = pkg.Context(0)
        tf = time.perf_counter()
        c.set_footprint(pkg.POLYGON, sc["polygon"])
        t_fp.append(time.perf_counter() - tf)
        c.set_points(sc["ox"], sc["oy"])
        ctxs.append(c)
    setup["contexts_footprints_points_s"] = time.perf_counter() - ts
    setup["set_footprint_ms_mean"] = float(np.mean(t_fp) * 1e3)
    ts = time.perf_counter()
    b = pkg.Batch(ctxs, [p for p, _ in cases])
    setup["batch_create_s"] = time.perf_counter() - ts
    ts = time.perf_counter()
    work = b.mppi_batch_autotune(reps=2)
    setup["batch_autotune_s"] = time.perf_counter() - ts
    n = len(cases)
    U = b.new_nominals()
    q0 = np.zeros((n, 3), np.float32)
    seeds = np.arange(1000, 1000 + n, dtype=np.uint64)
    for i in range(args.warmup):
        ts = time.perf_counter()
        b.mppi_step_batched(q0, U, seeds, np.full(n, i, np.uint64), use_graph=True)
        if i == 0:
            setup["first_graph_step_incl_capture_s"] = time.perf_counter() - ts
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        b.mppi_step_batched(q0, U, seeds, np.full(n, args.warmup + i, np.uint64), use_graph=True)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    # the distance pass timed with HIP events on eager steps of the same batch
    b.set_profiling(True)
    n_eager = max(3, min(args.steps, 10))
    for i in range(n_eager):
        b.mppi_step_batched(q0, U, seeds, np.full(n, 10 ** 6 + i, np.uint64), use_graph=False)
    k_ms, k_n = b.get_profile()
    b.set_profiling(False)
    Ks = np.array([p["K"] for p, _ in cases], np.float64)
    Ts = np.array([p["T"] for p, _ in cases], np.float64)
    Ns = np.array([sc["ox"].size for _, sc in cases], np.float64)
    Bs = np.array([len(sc["polygon"]) for _, sc in cases], np.float64)
    pairs_main = float(np.sum(Ks * Ts * Ns * Bs))
    pairs_step = pairs_main + float(np.sum(Ts * Ns * Bs))
    pose_points = float(np.sum(Ks * Ts * Ns))
    ops = roofline_ops(0, pairs_main, pose_points)
    ops_kernel = roofline_ops(0, pairs_main, pose_points, kernel_count=True)
    k_avg = k_ms / max(k_n, 1)
    achieved = ops / (k_avg / 1e3) / 1e12
    achieved_kernel = ops_kernel / (k_avg / 1e3) / 1e12
    items_main, items_val, _ = b.mppi_batch_info()
    out = {
        "metric": "SDF evals/s (K*T*N*edges per MPPI step) and MPPI step latency",
        "value": pairs_step / (ms_step / 1e3), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p95": float(np.percentile(lat, 95) * 1e3)},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded scene generator)",
        "config": {"workload": "64 uneven scenes, batched persistent launch in a hipGraph",
                   "scenes": n, "pairs_per_step": pairs_step,
                   "K": "512..4096", "T": "20..60", "N": "1e3..3e4", "B": "4..32",
                   "motion_model": "unicycle / ackermann"},
        "roofline": {"bound": "alu", "kernel": "k_dmin_persistent (sampled-rollout pass)",
                     "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "T VALU lane-instr/s", "frac": achieved / VALU_PEAK_TOPS,
                     "count": "11 per point-edge pair + 5 per pose-point pair",
                     "frac_kernel_count": achieved_kernel / VALU_PEAK_TOPS,
                     "traffic": traffic_record("c4"), "kernel_ms": k_avg, "launches": k_n,
                     "timing": "HIP events around the persistent launches of eager steps",
                     "tiles": {"pairs_per_item": work, "items_main": items_main,
                               "items_validation": items_val, "source": "batch autotuner"}},
        "setup": setup,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(cases, pairs_step, max(1, 2 * args.cpu_reps))
    print(json.dumps(out))
    b.close()


def cpu_baseline_batched(cases, pairs_step, n_sample):
    """The oracle's whole step on the n_sample scenes of median size (by
    point-edge pairs) on all host threads, scaled to the batch by pair count;
    one scene at K = 64 on one thread."""
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import oracle as orc

    def pairs(prm, sc):
        return (prm["K"] * prm["T"] + prm["T"]) * sc["ox"].size * len(sc["polygon"])

    order = sorted(range(len(cases)), key=lambda s: pairs(*cases[s]))
    mid = len(order) // 2
    pick = sorted(order[max(0, mid - n_sample // 2):max(0, mid - n_sample // 2) + n_sample])
    ts = time.perf_counter()
    done = 0
    for s in pick:
        prm, sc = cases[s]
        orc.mppi_step(prm, np.zeros(3, np.float32), np.zeros((prm["T"], prm["nu"]), np.float32),
                      sc, 1000 + s, 0)
        done += pairs(prm, sc)
    cpu_s = time.perf_counter() - ts
    n_threads = orc.num_threads()
    prm, sc = cases[order[mid]]
    prm1 = dict(prm, K=64)
    orc.set_num_threads(1)
    ts = time.perf_counter()
    orc.mppi_step(prm1, np.zeros(3, np.float32), np.zeros((prm["T"], prm["nu"]), np.float32), sc,
                  1, 0)
    one_s = time.perf_counter() - ts
    orc.set_num_threads(n_threads)
    return {"value": done / cpu_s, "unit": "evals/s",
            "ms_per_step": cpu_s * 1e3 * pairs_step / done,
            "cores": n_threads, "kind": "oracle",
            "sample": f"whole oracle steps of the {len(pick)} scenes of median size "
                      f"(scenes {pick}, {done:.3g} of the batch's {pairs_step:.3g} point-edge "
                      f"pairs), {cpu_s:.1f} s; ms_per_step scaled to the whole batch by pair count",
            "one_thread": {"value": pairs(prm1, sc) / one_s, "unit": "evals/s",
                           "sample": f"one whole oracle step of scene {order[mid]} with K=64, "
                                     f"{one_s:.1f} s"},
            "host_cpu": host_cpu_model(), "host_cpus": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding across "
                                   "GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.config == "c4":
        run_batched(args)
        return
    if args.config == "hybrid":
        run_hybrid(args)
        return
    if args.config == "cloud":
        run_cloud(args)
        return
    if args.config == "proposal":
        run_proposal(args)
        return
    if args.config == "exp1":
        run_exp1(args)
        return
    import numpy as np
    import torch
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import scenes

    prm, sc = scenes.config(args.config)
    if args.polygon_vertices:
        if prm["footprint_kind"] != 0:
            sys.exit("--polygon-vertices applies to the polygon workloads (c1, c2)")
        B = args.polygon_vertices
        sc = dict(sc, polygon=scenes.star_polygon(np.random.default_rng(B), B, 0.15, 0.4))
    kind = prm["footprint_kind"]
    K, T, nu = prm["K"], prm["T"], prm["nu"]
    N = int(np.size(sc["ox"]))
    geom = sc["polygon"] if kind == 0 else sc["rects"]
    P = len(geom)

    setup = {}
    tl = time.perf_counter()
    pkg.load()
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    setup["library_load_and_device_init_s"] = time.perf_counter() - tl
    ts = time.perf_counter()
    ctx = pkg.Context(0)
    setup["context_create_ms"] = (time.perf_counter() - ts) * 1e3
    ts = time.perf_counter()
    ctx.set_footprint(kind, geom)
    setup["set_footprint_ms"] = (time.perf_counter() - ts) * 1e3
    ts = time.perf_counter()
    ctx.set_points(sc["ox"], sc["oy"], sc.get("ovx"), sc.get("ovy"), sc.get("valid"))
    setup["set_points_ms"] = (time.perf_counter() - ts) * 1e3
    U = torch.zeros((T, nu), dtype=torch.float32, device="cuda")
    params = pkg.make_params(prm)
    q0 = (0.0, 0.0, 0.0)
    seed = 0x5EED0002

    # tile shapes: the shipped table tuned on MI355X, else the autotuner
    table = os.path.join(ROOT, "paper_2605_29663_amd", "tiles_gfx950.txt")
    if os.path.exists(table) and not args.autotune:
        ctx.mppi_tune_set(open(table).read())
    key = [str(v) for v in (kind, padded_count(kind, P), int("ovx" in sc and sc["ovx"] is not None),
                            (K + 63) // 64 * 64 * T, N)]
    shipped = [ln.split() for ln in ctx.mppi_tune_get().splitlines() if ln.split()[:5] == key]
    if shipped and not args.autotune:
        tuned = (int(shipped[0][5]), int(shipped[0][6]))
        tile_source = "shipped table"
    else:
        ts = time.perf_counter()
        tuned = ctx.mppi_autotune(None, reps=3, params=params)
        setup["autotune_s"] = time.perf_counter() - ts
        tile_source = "autotuned in this run"
    if args.graph:
        ctx.mppi_set_graph(True)
    for i in range(args.warmup):
        ts = time.perf_counter()
        ctx.mppi_step(None, q0, U, seed, i, params=params)
        if i == 0:
            setup["first_step_s"] = time.perf_counter() - ts
    torch.cuda.synchronize()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        ctx.mppi_step(None, q0, U, seed, args.warmup + i, params=params)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the distance kernel timed with HIP events (recorded on the library's
    # stream around each launch) over as many steps right after the timed
    # region: the two event records per step add launch gaps that the
    # latency above should not carry (a graph replay cannot be bracketed per
    # launch at all)
    ctx.mppi_set_profiling(True)
    tp0 = time.perf_counter()
    for i in range(args.steps):
        ctx.mppi_step(None, q0, U, seed, args.warmup + args.steps + i, params=params)
    torch.cuda.synchronize()
    ms_step_events = (time.perf_counter() - tp0) * 1e3 / args.steps
    k_ms, k_n = ctx.mppi_get_profile()
    ctx.mppi_set_profiling(False)

    ms_step = (t1 - t0) * 1e3 / args.steps
    pairs_main = K * T * N * P
    pairs_step = pairs_main + (T * N * P if prm["validate"] else 0)
    value = pairs_step / (ms_step / 1e3)
    moving = sc.get("ovx") is not None
    ops_launch = roofline_ops(kind, pairs_main, K * T * N, moving)
    ops_kernel = roofline_ops(kind, pairs_main, K * T * N, moving, kernel_count=True)
    k_avg_ms = k_ms / max(k_n, 1)
    achieved = ops_launch / (k_avg_ms / 1e3) / 1e12
    achieved_kernel = ops_kernel / (k_avg_ms / 1e3) / 1e12
    workload = args.config

    out = {
        "metric": "SDF evals/s (K*T*N*edges per MPPI step) and MPPI step latency",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p95": float(np.percentile(lat, 95) * 1e3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene generator)",
        "execution": "hipGraph replay" if args.graph else "eager launches",
        "config": {"workload": {"c1": "unicycle open field", "c2": "ackermann corridor",
                                "c3": "omni rectangle cover, moving points"}[args.config]
                               + (f", star footprint of {P} vertices" if args.polygon_vertices else ""),
                   "K": K, "T": T, "N": N, ("B" if kind == 0 else "R"): P,
                   "motion_model": prm["model"], "dt": prm["dt"]},
        "roofline": {"bound": "alu",
                     "kernel": ("k_dmin_persistent (one-scene batch)" if args.graph else
                                "k_dmin_rect" if kind else
                                "k_dmin_poly" if P <= 16 else "k_dmin_poly_part"),
                     "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "T VALU lane-instr/s", "frac": achieved / VALU_PEAK_TOPS,
                     "count": f"11 per point-{'edge' if kind == 0 else 'box'} pair + "
                              f"{5 + (1 if moving else 0)} per pose-point pair",
                     "frac_kernel_count": achieved_kernel / VALU_PEAK_TOPS,
                     "traffic": (None if args.graph or args.polygon_vertices else
                                 traffic_record(workload)),
                     "kernel_ms": k_avg_ms, "launches": k_n,
                     "timing": "HIP events around every distance launch of as many steps right after "
                               "the timed region (%.4f ms per step with the events)" % ms_step_events,
                     "tiles": ({"source": "batch autotuner (queue item size)"} if args.graph else
                               {"block": tuned[0], "chunks": tuned[1], "source": tile_source})},
        "setup": setup,
    }

    if not args.no_cpu_baseline:
        sys.path.insert(0, ROOT)
        from oracle import oracle as orc
        reps = max(1, args.cpu_reps)
        ts = time.perf_counter()
        for k in range(reps):
            orc.mppi_step(prm, np.zeros(3, np.float32), np.zeros((T, nu), np.float32), sc, seed, k)
        cpu_s = time.perf_counter() - ts
        n_threads = orc.num_threads()
        # the same on one thread, over a bounded sample: one step with K / 16 rollouts
        K1 = max(64, K // 16)
        orc.set_num_threads(1)
        ts = time.perf_counter()
        orc.mppi_step(dict(prm, K=K1), np.zeros(3, np.float32), np.zeros((T, nu), np.float32), sc,
                      seed, 0)
        one_s = time.perf_counter() - ts
        orc.set_num_threads(n_threads)
        pairs_one = (K1 * T + (T if prm["validate"] else 0)) * N * P
        out["cpu_baseline"] = {"value": reps * pairs_step / cpu_s, "unit": "evals/s",
                               "ms_per_step": cpu_s * 1e3 / reps,
                               "cores": n_threads, "kind": "oracle",
                               "sample": f"{reps} whole oracle steps of the same workload "
                                         f"(K={K}, T={T}, N={N}, {P} primitives), {cpu_s:.1f} s",
                               "one_thread": {"value": pairs_one / one_s, "unit": "evals/s",
                                              "sample": f"one whole oracle step with K={K1} "
                                                        f"(otherwise the same workload), {one_s:.1f} s"},
                               "host_cpu": host_cpu_model(), "host_cpus": os.cpu_count()}
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
