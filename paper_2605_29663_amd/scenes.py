"""Seeded synthetic inputs: footprints, obstacle point sets and step parameters.

This module holds no part of the method's arithmetic (no signed distance, no
rollout, no cost).  Both the HIP path and the CPU oracle are fed from it.
Every generator takes an explicit seed and uses ``numpy.random.default_rng``.

Footprints are given as CCW vertex arrays (B x 2, metres, body frame: +x
forward, +y left) or as rectangle covers (R x 4: centre x, centre y, half
extent x, half extent y).
"""
from __future__ import annotations

import math

import numpy as np

# --------------------------------------------------------------------------
# Footprints
# --------------------------------------------------------------------------

# 8-vertex concave L: 1.2 x 0.8 m body with a 0.4 m wide, 0.6 m long arm on
# its left side, inset 0.1 m from the front face.  Area 1.20 m^2.
FOOTPRINT_L8 = np.array([(-0.6, -0.4), (0.6, -0.4), (0.6, 0.4), (0.5, 0.4), (0.5, 1.0),
                         (0.1, 1.0), (0.1, 0.4), (-0.6, 0.4)], dtype=np.float64)

# 16-vertex rigid vehicle + towed implement: 0.7 m wide, 3.2 m long,
# area 1.8225 m^2.
FOOTPRINT_TOWED16 = np.array([(-0.4, -0.35), (1.05, -0.35), (1.3, 0.0), (1.05, 0.35),
                              (-0.4, 0.35), (-0.4, 0.05), (-0.9, 0.05), (-0.9, 0.35),
                              (-1.9, 0.35), (-1.9, 0.12), (-1.65, 0.0), (-1.9, -0.12),
                              (-1.9, -0.35), (-0.9, -0.35), (-0.9, -0.05), (-0.4, -0.05)],
                             dtype=np.float64)

# Union of 4 axis-aligned rectangles (cx, cy, hx, hy), each overlapping the
# body by at least 5 cm, and the 20-vertex boundary of that union.
RECTS_4 = np.array([(0.0, 0.0, 0.35, 0.15), (0.1, 0.0, 0.05, 0.7), (0.4, 0.0, 0.1, 0.1),
                    (-0.35, 0.0, 0.1, 0.2)], dtype=np.float64)
RECTS_4_BOUNDARY = np.array([(0.05, -0.7), (0.15, -0.7), (0.15, -0.15), (0.35, -0.15),
                             (0.35, -0.1), (0.5, -0.1), (0.5, 0.1), (0.35, 0.1), (0.35, 0.15),
                             (0.15, 0.15), (0.15, 0.7), (0.05, 0.7), (0.05, 0.15),
                             (-0.25, 0.15), (-0.25, 0.2), (-0.45, 0.2), (-0.45, -0.2),
                             (-0.25, -0.2), (-0.25, -0.15), (0.05, -0.15)], dtype=np.float64)

# The narrow-gap L footprint of the paper's omni experiment: 2.0 x 2.0 m with
# 0.4 m wide legs (polygon, and an overlapping two-rectangle cover).
FOOTPRINT_GAP_L = np.array([(0.0, 0.0), (2.0, 0.0), (2.0, 0.4), (0.4, 0.4), (0.4, 2.0),
                            (0.0, 2.0)], dtype=np.float64)
RECTS_GAP_L = np.array([(1.0, 0.2, 1.0, 0.2), (0.2, 1.0, 0.2, 1.0)], dtype=np.float64)

# Rectilinear L, T and F footprints for the rectangle-cover versus polygon
# comparison (B = 6, 8, 10 vertices; R = 2, 2, 3 overlapping rectangles).
SHAPES_LTF = {
    "L": (np.array([(-0.5, -0.5), (0.7, -0.5), (0.7, -0.1), (-0.1, -0.1), (-0.1, 0.9),
                    (-0.5, 0.9)], dtype=np.float64),
          np.array([(0.1, -0.3, 0.6, 0.2), (-0.3, 0.2, 0.2, 0.7)], dtype=np.float64)),
    "T": (np.array([(-0.8, 0.3), (-0.8, 0.7), (0.8, 0.7), (0.8, 0.3), (0.2, 0.3),
                    (0.2, -0.7), (-0.2, -0.7), (-0.2, 0.3)], dtype=np.float64)[::-1].copy(),
          np.array([(0.0, 0.5, 0.8, 0.2), (0.0, -0.15, 0.2, 0.55)], dtype=np.float64)),
    "F": (np.array([(-0.4, -0.8), (-0.1, -0.8), (-0.1, -0.1), (0.4, -0.1), (0.4, 0.2),
                    (-0.1, 0.2), (-0.1, 0.5), (0.6, 0.5), (0.6, 0.8), (-0.4, 0.8)],
                   dtype=np.float64),
          np.array([(-0.25, 0.0, 0.15, 0.8), (0.1, 0.05, 0.3, 0.15),
                    (0.2, 0.65, 0.4, 0.15)], dtype=np.float64)),
}


def star_polygon(rng, B, r_lo=0.3, r_hi=1.2):
    """Random star-shaped (hence simple) CCW polygon: sorted angles, random radii."""
    while True:
        ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=B))
        gaps = np.diff(np.concatenate([ang, ang[:1] + 2.0 * math.pi]))
        if gaps.min() > 1e-3 and gaps.max() < math.pi:
            break
    rad = rng.uniform(r_lo, r_hi, size=B)
    return np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)


def bbox(V):
    V = np.asarray(V)
    if V.shape[1] == 4:   # rectangle cover
        lo = (V[:, :2] - V[:, 2:]).min(axis=0)
        hi = (V[:, :2] + V[:, 2:]).max(axis=0)
    else:
        lo, hi = V.min(axis=0), V.max(axis=0)
    return lo, hi


def _outside_box(x, y, lo, hi, margin):
    return ~((x > lo[0] - margin) & (x < hi[0] + margin) & (y > lo[1] - margin) &
             (y < hi[1] + margin))


# --------------------------------------------------------------------------
# Step parameters
# --------------------------------------------------------------------------

COST_DEFAULTS = dict(lambda_=1.0, d_safe=0.05, w_coll=1e3, w_rep=1e2, w_inf=1e4, w_goal=1.0,
                     w_ctrl=(0.1, 0.1, 0.1), state_offset=1, validate=1, wheelbase=1.0)


def params(name, **over):
    """Step parameters of one named configuration (see CONFIG_DOC)."""
    if name == "c1":
        p = dict(K=256, T=20, nu=2, model="unicycle", footprint_kind=0, dt=0.1,
                 sigma=(math.sqrt(0.3), math.sqrt(0.6)), u_min=(-1.5, -1.0), u_max=(1.5, 1.0),
                 goal=(2.5, 0.0))
    elif name == "c2":
        p = dict(K=2048, T=40, nu=2, model="ackermann", footprint_kind=0, dt=0.05,
                 sigma=(0.5, 0.3), u_min=(-1.5, -0.6), u_max=(1.5, 0.6), goal=(0.0, 0.0))
    elif name == "c3":
        p = dict(K=4096, T=50, nu=3, model="omni", footprint_kind=1, dt=0.05,
                 sigma=(0.4, 0.2, 0.5), u_min=(-1.0, -0.4, -1.0), u_max=(1.0, 0.4, 1.0),
                 goal=(8.0, 0.0))
    else:
        raise KeyError(name)
    q = dict(COST_DEFAULTS)
    q.update(p)
    q.update(over)
    return q


# Hybrid-mode platform (Section "Extension to Hybrid-Mode Platforms"; the
# command limits of the Ranger-mini modes of the platform table): a 0.74 x
# 0.50 m body with a 0.27 x 0.2 m side attachment; dual-Ackermann (v, delta)
# with the effective wheelbase = half the 0.5 m axle distance, parallel
# motion (v_para, the lateral-translation model) and spin in place (omega).
FOOTPRINT_RANGER6 = np.array([(-0.37, -0.25), (0.37, -0.25), (0.37, 0.25), (0.10, 0.25),
                              (0.10, 0.45), (-0.37, 0.45)], dtype=np.float64)


def hybrid_modes(K=1024, T=40, dt=0.05, goal=(3.0, 0.0), **over):
    """Parameter sets of the three Ranger-mini modes (dual-Ackermann, parallel, spin)."""
    base = dict(COST_DEFAULTS, K=K, T=T, dt=dt, footprint_kind=0, goal=goal, wheelbase=0.25)
    modes = [dict(base, model="ackermann", nu=2, sigma=(0.5, 0.3), u_min=(-1.5, -0.6),
                  u_max=(1.5, 0.6)),
             dict(base, model="parallel", nu=1, sigma=(0.3,), u_min=(-0.6,), u_max=(0.6,)),
             dict(base, model="spin", nu=1, sigma=(0.5,), u_min=(-1.0,), u_max=(1.0,))]
    for m in modes:
        m.update(over)
    return modes


CONFIG_DOC = {
    "c1": "unicycle dt=0.1 K=256 T=20, L8 footprint (B=8), N=512 uniform in [-3,3]^2",
    "c2": "ackermann L=1 dt=0.05 K=2048 T=40, towed16 footprint (B=16), N=8192 corridor",
    "c3": "omni dt=0.05 K=4096 T=50, 4-rect cover (R=4), N=20000, 30% moving",
}

# --------------------------------------------------------------------------
# Obstacle point sets
# --------------------------------------------------------------------------


def scene_c1(seed=0x5EED0001, N=512):
    """N points uniform in [-3,3]^2, none inside the start footprint's box + 0.3 m."""
    rng = np.random.default_rng(seed)
    lo, hi = bbox(FOOTPRINT_L8)
    xs, ys = [], []
    while sum(len(a) for a in xs) < N:
        x = rng.uniform(-3, 3, size=N)
        y = rng.uniform(-3, 3, size=N)
        keep = _outside_box(x, y, lo, hi, 0.3)
        xs.append(x[keep]); ys.append(y[keep])
    x = np.concatenate(xs)[:N]; y = np.concatenate(ys)[:N]
    return dict(ox=x.astype(np.float32), oy=y.astype(np.float32), polygon=FOOTPRINT_L8,
                rects=None, goal=(2.5, 0.0))


def corridor(rng, n_seg=4, seg_len=(3.0, 5.0), turn_deg=45.0, width=(1.0, 1.6)):
    """Centreline vertices (n_seg+1, 2) starting at the origin heading +x, widths per segment."""
    pts = [np.zeros(2)]
    heading = 0.0
    widths = []
    for k in range(n_seg):
        if k > 0:
            heading += math.radians(rng.uniform(-turn_deg, turn_deg))
        L = rng.uniform(*seg_len)
        pts.append(pts[-1] + L * np.array([math.cos(heading), math.sin(heading)]))
        widths.append(rng.uniform(*width))
    return np.array(pts), np.array(widths)


def scene_c2(seed=0x5EED0002, N=8192, clutter_frac=0.10, clutter_keep=1.0, footprint=None):
    """Noisy corridor walls (90 %) plus uniform clutter (10 %) in the corridor box + 2 m.

    clutter_keep < 1 thins clutter that falls inside the corridor (used for
    learning data, so that most scenes stay traversable).
    """
    rng = np.random.default_rng(seed)
    fp = FOOTPRINT_TOWED16 if footprint is None else footprint
    cl, widths = corridor(rng)
    n_wall = int(round(N * (1.0 - clutter_frac)))
    n_clut = N - n_wall
    seg = rng.integers(0, len(widths), size=n_wall)
    a, b = cl[seg], cl[seg + 1]
    d = b - a
    L = np.linalg.norm(d, axis=1, keepdims=True)
    t = d / L
    nrm = np.stack([-t[:, 1], t[:, 0]], axis=1)
    s = rng.uniform(0, 1, size=(n_wall, 1)) * L
    side = np.where(rng.uniform(size=(n_wall, 1)) < 0.5, -1.0, 1.0)
    off = side * (widths[seg][:, None] / 2.0) + rng.normal(0.0, 0.02, size=(n_wall, 1))
    walls = a + s * t + off * nrm
    lo = cl.min(axis=0) - 2.0
    hi = cl.max(axis=0) + 2.0
    flo, fhi = bbox(fp)
    cx, cy = [], []
    while sum(len(v) for v in cx) < n_clut:
        x = rng.uniform(lo[0], hi[0], size=4 * n_clut)
        y = rng.uniform(lo[1], hi[1], size=4 * n_clut)
        keep = _outside_box(x, y, flo, fhi, 0.3)
        if clutter_keep < 1.0:
            # "inside the corridor": inside the oriented strip of some segment
            inside = np.zeros(x.shape, dtype=bool)
            for k in range(len(widths)):
                p0, p1 = cl[k], cl[k + 1]
                seg_len = float(np.hypot(*(p1 - p0)))
                tx, ty = (p1 - p0) / seg_len
                along = (x - p0[0]) * tx + (y - p0[1]) * ty
                across = -(x - p0[0]) * ty + (y - p0[1]) * tx
                inside |= (along >= 0) & (along <= seg_len) & (np.abs(across) < widths[k] / 2)
            keep &= ~inside | (rng.uniform(size=x.shape) < clutter_keep)
        cx.append(x[keep]); cy.append(y[keep])
    clut = np.stack([np.concatenate(cx)[:n_clut], np.concatenate(cy)[:n_clut]], axis=1)
    P = np.concatenate([walls, clut]).astype(np.float32)
    perm = rng.permutation(N)
    P = P[perm]
    return dict(ox=P[:, 0].copy(), oy=P[:, 1].copy(), polygon=fp, rects=None,
                goal=tuple(cl[-1]), centreline=cl, widths=widths)


def scene_c3(seed=0x5EED0003, N=20000, static_frac=0.7, n_clusters=50):
    """Gaussian clusters (70 %, static) plus uniform moving points (30 %, v ~ U(-1,1)^2)."""
    rng = np.random.default_rng(seed)
    n_st = int(round(N * static_frac))
    n_mv = N - n_st
    cen = []
    while len(cen) < n_clusters:
        c = rng.uniform(-10, 10, size=2)
        if np.hypot(*c) > 1.5:
            cen.append(c)
    cen = np.array(cen)
    lab = rng.integers(0, n_clusters, size=n_st)
    st = cen[lab] + rng.normal(0.0, 0.25, size=(n_st, 2))
    mv = rng.uniform(-10, 10, size=(n_mv, 2))
    vel = np.concatenate([np.zeros((n_st, 2)), rng.uniform(-1, 1, size=(n_mv, 2))])
    P = np.concatenate([st, mv])
    perm = rng.permutation(N)
    P, vel = P[perm].astype(np.float32), vel[perm].astype(np.float32)
    return dict(ox=P[:, 0].copy(), oy=P[:, 1].copy(), ovx=vel[:, 0].copy(),
                ovy=vel[:, 1].copy(), polygon=RECTS_4_BOUNDARY, rects=RECTS_4, goal=(8.0, 0.0))


def scene(name, **kw):
    return {"c1": scene_c1, "c2": scene_c2, "c3": scene_c3}[name](**kw)


def config(name, **over):
    """(params, scene) of a named configuration, the goal taken from the scene."""
    sc = scene(name)
    p = params(name, **over)
    if "goal" not in over:
        p["goal"] = tuple(float(g) for g in sc["goal"])
    return p, sc


def batch_scenes(n=64, base_seed=1000):
    """Uneven multi-scene batch: N log-uniform in [1e3, 3e4], B in 4..32 star polygons,
    K in {512, 1024, 2048, 4096}, T in 20..60, unicycle or Ackermann, points in [-8,8]^2."""
    out = []
    for s in range(n):
        rng = np.random.default_rng(base_seed + s)
        N = int(round(math.exp(rng.uniform(math.log(1e3), math.log(3e4)))))
        B = int(rng.integers(4, 33))
        K = int(rng.choice([512, 1024, 2048, 4096]))
        T = int(rng.integers(20, 61))
        uni = bool(rng.uniform() < 0.5)
        V = star_polygon(rng, B)
        P = rng.uniform(-8, 8, size=(N, 2)).astype(np.float32)
        lo, hi = bbox(V)
        keep = _outside_box(P[:, 0], P[:, 1], lo, hi, 0.3)
        P = P[keep]
        if uni:
            prm = dict(K=K, T=T, nu=2, model="unicycle", footprint_kind=0, dt=0.1,
                       sigma=(math.sqrt(0.3), math.sqrt(0.6)), u_min=(-1.5, -1.0),
                       u_max=(1.5, 1.0))
        else:
            prm = dict(K=K, T=T, nu=2, model="ackermann", footprint_kind=0, dt=0.05,
                       sigma=(0.5, 0.3), u_min=(-1.5, -0.6), u_max=(1.5, 0.6))
        q = dict(COST_DEFAULTS)
        q.update(prm)
        q["goal"] = tuple(rng.uniform(-6, 6, size=2))
        out.append((q, dict(ox=P[:, 0].copy(), oy=P[:, 1].copy(), polygon=V, rects=None,
                            goal=q["goal"])))
    return out
