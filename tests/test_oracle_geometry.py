"""Pins for the oracle's signed-distance functions (CPU only).

Each test checks the oracle against something other than itself: hand-derived
values, a different algorithm with a closed form (box formula, support-line
form of convex polygons), exact rational brute force on tiny inputs, and the
invariants a signed distance must satisfy.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from paper_2605_29663_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- closed forms

def test_golden_gap_l_footprint(orc):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "gap_l_footprint.txt"))
            if ln.strip() and not ln.startswith("#")]
    px = np.array([float(r[0]) for r in rows])
    py = np.array([float(r[1]) for r in rows])
    want = np.array([float(r[2]) for r in rows])
    got = orc.sdf_polygon(scenes.FOOTPRINT_GAP_L, px, py)
    np.testing.assert_allclose(got, want, atol=1e-12)
    got_r = orc.sdf_rectcover(scenes.RECTS_GAP_L, px, py)
    out = want >= 0     # rect cover: exact outside, sign-correct everywhere
    np.testing.assert_allclose(got_r[out], want[out], atol=1e-12)
    assert np.all((got_r < 0) == (want < 0))


def test_box_hand_values(orc):
    r = np.array([0.5, -1.0, 1.0, 0.5])           # centre (0.5,-1), half extents (1, 0.5)
    cases = [((0.5, -1.0), -0.5), ((3.5, -1.0), 2.0), ((0.5, 1.0), 1.5),
             ((2.5, 0.5), math.hypot(1.0, 1.0)), ((1.4, -1.0), -0.1), ((1.5, -1.5), 0.0)]
    for (x, y), d in cases:
        assert orc.sdf_rectcover(r[None], [x], [y])[0] == pytest.approx(d, abs=1e-14)


def test_polygon_route_equals_box_formula_on_rectangles(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        c = rng.uniform(-2, 2, 2)
        s = rng.uniform(0.05, 1.5, 2)
        V = np.array([c + [-s[0], -s[1]], c + [s[0], -s[1]], c + [s[0], s[1]], c + [-s[0], s[1]]])
        if rng.uniform() < 0.5:
            V = V[::-1]
        p = rng.uniform(-4, 4, size=(200, 2))
        dp = orc.sdf_polygon(V, p[:, 0], p[:, 1])
        db = orc.sdf_rectcover(np.concatenate([c, s])[None], p[:, 0], p[:, 1])
        np.testing.assert_allclose(dp, db, atol=1e-12)


def _regular(B, R=1.0, rot=0.3, c=(0.2, -0.1)):
    a = rot + 2 * np.pi * np.arange(B) / B
    return np.stack([c[0] + R * np.cos(a), c[1] + R * np.sin(a)], axis=1)


@pytest.mark.parametrize("B", [3, 4, 5, 7, 16, 33, 64])
def test_convex_polygon_support_form(orc, B):
    """Inside a convex polygon d = max_b n_b.(p - v_b); at the centre d = -R cos(pi/B)."""
    V = _regular(B)
    assert orc.sdf_polygon(V, [0.2], [-0.1])[0] == pytest.approx(-math.cos(math.pi / B), abs=1e-12)
    rng = np.random.default_rng(B)
    e = np.roll(V, -1, axis=0) - V
    n = np.stack([e[:, 1], -e[:, 0]], axis=1) / np.linalg.norm(e, axis=1)[:, None]  # outward (CCW)
    p = rng.uniform(-1.5, 1.5, size=(4000, 2))
    sup = ((p[:, None, :] - V[None]) * n[None]).sum(-1).max(axis=1)
    d = orc.sdf_polygon(V, p[:, 0], p[:, 1])
    inside = sup < 0
    np.testing.assert_allclose(d[inside], sup[inside], atol=1e-12)
    # outside, in the normal slab of an edge, the distance is that edge's support value
    t = ((p[:, None, :] - V[None]) * e[None]).sum(-1) / (e * e).sum(1)[None]
    for b in range(B):
        m = (sup > 0) & (np.argmax(((p[:, None, :] - V[None]) * n[None]).sum(-1), axis=1) == b) \
            & (t[:, b] > 0) & (t[:, b] < 1)
        np.testing.assert_allclose(d[m], sup[m], atol=1e-12)


def test_exterior_vertex_region(orc):
    """Points in the outer cone of a convex vertex are at the vertex distance."""
    V = _regular(6)
    for b in range(6):
        v = V[b]
        out = (v - np.array([0.2, -0.1]))
        p = v + 0.7 * out / np.linalg.norm(out)
        assert orc.sdf_polygon(V, [p[0]], [p[1]])[0] == pytest.approx(0.7, abs=1e-12)


# ---------------------------------------------------------------- brute force

def _frac_inside(V, p):
    """Exact crossing parity with rationals (half-open rule)."""
    odd = False
    B = len(V)
    for b in range(B):
        a, c = V[b], V[(b + 1) % B]
        if (a[1] > p[1]) != (c[1] > p[1]):
            xc = a[0] + (p[1] - a[1]) * (c[0] - a[0]) / (c[1] - a[1])
            if p[0] < xc:
                odd = not odd
    return odd


def _frac_seg_d2(p, a, b):
    ex, ey = b[0] - a[0], b[1] - a[1]
    t = ((p[0] - a[0]) * ex + (p[1] - a[1]) * ey) / (ex * ex + ey * ey)
    t = min(max(t, Fraction(0)), Fraction(1))
    dx, dy = p[0] - a[0] - t * ex, p[1] - a[1] - t * ey
    return dx * dx + dy * dy


TINY_POLYS = [
    [(0, 0), (4, 0), (4, 1), (1, 1), (1, 4), (0, 4)],                      # L
    [(0, 0), (5, 0), (5, 5), (3, 5), (3, 2), (2, 2), (2, 5), (0, 5)],      # U
    [(0, 0), (6, 0), (3, 2), (6, 4), (0, 4), (2, 2)],                      # bow-tie-like concave
    [(1, 0), (3, 0), (4, 2), (2, 4), (0, 2)],                              # convex pentagon
    [(0, 0), (3, 1), (6, 0), (5, 3), (6, 6), (3, 5), (0, 6), (1, 3)],      # star
]


@pytest.mark.parametrize("poly", TINY_POLYS)
def test_bruteforce_exact_grid(orc, poly):
    """Exact rational sign and squared distance on a grid that avoids the boundary."""
    V = [(Fraction(x), Fraction(y)) for x, y in poly]
    # offsets 1/7 and 1/11: a grid point on an edge line a x + b y = c with
    # integers |a|, |b| <= 6 would need 77 | (11 a + 7 b), impossible unless a = b = 0
    xs = [Fraction(k) / 2 + Fraction(1, 7) for k in range(-4, 15)]
    ys = [Fraction(k) / 2 + Fraction(1, 11) for k in range(-4, 15)]
    pts = [(x, y) for x in xs for y in ys]
    px = np.array([float(p[0]) for p in pts])
    py = np.array([float(p[1]) for p in pts])
    d = orc.sdf_polygon(np.array(poly, dtype=float), px, py)
    for k, p in enumerate(pts):
        d2 = min(_frac_seg_d2(p, V[b], V[(b + 1) % len(V)]) for b in range(len(V)))
        inside = _frac_inside(V, p)
        assert (d[k] < 0) == inside, (p, d[k])
        assert d[k] * d[k] == pytest.approx(float(d2), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("poly", TINY_POLYS)
def test_distance_vs_dense_boundary_samples(orc, poly):
    V = np.array(poly, dtype=float)
    E = np.roll(V, -1, axis=0)
    s = np.linspace(0, 1, 20001)[:-1]
    bpts = np.concatenate([V[b] + s[:, None] * (E[b] - V[b]) for b in range(len(V))])
    h = max(np.linalg.norm(E - V, axis=1)) / 20000
    rng = np.random.default_rng(7)
    p = rng.uniform(-3, 9, size=(300, 2))
    d = np.abs(orc.sdf_polygon(V, p[:, 0], p[:, 1]))
    ref = np.sqrt(((p[:, None, :] - bpts[None]) ** 2).sum(-1)).min(axis=1)
    assert np.all(d <= ref + 1e-12)
    assert np.all(ref - d <= h / 2 + 1e-12)


def test_raycast_and_winding_agree(orc):
    rng = np.random.default_rng(3)
    for _ in range(30):
        V = scenes.star_polygon(rng, int(rng.integers(3, 65)))
        for p in rng.uniform(-1.5, 1.5, size=(200, 2)):
            assert (orc.winding(V, *p) != 0) == bool(orc.inside_raycast(V, *p))


def test_shapes_are_simple_and_covers_match(orc):
    """Every polygon of the scene module is simple (area check via shoelace with the
    right sign) and each rectangle cover equals its polygon outside, with agreeing
    signs inside (rectangle cover: exact outside, sign-correct everywhere)."""
    pairs = [(scenes.RECTS_4_BOUNDARY, scenes.RECTS_4), (scenes.FOOTPRINT_GAP_L, scenes.RECTS_GAP_L)]
    pairs += [scenes.SHAPES_LTF[k] for k in "LTF"]
    rng = np.random.default_rng(11)
    for V, R in pairs:
        p = rng.uniform(-2.5, 2.5, size=(20000, 2))
        dp = orc.sdf_polygon(V, p[:, 0], p[:, 1])
        dr = orc.sdf_rectcover(R, p[:, 0], p[:, 1])
        keep = np.abs(dp) > 1e-9
        assert np.array_equal(dp[keep] < 0, dr[keep] < 0)
        out = dp > 1e-9
        np.testing.assert_allclose(dr[out], dp[out], atol=1e-12)
        inn = dp < -1e-9
        assert np.all(dr[inn] >= dp[inn] - 1e-12)   # cover interior depth never exceeds the exact one


# ---------------------------------------------------------------- invariants

def _poly_strategy():
    return st.tuples(st.integers(3, 64), st.integers(0, 2**31 - 1))


@settings(max_examples=40, deadline=None)
@given(_poly_strategy())
def test_invariants(args):
    from oracle import oracle as orc
    B, seed = args
    rng = np.random.default_rng(seed)
    V = scenes.star_polygon(rng, B)
    p = rng.uniform(-1.6, 1.6, size=(300, 2))
    d = orc.sdf_polygon(V, p[:, 0], p[:, 1])
    # 1-Lipschitz
    q = p + rng.normal(0, 0.05, size=p.shape)
    dq = orc.sdf_polygon(V, q[:, 0], q[:, 1])
    assert np.all(np.abs(d - dq) <= np.linalg.norm(p - q, axis=1) + 1e-12)
    # rigid motion of points and footprint together
    th = rng.uniform(-np.pi, np.pi)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    t = rng.uniform(-5, 5, 2)
    d2 = orc.sdf_polygon(V @ R.T + t, *(p @ R.T + t).T)
    np.testing.assert_allclose(d2, d, atol=1e-11)
    # scaling
    sc = rng.uniform(0.2, 5)
    np.testing.assert_allclose(orc.sdf_polygon(V * sc, *(p * sc).T), sc * d, atol=1e-11)
    # vertex order: reversed and cyclically shifted
    np.testing.assert_allclose(orc.sdf_polygon(V[::-1].copy(), *p.T), d, atol=1e-13)
    k = int(rng.integers(0, B))
    np.testing.assert_allclose(orc.sdf_polygon(np.roll(V, k, axis=0), *p.T), d, atol=1e-13)
    # sign flips across every edge midpoint, |d| = eps on both sides
    E = np.roll(V, -1, axis=0) - V
    n = np.stack([E[:, 1], -E[:, 0]], axis=1) / np.linalg.norm(E, axis=1)[:, None]
    mid = V + 0.5 * E
    eps = 1e-4
    dout = orc.sdf_polygon(V, *(mid + eps * n).T)
    din = orc.sdf_polygon(V, *(mid - eps * n).T)
    # a star polygon's edge midpoint can be within eps of another edge only if
    # that edge is closer than eps; the radii keep that from happening here
    assert np.all(dout > 0) and np.all(din < 0)
    np.testing.assert_allclose(dout, eps, rtol=1e-6)
    np.testing.assert_allclose(din, -eps, rtol=1e-6)


# ---------------------------------------------------------------- d_min matrix

def test_dmin_transform_mask_and_motion(orc):
    rng = np.random.default_rng(5)
    V = scenes.FOOTPRINT_L8
    P = 40
    th = rng.uniform(-np.pi, np.pi, P)
    poses = np.stack([rng.uniform(-2, 2, P), rng.uniform(-2, 2, P), np.cos(th), np.sin(th)], 1)
    body = rng.uniform(-2, 2, size=(P, 2))            # one chosen body-frame point per pose
    n = 64
    ox = rng.uniform(-6, 6, n)
    oy = rng.uniform(-6, 6, n)
    vx = rng.uniform(-1, 1, n)
    vy = rng.uniform(-1, 1, n)
    tau = rng.uniform(0, 3, P)
    valid = rng.uniform(size=n) < 0.7
    d_all = orc.dmin(poses, tau, ox, oy, vx, vy, valid, 0, V)
    # brute force in numpy: world point at tau, rotate into the body frame
    for k in range(P):
        wx = ox + vx * tau[k] - poses[k, 0]
        wy = oy + vy * tau[k] - poses[k, 1]
        c, s = poses[k, 2], poses[k, 3]
        bx, by = c * wx + s * wy, -s * wx + c * wy
        dd = orc.sdf_polygon(V, bx[valid], by[valid])
        assert d_all[k] == pytest.approx(dd.min(), abs=1e-13)
    # a world point built from a body point by the forward rigid transform
    for k in range(P):
        c, s = poses[k, 2], poses[k, 3]
        w = np.array([c * body[k, 0] - s * body[k, 1], s * body[k, 0] + c * body[k, 1]]) + poses[k, :2]
        d1 = orc.dmin(poses[k:k + 1], None, w[:1], w[1:], kind=0, geom=V)[0]
        assert d1 == pytest.approx(orc.sdf_polygon(V, body[k, :1], body[k, 1:])[0], abs=1e-12)
    # masked points never contribute; all masked gives +inf and argmin -1
    d_none, am = orc.dmin(poses, tau, ox, oy, vx, vy, np.zeros(n, bool), 0, V, want_argmin=True)
    assert np.all(np.isinf(d_none)) and np.all(d_none > 0) and np.all(am == -1)
    # argmin: lowest index among equal minima
    d_dup, am = orc.dmin(poses[:1], None, np.array([3.0, 3.0, 3.0]), np.array([0.0, 0.0, 0.0]),
                         kind=0, geom=V, want_argmin=True)
    assert am[0] == 0
