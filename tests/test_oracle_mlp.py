"""Pins for the learned-proposal oracle (CPU only): the analytic gradient
against central finite differences, bfloat16 rounding, Adam's first step,
and hand-derived feature values."""
import math

import numpy as np
import pytest

from oracle import mlp


def _params(rng, n_in, H, n_out, scale=0.3):
    return np.concatenate([rng.normal(0, scale, n_in * H), rng.normal(0, 0.1, H),
                           rng.normal(0, scale, H * H), rng.normal(0, 0.1, H),
                           rng.normal(0, scale, H * n_out), rng.normal(0, 0.1, n_out)])


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_in, H, n_out, M = 7, 6, 5, 9
    th = _params(rng, n_in, H, n_out)
    X = rng.normal(size=(M, n_in))
    Y = rng.normal(size=(M, n_out))
    g, _ = mlp.backward(th, X, Y, n_in, H, n_out, bf=False)
    h = 1e-6
    fd = np.empty_like(th)
    for k in range(th.size):
        e = np.zeros_like(th)
        e[k] = h
        fd[k] = (mlp.loss(th + e, X, Y, n_in, H, n_out) - mlp.loss(th - e, X, Y, n_in, H, n_out)) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_gelu_and_derivative():
    x = np.linspace(-6, 6, 1001)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([1.0])), [0.5 * (1 + math.erf(1 / math.sqrt(2)))])
    fd = (mlp.gelu(x + 1e-6) - mlp.gelu(x - 1e-6)) / 2e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def test_bf16_rounding():
    vals = np.float32([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -2.5, 3.0e38, 1e-30, 0.0])
    want = [1.0, 1.0, 1 + 2.0 ** -6, -2.5, None, None, 0.0]
    got = mlp.bf16(vals)
    for g, w, v in zip(got, want, vals):
        if w is not None:
            assert g == w
        else:
            assert abs(g - float(v)) <= abs(float(v)) * 2.0 ** -8


def test_adam_first_step_is_signed_lr():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = mlp.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(t1, th - 0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_hand_values(orc):
    T, nu = 3, 2
    U_prev = np.float32([[0.75, -0.5], [0.0, 0.25], [-1.5, 1.0]])
    u_min, u_max = (-1.5, -1.0), (1.5, 1.0)
    q0 = np.float32([1.0, 2.0, 0.0])
    e = 0.05

    def at(r, a):
        return [1.0 + r * math.cos(a), 2.0 + r * math.sin(a)]

    pts = np.float32([at(2.0, e),                  # ahead          -> bin 0
                      at(3.0, math.pi / 2 - e),    # left           -> bin 15
                      at(1.0, math.pi - e),        # behind         -> bin 31
                      at(3.0, -math.pi / 2 + e),   # right          -> bin 48
                      at(30.0, e),                 # beyond r_max   -> bin 0 unchanged
                      at(0.5, e)])                 # masked
    valid = np.uint8([1, 1, 1, 1, 1, 0])
    f = orc.f32_features(pts[:, 0], pts[:, 1], valid, q0, (9.0, 2.0), U_prev, u_min, u_max, 8.0)
    assert f.shape == (66 + T * nu,)
    hist = f[:64]
    np.testing.assert_allclose(hist[[0, 15, 31, 48]], [0.25, 0.375, 0.125, 0.375], atol=1e-6)
    assert np.all(np.delete(hist, [0, 15, 31, 48]) == 1.0)
    np.testing.assert_allclose(f[64:66], [1.0, 0.0], atol=1e-7)   # goal 8 m ahead
    np.testing.assert_allclose(f[66:], [0.5, -0.5, 0.0, 0.25, -1.0, 1.0], atol=1e-7)
    # the same scene seen from a robot turned by +90 degrees: "ahead" is now +y
    f90 = orc.f32_features(np.float32([1.0 + 2 * math.cos(math.pi / 2 + e)]),
                           np.float32([2.0 + 2 * math.sin(math.pi / 2 + e)]), None,
                           np.float32([1.0, 2.0, math.pi / 2]), (1.0, 10.0), U_prev, u_min,
                           u_max, 8.0)
    assert abs(f90[0] - 0.25) < 1e-6 and np.all(f90[1:64] == 1.0)
    np.testing.assert_allclose(f90[64:66], [1.0, 0.0], atol=1e-6)
    # no valid point: every bin empty
    f0 = orc.f32_features(pts[:, 0], pts[:, 1], np.zeros(6, np.uint8), q0, (1.0, 10.0), U_prev,
                          u_min, u_max, 8.0)
    assert np.all(f0[:64] == 1.0)


def test_feature_bins_cover_all_directions(orc):
    """Every direction maps to one of the 64 bins in angular order, 16 per quadrant."""
    ang = np.linspace(-math.pi, math.pi, 4001)[:-1] + 1e-4
    bins = []
    for a in ang:
        p = np.float32([[2.0 * math.cos(a), 2.0 * math.sin(a)]])
        f = orc.f32_features(p[:, 0], p[:, 1], None, np.float32([0, 0, 0]), (1.0, 0.0),
                             np.zeros((1, 2), np.float32), (-1, -1), (1, 1), 8.0)
        hit = np.flatnonzero(f[:64] < 1.0)
        assert hit.size == 1
        bins.append(int(hit[0]))
    bins = np.array(bins)
    order = np.roll(bins, -int(np.argmin(bins)))     # start at the bin of angle 0
    assert np.all(np.diff(order) >= 0) and set(bins) == set(range(64))
    quad = ((ang % (2 * math.pi)) // (math.pi / 2)).astype(int)
    assert np.all(bins // 16 == quad)
