"""Hybrid-mode cycle (Algorithm 2) on the GPU against the oracle.

Every mode's Algorithm-1 cycle is checked row by row from the GPU's own
intermediates, at the single-scene step's contract (noise and rollouts on the
mode's own stream bit-exact, distances within 1e-5 m, J~ within 1e-5
relative, update within 1e-5, validation, command and shifted nominal
bit-exact); the device-side selection is reproduced by the oracle's selection
on the GPU's per-mode results (mode, cooldown and stop exactly, the command
to the rounding of the single-precision deadzone scaling); and the oracle's
from-scratch cycle gives the same validation decisions (unless a distance
sits within 1e-5 of d_safe) and the same mode (unless two penalised costs are
within 1e-3)."""
import math

import numpy as np
import pytest

from paper_2605_29663_amd import scenes
from rowcheck import check_step_rows

pytestmark = pytest.mark.gpu

HP = dict(lambda_switch=2.0, cool_max=2, v_min=0.15, w_min=0.3, noise_v=0.01, noise_w=0.01)


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29663_amd as p
    p.load()
    return p


def _scene(N=1200, seed=3):
    sc = scenes.scene_c2(seed=seed, N=N, clutter_keep=0.1)
    sc["polygon"] = scenes.FOOTPRINT_RANGER6
    return sc


def _ctx(pkg, sc):
    c = pkg.Context(0)
    c.set_footprint(pkg.POLYGON, sc["polygon"])
    c.set_points(sc["ox"], sc["oy"])
    return c


def _modes(goal, **over):
    return scenes.hybrid_modes(K=192, T=24, goal=goal, **over)


def _run(pkg, orc, sc, modes, q0, U0s, seed, step, m_prev, tau, use_graph=False, hyb=None):
    import torch
    ctx = _ctx(pkg, sc) if hyb is None else None
    h = hyb or pkg.Hybrid(ctx, modes)
    U = h.new_nominals()
    for m, U0 in enumerate(U0s):
        h.nominal(U, m).copy_(torch.tensor(U0, device="cuda"))
    r = h.step(q0, U, seed, step, HP, m_prev, tau, use_graph=use_graph)
    Ua = [h.nominal(U, m).cpu().numpy() for m in range(len(modes))]
    return h, r, Ua


def _check(orc, sc, modes, q0, U0s, seed, step, m_prev, tau, r, Ua, h):
    # every mode's Algorithm-1 cycle from the GPU's own intermediates
    u_star = []
    for m, p in enumerate(modes):
        D = h.mode_diag(m)
        U_upd = D["U_upd"].cpu().numpy()
        us = U_upd[0].copy() if r["valid"][m] else np.zeros(p["nu"], np.float32)
        check_step_rows(orc, p, sc, q0, U0s[m], seed, step, us, bool(r["valid"][m]), D, Ua[m],
                        stream=m)
        assert float(D["J_nom"].cpu()[0]) == r["J"][m]
        u_star.append(us)
    # the selection on the GPU's own per-mode results
    models = [pkgmodel(p) for p in modes]
    u, mode, tau_n, stopped = orc.hybrid_select(r["J"].astype(np.float64), r["valid"], u_star,
                                                models, m_prev, tau, HP)
    assert (mode, tau_n, stopped) == (r["mode"], r["tau_cool"], r["stopped"])
    np.testing.assert_allclose(r["u"], u, rtol=1e-6, atol=1e-7)
    # the oracle's from-scratch cycle: same decisions away from the thresholds
    ref = orc.hybrid_step(modes, q0, U0s, sc, seed, step, m_prev, tau, HP)
    for m, res in enumerate(ref["modes"]):
        near = np.any(np.abs(res["d_nom"] - np.float32(modes[m]["d_safe"])) < 1e-5)
        if not near:
            assert bool(r["valid"][m]) == bool(res["valid"]), m
    Jb = [res["J_nom"] + (HP["lambda_switch"] if m != m_prev else 0) if res["valid"] else math.inf
          for m, res in enumerate(ref["modes"])]
    fin = sorted(j for j in Jb if j < math.inf)
    if len(fin) < 2 or fin[1] - fin[0] > 1e-3 * max(1.0, abs(fin[0])):
        assert ref["mode"] == r["mode"]
    return ref


def pkgmodel(p):
    from oracle import oracle as orc
    return orc.MODELS[p["model"]] if isinstance(p["model"], str) else p["model"]


@pytest.mark.parametrize("B", [None, 64])
def test_hybrid_cycle_matches_oracle(pkg, orc, B):
    """The Ranger-like 6-vertex footprint, and a 64-vertex one (the lane-quad
    register class of the batched distance pass)."""
    sc = _scene()
    if B:
        sc["polygon"] = scenes.star_polygon(np.random.default_rng(B), B, 0.15, 0.4)
    modes = _modes(goal=tuple(float(g) for g in sc["goal"]))
    rng = np.random.default_rng(2)
    U0s = [np.clip(0.3 * rng.standard_normal((24, p["nu"])), p["u_min"], p["u_max"]).astype(np.float32)
           for p in modes]
    q0 = np.float32([0.05, -0.02, 0.03])
    for m_prev, tau in ((0, 0), (1, 0), (2, 1), (1, 2)):
        h, r, Ua = _run(pkg, orc, sc, modes, q0, U0s, 77, 4, m_prev, tau)
        _check(orc, sc, modes, q0, U0s, 77, 4, m_prev, tau, r, Ua, h)
        h.close()


def test_hybrid_closed_loop_graph_equals_eager(pkg, orc):
    """Three chained cycles: the graph replay is bit-identical to eager
    execution, and each cycle matches the oracle from the GPU's state."""
    import torch
    sc = _scene(seed=5)
    modes = _modes(goal=tuple(float(g) for g in sc["goal"]))
    ctx = _ctx(pkg, sc)
    he, hg = pkg.Hybrid(ctx, modes), pkg.Hybrid(ctx, modes)
    Ue, Ug = he.new_nominals(), hg.new_nominals()
    q = np.zeros(3, np.float32)
    state_e = state_g = (0, 0)
    for t in range(3):
        U0s = [he.nominal(Ue, m).cpu().numpy().copy() for m in range(3)]
        re = he.step(q, Ue, 11, t, HP, *state_e, use_graph=False)
        rg = hg.step(q, Ug, 11, t, HP, *state_g, use_graph=True)
        assert torch.equal(Ue, Ug)
        np.testing.assert_array_equal(re["u"], rg["u"])
        np.testing.assert_array_equal(re["J"], rg["J"])
        assert (re["mode"], re["tau_cool"]) == (rg["mode"], rg["tau_cool"])
        Ua = [he.nominal(Ue, m).cpu().numpy() for m in range(3)]
        _check(orc, sc, modes, q, U0s, 11, t, *state_e, re, Ua, he)
        state_e = state_g = (re["mode"], re["tau_cool"])
        q = q + np.float32([0.02, 0.0, 0.0])
    he.close()
    hg.close()


def test_hybrid_safe_stop(pkg, orc):
    """Points inside the footprint at every pose: no mode validates; zero
    command, the previous mode and cooldown are kept, every mode resets."""
    import torch
    ang = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    sc = dict(ox=(0.05 * np.cos(ang)).astype(np.float32), oy=(0.05 * np.sin(ang)).astype(np.float32),
              polygon=scenes.FOOTPRINT_RANGER6)
    modes = _modes(goal=(3.0, 0.0), sigma=(1e-3, 1e-3), u_min=(-0.01, -0.01), u_max=(0.01, 0.01))
    for p in modes:
        p["sigma"], p["u_min"], p["u_max"] = p["sigma"][:p["nu"]], p["u_min"][:p["nu"]], p["u_max"][:p["nu"]]
    U0s = [np.zeros((24, p["nu"]), np.float32) for p in modes]
    h, r, Ua = _run(pkg, orc, sc, modes, np.zeros(3, np.float32), U0s, 1, 0, 2, 1)
    assert r["stopped"] and r["mode"] == 2 and r["tau_cool"] == 1
    assert np.all(r["u"] == 0) and not r["valid"].any()
    assert all(np.all(u == 0) for u in Ua)
    h.close()


def test_hybrid_argument_errors(pkg):
    sc = _scene(N=200)
    ctx = _ctx(pkg, sc)
    modes = _modes(goal=(3.0, 0.0))
    with pytest.raises(pkg.MppiError):
        pkg.Hybrid(ctx, [dict(m, validate=0) for m in modes])
    with pytest.raises(pkg.MppiError):
        pkg.Hybrid(ctx, modes * 3)          # more than 8 modes
    h = pkg.Hybrid(ctx, modes)
    U = h.new_nominals()
    with pytest.raises(pkg.MppiError):
        h.step(np.zeros(3), U, 0, 0, HP, 3, 0)     # m_prev out of range
    with pytest.raises(pkg.MppiError):
        h.step(np.zeros(3), U, 0, 0, dict(HP, cool_max=-1), 0, 0)
    h.close()


def test_hybrid_autotuned_equals_default(pkg):
    """The autotuned queue item size changes no bit of the cycle."""
    import torch
    sc = _scene()
    modes = _modes(tuple(float(g) for g in sc["goal"]))
    q0 = np.float32([0.0, 0.05, 0.02])
    res = []
    for tune in (False, True):
        c = _ctx(pkg, sc)
        h = pkg.Hybrid(c, modes)
        if tune:
            assert 2 ** 16 <= h.autotune(reps=1) <= 2 ** 26
        U = h.new_nominals()
        r = h.step(q0, U, 11, 0, HP, 0, 0, use_graph=True)
        res.append((r["u"], r["mode"], r["J"], U.cpu().numpy()))
        h.close()
    np.testing.assert_array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]
    np.testing.assert_array_equal(res[0][2], res[1][2])
    np.testing.assert_array_equal(res[0][3], res[1][3])
