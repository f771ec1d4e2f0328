"""Row-by-row parity of one control cycle against the oracle (shared by the
single-scene, batched and hybrid-mode GPU tests).

Contract (the tolerances of the method): signed distances within 1e-5 m
absolute, signs identical except where the oracle's |d| < 1e-6 m; sampled
noise and rollouts bit-identical; augmented costs within 1e-5 relative of the
oracle's costs of the GPU's own distances (FP32 sums of at most 128 terms);
weights and updated controls within 1e-5 of the oracle's update from the
GPU's own costs; the validation decision, the executed command and the
shifted / reset nominal bit-identical given the GPU's update.
"""
import numpy as np

TOL_D = 1e-5
SIGN_BAND = 1e-6


def _np(t):
    return t if isinstance(t, np.ndarray) else t.detach().cpu().numpy()


def assert_sdf_close(d_gpu, d_orc, tol=TOL_D, band=SIGN_BAND):
    d_gpu = np.asarray(d_gpu, dtype=np.float64)
    fin = np.isfinite(d_orc)
    assert np.array_equal(np.isfinite(d_gpu), fin)
    assert np.all(d_gpu[~fin] == d_orc[~fin])
    err = np.abs(d_gpu[fin] - d_orc[fin])
    assert err.max(initial=0.0) <= tol, f"max |d err| {err.max()}"
    far = fin & (np.abs(d_orc) >= band)
    assert np.array_equal(np.signbit(d_gpu[far]), np.signbit(d_orc[far]))


def check_step_rows(orc, prm, sc, q0, U0, seed, step, u_star, valid, D, U_after, sample=None,
                    stream=0):
    """Parity of one step from the GPU's own intermediates.

    D holds device tensors of the step's diagnostics (mppi_diag layouts).  A
    batched step keeps no sampled controls (``u``) nor weights (``w``): the
    oracle's controls are used once the perturbations are found bit-exact,
    and the weights are checked through the update they produce.  sample:
    flat (r, h) indices whose d_min is checked (None: every pose).  Returns
    the oracle's J~ of the GPU's distances.
    """
    K, T, nu = prm["K"], prm["T"], prm["nu"]
    kind, geom = (0, sc["polygon"]) if prm["footprint_kind"] == 0 else (1, sc["rects"])
    # a1, a2: noise and rollouts bit-exact
    p_o, e_o, u_o = orc.rollout_f32(prm, q0, U0, seed, step, stream)
    poses, eps = _np(D["poses"]), _np(D["eps"])
    np.testing.assert_array_equal(eps, e_o)
    np.testing.assert_array_equal(poses, p_o)
    if "u" in D:
        np.testing.assert_array_equal(_np(D["u"]), u_o)
    us = _np(D["u"]) if "u" in D else u_o
    # a3-a6: d_min on the GPU's poses (all, or a sample at full size)
    d = _np(D["d_min"]).astype(np.float64)
    tau = orc.tau_of(prm, T, K)
    flat = np.arange(K * T) if sample is None else np.asarray(sample)
    d_o = orc.dmin(poses.reshape(-1, 4)[flat], tau.ravel()[flat], sc["ox"], sc["oy"],
                   sc.get("ovx"), sc.get("ovy"), sc.get("valid"), kind, geom)
    assert_sdf_close(d.ravel()[flat], d_o)
    # a7: J~ from the GPU's d_min, poses and controls
    J, chi, Jt = orc.costs(prm, poses[..., :2], us, d)
    Jg = _np(D["J"]).astype(np.float64)
    np.testing.assert_allclose(Jg, Jt, rtol=1e-5)
    # a8, a9: weights and update from the GPU's J~
    w_o = orc.weights(Jg, prm["lambda_"])
    if "w" in D:
        np.testing.assert_allclose(_np(D["w"]), w_o, atol=1e-6, rtol=1e-5)
    U_upd_o = orc.update(U0, w_o, eps)
    U_upd = _np(D["U_upd"])
    np.testing.assert_allclose(U_upd, U_upd_o, atol=1e-5)
    # a10: nominal re-rollout of the GPU's update, validation, shift / reset
    if prm.get("validate", 1):
        nom = orc.rollout_nominal_f32(prm, q0, U_upd)
        dn_o = orc.dmin(nom, orc.tau_of(prm, T), sc["ox"], sc["oy"], sc.get("ovx"),
                        sc.get("ovy"), sc.get("valid"), kind, geom)
        dn = _np(D["d_nom"]).astype(np.float64)
        assert_sdf_close(dn, dn_o)
        near = np.abs(dn_o - np.float32(prm["d_safe"])) < TOL_D
        # the decision on the GPU's own d_nom is reproduced exactly, and the
        # oracle's d_nom gives the same decision unless a value sits at d_safe
        ok_o, us_o, Un_o = orc.validate_shift(U_upd, dn, prm["d_safe"])
        assert valid == ok_o
        if not near.any():
            assert valid == orc.validate_shift(U_upd, dn_o, prm["d_safe"])[0]
        np.testing.assert_array_equal(u_star, np.float32(us_o))
        np.testing.assert_array_equal(_np(U_after), np.float32(Un_o))
        # noise-free cost of the updated nominal, from the GPU's nominal and d_nom
        Jn_o = orc.costs(prm, nom[None, :, :2], U_upd[None], dn[None])[2][0]
        np.testing.assert_allclose(float(_np(D["J_nom"])[0]), Jn_o, rtol=1e-5, atol=1e-5)
    else:
        assert np.isnan(_np(D["J_nom"])[0])
    return Jt
