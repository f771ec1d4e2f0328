"""CPU oracle for the exact-footprint MPPI step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library:
the arithmetic lives in ``oracle.c`` (plain scalar C, IEEE double precision,
plus one documented single-precision sequence for the counter-based noise and
the rollout) and in the numpy code below.

Parameters are plain dicts with the keys of :data:`PARAM_KEYS`, so the same
dict can be handed to the HIP binding and to the oracle.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
           "-fPIC", "-Wall", "-o", _LIB, _SRC, "-lm"]

MODELS = {"unicycle": 0, "ackermann": 1, "omni": 2, "spin": 3, "parallel": 4}
POLYGON, RECTS = 0, 1

PARAM_KEYS = ("K", "T", "nu", "model", "footprint_kind", "dt", "lambda_", "wheelbase",
              "sigma", "u_min", "u_max", "d_safe", "w_coll", "w_rep", "w_inf", "w_goal",
              "w_ctrl", "goal", "state_offset", "validate", "w_path", "path")


# The same source built with AddressSanitizer and UndefinedBehaviorSanitizer
# (every report fatal), for a run of the oracle's tests under the sanitizers:
# load it with EXACT_MPPI_ORACLE_LIB=<path> and the sanitizer runtimes
# preloaded into the (uninstrumented) Python process.
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
GCC_SAN_CMD = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-Wall",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-o", _LIB_SAN, _SRC, "-lm"]


def build() -> str:
    """Compile oracle.c with gcc into liboracle.so (always recompiles)."""
    subprocess.run(GCC_CMD, check=True)
    return _LIB


def build_sanitized() -> str:
    """Compile the sanitizer build liboracle_san.so (always recompiles)."""
    subprocess.run(GCC_SAN_CMD, check=True)
    return _LIB_SAN


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("EXACT_MPPI_ORACLE_LIB") or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(path)
        d, i, l, vp = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        u64, u32, f = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_float
        L.orc_seg_dist.restype = d
        L.orc_seg_dist.argtypes = [d] * 6
        L.orc_winding.restype = i
        L.orc_winding.argtypes = [vp, i, d, d]
        L.orc_inside_raycast.restype = i
        L.orc_inside_raycast.argtypes = [vp, i, d, d]
        L.orc_sdf_polygon.restype = d
        L.orc_sdf_polygon.argtypes = [vp, i, d, d]
        L.orc_sdf_box.restype = d
        L.orc_sdf_box.argtypes = [vp, d, d]
        L.orc_sdf_rectcover.restype = d
        L.orc_sdf_rectcover.argtypes = [vp, i, d, d]
        L.orc_sdf_polygon_batch.argtypes = [vp, i, vp, vp, l, vp]
        L.orc_sdf_rectcover_batch.argtypes = [vp, i, vp, vp, l, vp]
        L.orc_dmin.argtypes = [vp, vp, l, vp, vp, vp, vp, vp, l, i, vp, i, vp, vp]
        L.orc_rollout_f64.argtypes = [i, i, i, d, d, vp, vp, vp]
        L.orc_phi_obs.restype = d
        L.orc_phi_obs.argtypes = [vp, d]
        L.orc_phi_task.restype = d
        L.orc_phi_task.argtypes = [vp, d, d]
        L.orc_costs.argtypes = [vp, i, i, i, vp, vp, vp, vp, vp, vp]
        L.orc_weights.argtypes = [i, vp, d, vp]
        L.orc_update.argtypes = [i, i, i, vp, vp, vp]
        L.orc_validate_shift.restype = i
        L.orc_validate_shift.argtypes = [i, i, vp, d, vp, vp]
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_f32_sincos.argtypes = [f, vp, vp]
        L.orc_f32_log.restype = f
        L.orc_f32_log.argtypes = [f]
        L.orc_f32_tan.restype = f
        L.orc_f32_tan.argtypes = [f]
        L.orc_f32_normals.argtypes = [u64, u64, u32, u32, u64, vp]
        L.orc_f32_normals_batch.argtypes = [u64, u64, u32, u64, l, vp]
        L.orc_rollout_f32.argtypes = [i, i, i, i, f, f, vp, vp, vp, vp, vp, u64, u64, u64, i,
                                      vp, vp, vp]
        L.orc_rollout_nominal_f32.argtypes = [i, i, i, f, f, vp, vp, i, vp]
        L.orc_num_threads.restype = i
        L.orc_set_num_threads.argtypes = [i]
        L.orc_f32_features.argtypes = [vp, vp, vp, l, vp, vp, vp, i, i, vp, vp, f, vp]
        _lib = L
    return _lib


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------

def sdf_polygon(V, px, py):
    """Exact signed distance of body-frame points to the simple polygon V (B x 2)."""
    V = _f64(V)
    px, py = _f64(px).ravel(), _f64(py).ravel()
    out = np.empty(px.size)
    lib().orc_sdf_polygon_batch(_p(V), V.shape[0], _p(px), _p(py), px.size, _p(out))
    return out


def sdf_rectcover(rects, px, py):
    """Rectangle-cover signed distance (min over boxes of the box formula)."""
    rects = _f64(rects)
    px, py = _f64(px).ravel(), _f64(py).ravel()
    out = np.empty(px.size)
    lib().orc_sdf_rectcover_batch(_p(rects), rects.shape[0], _p(px), _p(py), px.size, _p(out))
    return out


def winding(V, x, y):
    V = _f64(V)
    return lib().orc_winding(_p(V), V.shape[0], float(x), float(y))


def inside_raycast(V, x, y):
    V = _f64(V)
    return lib().orc_inside_raycast(_p(V), V.shape[0], float(x), float(y))


def seg_dist(p, a, b):
    return lib().orc_seg_dist(float(p[0]), float(p[1]), float(a[0]), float(a[1]),
                              float(b[0]), float(b[1]))


def dmin(poses, tau, ox, oy, ovx=None, ovy=None, valid=None, kind=POLYGON, geom=None,
         want_argmin=False):
    """Minimum signed distance per pose over the valid (possibly moving) points.

    poses: (P, 4) (x, y, cos, sin); tau: (P,) time of each pose for moving points.
    """
    poses = _f64(poses).reshape(-1, 4)
    P = poses.shape[0]
    tau = _f64(np.zeros(P) if tau is None else tau)
    ox, oy = _f64(ox), _f64(oy)
    ovx = None if ovx is None else _f64(ovx)
    ovy = None if ovy is None else _f64(ovy)
    valid = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    geom = _f64(geom)
    out = np.empty(P)
    am = np.empty(P, dtype=np.int32) if want_argmin else None
    lib().orc_dmin(_p(poses), _p(tau), P, _p(ox), _p(oy), _p(ovx), _p(ovy), _p(valid),
                   ox.size, int(kind), _p(geom), geom.shape[0], _p(out), _p(am))
    return (out, am) if want_argmin else out


# --------------------------------------------------------------------------
# Random numbers and the FP32 sequence
# --------------------------------------------------------------------------

def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def f32_sincos(x):
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().orc_f32_sincos(float(x), ctypes.byref(s), ctypes.byref(c))
    return np.float32(s.value), np.float32(c.value)


def f32_log(x):
    return np.float32(lib().orc_f32_log(float(x)))


def f32_tan(x):
    return np.float32(lib().orc_f32_tan(float(x)))


def f32_normals(seed, step, r, h, stream=0):
    z = np.empty(4, dtype=np.float32)
    lib().orc_f32_normals(seed, step, r, h, stream, _p(z))
    return z


def f32_normals_batch(seed, step, n, h=0, stream=0):
    z = np.empty((n, 4), dtype=np.float32)
    lib().orc_f32_normals_batch(seed, step, h, stream, n, _p(z))
    return z


def _vec3(v, fill=0.0):
    a = np.full(3, fill, dtype=np.float32)
    v = np.atleast_1d(np.asarray(v, dtype=np.float32))
    a[:v.size] = v
    return a


def rollout_f32(prm, q0, U, seed, step, stream=0):
    """Noise + clamp + Euler rollout in the FP32 sequence.

    Returns poses (K, T, 4), eps_eff (K, T, nu), u (K, T, nu), all float32.
    """
    K, T, nu = prm["K"], prm["T"], prm["nu"]
    U = _f32(U).reshape(T, nu)
    q0 = _f32(q0)
    poses = np.empty((K, T, 4), dtype=np.float32)
    eps = np.empty((K, T, nu), dtype=np.float32)
    us = np.empty((K, T, nu), dtype=np.float32)
    lib().orc_rollout_f32(MODELS[prm["model"]], K, T, nu, np.float32(prm["dt"]),
                          np.float32(prm["wheelbase"]), _p(q0), _p(U), _p(_vec3(prm["sigma"])),
                          _p(_vec3(prm["u_min"], -np.inf)), _p(_vec3(prm["u_max"], np.inf)),
                          seed, step, stream, int(prm["state_offset"]), _p(poses), _p(eps),
                          _p(us))
    return poses, eps, us


def rollout_nominal_f32(prm, q0, U):
    T, nu = prm["T"], prm["nu"]
    U = _f32(U).reshape(T, nu)
    poses = np.empty((T, 4), dtype=np.float32)
    lib().orc_rollout_nominal_f32(MODELS[prm["model"]], T, nu, np.float32(prm["dt"]),
                                  np.float32(prm["wheelbase"]), _p(_f32(q0)), _p(U),
                                  int(prm["state_offset"]), _p(poses))
    return poses


def rollout_f64(model, q0, u, dt, L=1.0):
    """Double-precision Euler rollout; returns the (T+1, 3) states q_0..q_T."""
    u = _f64(u)
    T, nu = u.shape
    st = np.empty((T + 1, 3))
    lib().orc_rollout_f64(MODELS[model] if isinstance(model, str) else model, T, nu,
                          float(dt), float(L), _p(_f64(q0)), _p(u), _p(st))
    return st


# --------------------------------------------------------------------------
# Costs, weights, update, validation
# --------------------------------------------------------------------------

class _CostParams(ctypes.Structure):
    _fields_ = [("d_safe", ctypes.c_double), ("w_coll", ctypes.c_double),
                ("w_rep", ctypes.c_double), ("w_inf", ctypes.c_double),
                ("w_goal", ctypes.c_double), ("goal_x", ctypes.c_double),
                ("goal_y", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("w_ctrl", ctypes.c_double * 3), ("w_path", ctypes.c_double),
                ("n_path", ctypes.c_int), ("path", ctypes.c_void_p)]


def _cost_params(prm):
    # Every value goes through float32 first: the GPU receives the same numbers.
    f = lambda v: float(np.float32(v))
    cp = _CostParams(f(prm["d_safe"]), f(prm["w_coll"]), f(prm["w_rep"]), f(prm["w_inf"]),
                     f(prm["w_goal"]), f(prm["goal"][0]), f(prm["goal"][1]),
                     f(prm["lambda_"]))
    wc = _vec3(prm["w_ctrl"])
    for c in range(3):
        cp.w_ctrl[c] = float(wc[c])
    path = prm.get("path")
    if path is not None and len(path):
        # the waypoints go through float32 like every other GPU input
        pa = np.ascontiguousarray(np.asarray(path, dtype=np.float32).astype(np.float64).reshape(-1))
        cp.w_path = f(prm.get("w_path", 0.0))
        cp.n_path = pa.size // 2
        cp.path = pa.ctypes.data
        cp._keep = pa
    return cp


def phi_task(prm, x, y):
    cp = _cost_params(prm)
    return lib().orc_phi_task(ctypes.byref(cp), float(x), float(y))


def phi_obs(prm, d):
    cp = _cost_params(prm)
    return lib().orc_phi_obs(ctypes.byref(cp), float(d))


def costs(prm, xy, u, d):
    """J, chi, J~ per rollout from scored positions (K,T,2), controls (K,T,nu), d_min (K,T)."""
    K, T = d.shape
    nu = u.shape[-1]
    cp = _cost_params(prm)
    xy, u, d = _f64(xy), _f64(u), _f64(d)
    J = np.empty(K)
    chi = np.empty(K, dtype=np.uint8)
    Jt = np.empty(K)
    lib().orc_costs(ctypes.byref(cp), K, T, nu, _p(xy), _p(u), _p(d), _p(J), _p(chi), _p(Jt))
    return J, chi.astype(bool), Jt


def weights(Jt, lam):
    Jt = _f64(Jt)
    w = np.empty(Jt.size)
    lib().orc_weights(Jt.size, _p(Jt), float(lam), _p(w))
    return w


def update(U, w, eps):
    """U + sum_r w_r eps_r (returns a new array)."""
    eps = _f64(eps)
    K, T, nu = eps.shape
    Un = _f64(U).reshape(T, nu).copy()
    lib().orc_update(K, T, nu, _p(_f64(w)), _p(eps), _p(Un))
    return Un


def validate_shift(U, dnom, d_safe):
    """Returns (valid, u_star, U_next)."""
    U = _f64(U).copy()
    T, nu = U.shape
    us = np.empty(nu)
    ok = lib().orc_validate_shift(T, nu, _p(_f64(dnom)), float(np.float32(d_safe)), _p(U), _p(us))
    return bool(ok), us, U


def tau_of(prm, T, K=None):
    """Time of each scored pose, (h + state_offset) dt, shaped (K, T) or (T,)."""
    t = (np.arange(T) + int(prm["state_offset"])) * float(np.float32(prm["dt"]))
    return t if K is None else np.broadcast_to(t, (K, T))


def footprint_geom(prm, polygon, rects):
    kind = prm["footprint_kind"]
    return kind, (polygon if kind == POLYGON else rects)


def mppi_step(prm, q0, U, scene, seed, step, stream=0):
    """One control cycle of Algorithm 1, from scratch.

    scene: dict with ox, oy, (ovx, ovy), valid, polygon, rects.
    Sampling and rollouts use the FP32 sequence (the bit-exact contract);
    signed distances, costs, weights, update and validation are double.
    Returns a dict with every intermediate.
    """
    K, T, nu = prm["K"], prm["T"], prm["nu"]
    poses, eps, us = rollout_f32(prm, q0, U, seed, step, stream)
    kind, geom = footprint_geom(prm, scene.get("polygon"), scene.get("rects"))
    tau = tau_of(prm, T, K).ravel()
    d = dmin(poses.reshape(-1, 4), tau, scene["ox"], scene["oy"], scene.get("ovx"),
             scene.get("ovy"), scene.get("valid"), kind, geom).reshape(K, T)
    J, chi, Jt = costs(prm, poses[..., :2], us, d)
    w = weights(Jt, prm["lambda_"])
    Un = update(U, w, eps)
    out = dict(poses=poses, eps=eps, u=us, d=d, J=J, chi=chi, Jt=Jt, w=w, U_upd=Un)
    if prm.get("validate", 1):
        nom = rollout_f64(prm["model"], q0, Un, np.float32(prm["dt"]),
                          np.float32(prm["wheelbase"]))
        st = nom[1:] if prm["state_offset"] else nom[:-1]
        npose = np.stack([st[:, 0], st[:, 1], np.cos(st[:, 2]), np.sin(st[:, 2])], axis=1)
        dn = dmin(npose, tau_of(prm, T), scene["ox"], scene["oy"], scene.get("ovx"),
                  scene.get("ovy"), scene.get("valid"), kind, geom)
        ok, ustar, Unext = validate_shift(Un, dn, prm["d_safe"])
        # noise-free cost of the updated nominal: the terms of J along its
        # validation rollout (+ w_inf when unsafe); Algorithm 2 compares it
        # across motion modes
        J_nom = costs(prm, st[None, :, :2], Un[None], dn[None])[2][0]
        out.update(d_nom=dn, valid=ok, u_star=ustar, U_next=Unext, J_nom=J_nom, nom_states=st)
    else:
        out.update(valid=True, u_star=Un[0].copy(), U_next=np.concatenate([Un[1:], Un[-1:]]))
    return out


def f32_features(ox, oy, valid, q0, goal, U_prev, u_min, u_max, r_max=8.0):
    """Proposal features of one state in the FP32 sequence (64 + 2 + T*nu floats)."""
    ox, oy = _f32(ox), _f32(oy)
    U_prev = _f32(U_prev)
    T, nu = U_prev.shape
    valid = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    out = np.empty(66 + T * nu, dtype=np.float32)
    lib().orc_f32_features(_p(ox), _p(oy), _p(valid), ox.size, _p(_f32(q0)), _p(_f32(goal)),
                           _p(U_prev), T, nu, _p(_vec3(u_min, -1.0)), _p(_vec3(u_max, 1.0)),
                           np.float32(r_max), _p(out))
    return out


# --------------------------------------------------------------------------
# Hybrid-mode cycle (Section "Extension to Hybrid-Mode Platforms", Algorithm 2)
# --------------------------------------------------------------------------
SPIN = 3
OMNI = 2


def hybrid_select(J, valid, u_star, models, m_prev, tau_cool, hp):
    """Mode selection with cooldown and the actuator post-processing.

    J, valid, u_star: each mode's cycle result (J_m = its J_nom, validation
    flag, executed command in the mode's own layout).  Returns
    (u, m_star, tau_cool', stopped).
    """
    n = len(J)
    Jbar = [J[m] + (hp["lambda_switch"] if m != m_prev else 0.0) if valid[m] else math.inf
            for m in range(n)]
    if all(j == math.inf for j in Jbar):
        return np.zeros(3), m_prev, tau_cool, True          # safe stop
    m_star = min(range(n), key=lambda m: (Jbar[m], m))
    if tau_cool > 0 and m_star != m_prev:
        m_star = m_prev
    tau_new = hp["cool_max"] if m_star != m_prev else max(tau_cool - 1, 0)
    u = np.zeros(3)
    u[:len(u_star[m_star])] = u_star[m_star]
    model = models[m_star]
    if model != SPIN:                                        # translational mode
        nlin = 2 if model == OMNI else 1
        vmag = math.sqrt(sum(float(u[k]) ** 2 for k in range(nlin)))
        if hp["noise_v"] < vmag < hp["v_min"]:
            u[:nlin] *= hp["v_min"] / vmag
    else:                                                    # pure rotation
        w = float(u[0])
        if hp["noise_w"] < abs(w) < hp["w_min"]:
            u[0] = math.copysign(hp["w_min"], w)
    return u, m_star, tau_new, False


def hybrid_step(mode_prms, q0, Us, scene, seed, step, m_prev, tau_cool, hp):
    """One Algorithm-2 cycle from scratch: an Algorithm-1 cycle per mode
    (mode m draws noise on stream m), then hybrid_select."""
    res = [mppi_step(p, q0, U, scene, seed, step, stream=m)
           for m, (p, U) in enumerate(zip(mode_prms, Us))]
    J = [r["J_nom"] for r in res]
    valid = [r["valid"] for r in res]
    u_star = [r["u_star"] for r in res]
    models = [MODELS[p["model"]] if isinstance(p["model"], str) else p["model"] for p in mode_prms]
    u, m, tau, stopped = hybrid_select(J, valid, u_star, models, m_prev, tau_cool, hp)
    return dict(u=u, mode=m, tau_cool=tau, stopped=stopped, modes=res)
