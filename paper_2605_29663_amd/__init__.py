"""MI355X (gfx950) library for one MPPI control step with exact footprint signed distance.

Thin ctypes binding over the C ABI declared in ``include/exact_mppi.h``:
argument checking and marshalling only, every step runs in the HIP kernels of
``libexact_mppi.so``.  PyTorch supplies device memory and streams.

Loading fails loudly (``RuntimeError``) when the library has not been built;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch  # noqa: F401  (load torch's HIP runtime before the library binds to it)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexact_mppi.so")

MPPI_OK, MPPI_E_ARG, MPPI_E_FOOTPRINT, MPPI_E_NO_FOOTPRINT = 0, -1, -2, -3
MPPI_E_CAPACITY, MPPI_E_HIP, MPPI_E_STATE = -4, -5, -6
POLYGON, RECTS = 0, 1
MODELS = {"unicycle": 0, "ackermann": 1, "omni": 2, "spin": 3, "parallel": 4}

EXPORTS = ("mppi_create", "mppi_destroy", "mppi_last_error", "mppi_check_footprint",
           "set_footprint", "set_points", "set_guidance", "cloud_downsample",
           "sdf_polygon", "sdf_rectcover", "sdf_min_poses", "sdf_min_poses_noalloc",
           "mppi_sequence_costs", "mppi_rollout", "mppi_step",
           "mppi_autotune", "mppi_tune_get", "mppi_tune_set", "mppi_set_tiles", "mppi_set_graph",
           "mppi_set_profiling", "mppi_get_profile",
           "mppi_batch_create", "mppi_batch_destroy", "mppi_batch_last_error",
           "mppi_batch_u_offsets", "mppi_batch_refresh", "mppi_step_batched",
           "mppi_batch_autotune", "mppi_batch_set_work", "mppi_batch_info", "mppi_batch_nominal_costs",
           "mppi_batch_set_profiling", "mppi_batch_get_profile", "mppi_batch_scene_diag",
           "mppi_hybrid_create", "mppi_hybrid_destroy", "mppi_hybrid_last_error",
           "mppi_hybrid_batch", "mppi_hybrid_step",
           "proposal_create", "proposal_destroy", "proposal_last_error", "proposal_num_params",
           "proposal_shape", "proposal_set_params", "proposal_get_params", "proposal_set_scaling",
           "proposal_features", "proposal_forward", "proposal_mean", "proposal_normalize",
           "proposal_set_residual",
           "proposal_train_step", "proposal_get_buffer", "proposal_save", "proposal_load")


class MppiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class MppiParams(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("T", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("model", ctypes.c_int32), ("footprint_kind", ctypes.c_int32),
                ("dt", ctypes.c_float), ("lambda_", ctypes.c_float), ("wheelbase", ctypes.c_float),
                ("sigma", ctypes.c_float * 3), ("u_min", ctypes.c_float * 3),
                ("u_max", ctypes.c_float * 3), ("d_safe", ctypes.c_float),
                ("w_coll", ctypes.c_float), ("w_rep", ctypes.c_float), ("w_inf", ctypes.c_float),
                ("w_goal", ctypes.c_float), ("w_ctrl", ctypes.c_float * 3),
                ("goal", ctypes.c_float * 2), ("state_offset", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("w_path", ctypes.c_float)]


class CloudParams(ctypes.Structure):
    _fields_ = [("z_min", ctypes.c_float), ("z_max", ctypes.c_float), ("r_max", ctypes.c_float),
                ("voxel", ctypes.c_float), ("n_out", ctypes.c_int32)]


class HybridParams(ctypes.Structure):
    _fields_ = [("lambda_switch", ctypes.c_float), ("cool_max", ctypes.c_int32),
                ("v_min", ctypes.c_float), ("w_min", ctypes.c_float),
                ("noise_v", ctypes.c_float), ("noise_w", ctypes.c_float)]


class MppiDiag(ctypes.Structure):
    @classmethod
    def names(cls):
        return [f[0] for f in cls._fields_]

    _fields_ = [(n, ctypes.c_void_p) for n in
                ("d_min", "argmin", "J", "w", "poses", "eps", "u", "U_upd", "d_nom", "J_nom")]


_lib = None


def load():
    """Load libexact_mppi.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2605_29663_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, f, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_uint64
    # every entry point returns an int status unless set otherwise below
    for name in EXPORTS:
        getattr(L, name).restype = i
    L.mppi_create.argtypes = [ctypes.POINTER(vp), i, vp]
    L.mppi_destroy.argtypes = [vp]
    L.mppi_last_error.argtypes = [vp]
    L.mppi_last_error.restype = ctypes.c_char_p
    L.mppi_check_footprint.argtypes = [i, vp, i, ctypes.c_char_p, i]
    L.set_footprint.argtypes = [vp, i, vp, i]
    L.set_points.argtypes = [vp, vp, vp, vp, vp, vp, i]
    L.set_guidance.argtypes = [vp, vp, i]
    L.cloud_downsample.argtypes = [vp, vp, i, vp, ctypes.POINTER(CloudParams), vp, vp, vp,
                                   ctypes.POINTER(i)]
    L.sdf_polygon.argtypes = [vp, vp, vp, i, vp]
    L.sdf_rectcover.argtypes = [vp, vp, vp, i, vp]
    L.sdf_min_poses.argtypes = [vp, vp, i, i, f, i, i, vp, vp]
    L.sdf_min_poses_noalloc.argtypes = [vp, vp, i, i, f, i, i, vp, vp]
    L.mppi_rollout.argtypes = [vp, ctypes.POINTER(MppiParams), vp, vp, u64, u64, vp, vp, vp]
    L.mppi_sequence_costs.argtypes = [vp, ctypes.POINTER(MppiParams), vp, vp, i, vp]
    L.mppi_step.argtypes = [vp, ctypes.POINTER(MppiParams), vp, vp, u64, u64, vp,
                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(MppiDiag)]
    L.mppi_autotune.argtypes = [vp, ctypes.POINTER(MppiParams), i, ctypes.POINTER(i),
                                ctypes.POINTER(i)]
    L.mppi_set_tiles.argtypes = [vp, i, i]
    L.mppi_set_graph.argtypes = [vp, i]
    L.mppi_tune_get.argtypes = [vp, ctypes.c_char_p, i]
    L.mppi_tune_set.argtypes = [vp, ctypes.c_char_p]
    L.mppi_set_profiling.argtypes = [vp, i]
    L.mppi_get_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_longlong)]
    L.mppi_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(MppiParams), i, vp]
    L.mppi_batch_destroy.argtypes = [vp]
    L.mppi_batch_last_error.argtypes = [vp]
    L.mppi_batch_last_error.restype = ctypes.c_char_p
    L.mppi_batch_u_offsets.argtypes = [vp, ctypes.POINTER(i)]
    L.mppi_batch_refresh.argtypes = [vp]
    L.mppi_step_batched.argtypes = [vp, vp, vp, vp, vp, vp, vp, i]
    L.mppi_batch_autotune.argtypes = [vp, i, ctypes.POINTER(ctypes.c_double)]
    L.mppi_batch_set_work.argtypes = [vp, ctypes.c_double]
    L.mppi_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]
    L.mppi_batch_nominal_costs.argtypes = [vp, vp]
    L.mppi_batch_set_profiling.argtypes = [vp, i]
    L.mppi_batch_get_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_longlong)]
    L.mppi_batch_scene_diag.argtypes = [vp, i, ctypes.POINTER(MppiDiag)]
    L.mppi_hybrid_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(MppiParams), i, vp]
    L.mppi_hybrid_destroy.argtypes = [vp]
    L.mppi_hybrid_last_error.argtypes = [vp]
    L.mppi_hybrid_last_error.restype = ctypes.c_char_p
    L.mppi_hybrid_batch.argtypes = [vp]
    L.mppi_hybrid_batch.restype = vp
    L.mppi_hybrid_step.argtypes = [vp, vp, vp, u64, u64, ctypes.POINTER(HybridParams),
                                   ctypes.POINTER(i), ctypes.POINTER(i), vp, ctypes.POINTER(i),
                                   vp, vp, i]
    ll = ctypes.c_longlong
    L.proposal_create.argtypes = [ctypes.POINTER(vp), i, vp, i, i, i, i]
    L.proposal_destroy.argtypes = [vp]
    L.proposal_last_error.argtypes = [vp]
    L.proposal_last_error.restype = ctypes.c_char_p
    L.proposal_num_params.argtypes = [vp]
    L.proposal_num_params.restype = ll
    L.proposal_shape.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.proposal_set_params.argtypes = [vp, vp, ll]
    L.proposal_get_params.argtypes = [vp, vp, ll]
    L.proposal_set_scaling.argtypes = [vp, ctypes.POINTER(MppiParams), f]
    L.proposal_features.argtypes = [vp, vp, vp, vp, i, vp]
    L.proposal_forward.argtypes = [vp, vp, i, vp]
    L.proposal_mean.argtypes = [vp, vp, i, vp]
    L.proposal_normalize.argtypes = [vp, vp, vp, i, vp]
    L.proposal_set_residual.argtypes = [vp, f]
    L.proposal_train_step.argtypes = [vp, vp, vp, i, f, ctypes.POINTER(f)]
    L.proposal_get_buffer.argtypes = [vp, i, vp, ll]
    L.proposal_save.argtypes = [vp, ctypes.c_char_p]
    L.proposal_load.argtypes = [vp, ctypes.c_char_p]
    _lib = L
    return L


def check_footprint(kind, data):
    """Host-only footprint validation: returns (code, message)."""
    a = np.ascontiguousarray(np.asarray(data, dtype=np.float32))
    count = a.shape[0] if a.ndim == 2 else a.size // (2 if kind == POLYGON else 4)
    msg = ctypes.create_string_buffer(512)
    rc = load().mppi_check_footprint(int(kind), a.ctypes.data_as(ctypes.c_void_p), int(count),
                                     msg, 512)
    return rc, msg.value.decode()


def make_params(p) -> MppiParams:
    """C parameter struct from a plain dict (the same dict the oracle takes)."""
    m = MppiParams()
    m.K, m.T, m.nu = int(p["K"]), int(p["T"]), int(p["nu"])
    m.model = MODELS[p["model"]] if isinstance(p["model"], str) else int(p["model"])
    m.footprint_kind = int(p["footprint_kind"])
    m.dt, m.lambda_, m.wheelbase = float(p["dt"]), float(p["lambda_"]), float(p["wheelbase"])
    for name in ("sigma", "u_min", "u_max", "w_ctrl"):
        v = list(p[name])
        arr = getattr(m, name)
        for c in range(3):
            arr[c] = float(v[c]) if c < len(v) else 0.0
    for name in ("d_safe", "w_coll", "w_rep", "w_inf", "w_goal"):
        setattr(m, name, float(p[name]))
    m.goal[0], m.goal[1] = float(p["goal"][0]), float(p["goal"][1])
    m.state_offset = int(p["state_offset"])
    m.validate = int(p.get("validate", 1))
    m.w_path = float(p.get("w_path", 0.0))
    return m


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, device, name):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t), dtype=torch.float32)
    if t.dtype != torch.float32:
        raise TypeError(f"{name}: float32 expected, got {t.dtype}")
    return t.to(device).contiguous()


class Context:
    """One library context (device buffers for footprint, points and workspaces)."""

    def __init__(self, device=0, stream=None):
        self.lib = load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.lib.mppi_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.mppi_last_error(None).decode())
        self.h = h
        self._keep = []
        self._step_bufs = ((ctypes.c_float * 3)(), (ctypes.c_float * 3)(), ctypes.c_int(0))

    def close(self):
        if getattr(self, "h", None):
            self.lib.mppi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.mppi_last_error(self.h).decode())

    # ------------------------------------------------------------------ API
    def set_guidance(self, waypoints):
        """Guidance polyline (n, 2) in the planning frame; None or empty clears it."""
        if waypoints is None or len(waypoints) == 0:
            self._check(self.lib.set_guidance(self.h, None, 0))
            return
        a = np.ascontiguousarray(np.asarray(waypoints, dtype=np.float32).reshape(-1, 2))
        self._check(self.lib.set_guidance(self.h, a.ctypes.data_as(ctypes.c_void_p), a.shape[0]))

    def cloud_downsample(self, xyz, center, z_min, z_max, r_max, voxel, n_out):
        """Height band + range filter and voxel downsampling of a device (m, 3)
        cloud to n_out slots.  Returns (x, y, valid, n_kept), device outputs."""
        xyz = _dev_f32(xyz, self.device, "xyz").reshape(-1, 3)
        m = xyz.shape[0]
        x = torch.empty(max(n_out, 1), dtype=torch.float32, device=self.device)
        y = torch.empty_like(x)
        valid = torch.empty(max(n_out, 1), dtype=torch.uint8, device=self.device)
        cp = CloudParams(float(z_min), float(z_max), float(r_max), float(voxel), int(n_out))
        c = (ctypes.c_float * 2)(float(center[0]), float(center[1]))
        k = ctypes.c_int(0)
        self._check(self.lib.cloud_downsample(self.h, _ptr(xyz), m, c, ctypes.byref(cp), _ptr(x),
                                              _ptr(y), _ptr(valid), ctypes.byref(k)))
        return x[:n_out], y[:n_out], valid[:n_out], k.value

    def set_footprint(self, kind, data):
        a = np.ascontiguousarray(np.asarray(data, dtype=np.float32))
        count = a.shape[0] if a.ndim == 2 else a.size // (2 if kind == POLYGON else 4)
        self._check(self.lib.set_footprint(self.h, int(kind), a.ctypes.data_as(ctypes.c_void_p),
                                           int(count)))

    def set_points(self, x, y, vx=None, vy=None, valid=None):
        x = _dev_f32(x, self.device, "x")
        y = _dev_f32(y, self.device, "y")
        vx = None if vx is None else _dev_f32(vx, self.device, "vx")
        vy = None if vy is None else _dev_f32(vy, self.device, "vy")
        if valid is not None:
            valid = torch.as_tensor(np.asarray(valid) if not isinstance(valid, torch.Tensor)
                                    else valid).to(self.device, torch.uint8).contiguous()
        n = x.numel()
        for t in (y, vx, vy, valid):
            if t is not None and t.numel() != n:
                raise ValueError("point arrays differ in length")
        self._check(self.lib.set_points(self.h, _ptr(x), _ptr(y), _ptr(vx), _ptr(vy),
                                        _ptr(valid), n))
        # the copy is stream-ordered: keep the sources alive until the stream passes it
        self._keep = [x, y, vx, vy, valid]

    def _sdf(self, fn, px, py):
        px = _dev_f32(px, self.device, "px")
        py = _dev_f32(py, self.device, "py")
        out = torch.empty_like(px)
        self._check(fn(self.h, _ptr(px), _ptr(py), px.numel(), _ptr(out)))
        return out

    def sdf_polygon(self, px, py):
        return self._sdf(self.lib.sdf_polygon, px, py)

    def sdf_rectcover(self, px, py):
        return self._sdf(self.lib.sdf_rectcover, px, py)

    def sdf_min_poses(self, poses, dt=0.0, state_offset=1, kind=POLYGON, argmin=False):
        """poses: (K, T, 4) (x, y, cos, sin).  Returns d_min (K, T) [and argmin]."""
        poses = _dev_f32(poses, self.device, "poses")
        K, T = poses.shape[0], poses.shape[1]
        d = torch.empty((K, T), dtype=torch.float32, device=self.device)
        am = torch.empty((K, T), dtype=torch.int32, device=self.device) if argmin else None
        self._check(self.lib.sdf_min_poses(self.h, _ptr(poses), K, T, float(dt),
                                           int(state_offset), int(kind), _ptr(d), _ptr(am)))
        return (d, am) if argmin else d

    def sdf_min_poses_noalloc(self, poses, d_min, argmin=None, dt=0.0, state_offset=1,
                              kind=POLYGON):
        """sdf_min_poses into caller-provided outputs with the library's fixed
        workspace (no device allocation in the call).  poses (K, T, 4), d_min
        (K, T) float32 and argmin (K, T) int32 or None: contiguous device tensors."""
        for t, dt_ in ((poses, torch.float32), (d_min, torch.float32), (argmin, torch.int32)):
            if t is not None and not (t.is_cuda and t.dtype == dt_ and t.is_contiguous()):
                raise TypeError("poses, d_min, argmin: contiguous device tensors of the right type")
        K, T = poses.shape[0], poses.shape[1]
        if d_min.shape != (K, T) or (argmin is not None and argmin.shape != (K, T)):
            raise ValueError("outputs must be (K, T)")
        self._check(self.lib.sdf_min_poses_noalloc(self.h, _ptr(poses), K, T, float(dt),
                                                   int(state_offset), int(kind), _ptr(d_min),
                                                   _ptr(argmin)))

    def mppi_rollout(self, prm, q0, U, seed, step):
        p = make_params(prm)
        U = _dev_f32(U, self.device, "U")
        K, T, nu = p.K, p.T, p.nu
        poses = torch.empty((K, T, 4), dtype=torch.float32, device=self.device)
        eps = torch.empty((K, T, nu), dtype=torch.float32, device=self.device)
        us = torch.empty((K, T, nu), dtype=torch.float32, device=self.device)
        q = (ctypes.c_float * 3)(*[float(v) for v in q0])
        self._check(self.lib.mppi_rollout(self.h, ctypes.byref(p), q, _ptr(U), int(seed),
                                          int(step), _ptr(poses), _ptr(eps), _ptr(us)))
        return poses, eps, us

    def mppi_sequence_costs(self, prm, q0, Useq):
        """Noise-free augmented costs J~ of the control sequences Useq (n, T, nu)
        from q0; returns a device tensor of n costs (stream-ordered)."""
        p = make_params(prm)
        Useq = _dev_f32(Useq, self.device, "Useq").contiguous()
        n = Useq.numel() // (p.T * p.nu)
        if n * p.T * p.nu != Useq.numel() or n < 1:
            raise ValueError("Useq must hold n whole (T, nu) sequences")
        J = torch.empty(n, dtype=torch.float32, device=self.device)
        q = (ctypes.c_float * 3)(*[float(v) for v in q0])
        self._check(self.lib.mppi_sequence_costs(self.h, ctypes.byref(p), q, _ptr(Useq), int(n), _ptr(J)))
        return J

    def mppi_autotune(self, prm, reps=3, params=None):
        """Time the candidate tile shapes for prm's shape; returns (block, nchunk)."""
        p = params if params is not None else make_params(prm)
        b, c = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.mppi_autotune(self.h, ctypes.byref(p), int(reps), ctypes.byref(b),
                                           ctypes.byref(c)))
        return b.value, c.value

    def mppi_tune_get(self):
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self.lib.mppi_tune_get(self.h, buf, len(buf)))
        return buf.value.decode()

    def mppi_tune_set(self, text):
        self._check(self.lib.mppi_tune_set(self.h, text.encode()))

    def mppi_set_graph(self, enable=True):
        """Replay steps without diagnostics from a captured graph (bit-identical)."""
        self._check(self.lib.mppi_set_graph(self.h, int(bool(enable))))

    def mppi_set_tiles(self, block=0, nchunk=0):
        self._check(self.lib.mppi_set_tiles(self.h, int(block), int(nchunk)))

    def mppi_set_profiling(self, enable=True):
        self._check(self.lib.mppi_set_profiling(self.h, int(bool(enable))))

    def mppi_get_profile(self):
        """(total ms, launch count) of the timed signed-distance launches."""
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(self.lib.mppi_get_profile(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def mppi_step(self, prm, q0, U, seed, step, diag=False, params=None):
        """One control cycle.  U (T, nu) device float32 is updated in place.
        diag: False, True (every diagnostic output) or a collection of
        MppiDiag field names (only those are produced).

        Returns (u_star ndarray, valid bool, diag dict or None).
        """
        p = params if params is not None else make_params(prm)
        if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.float32
                and U.is_contiguous()):
            raise TypeError("U must be a contiguous float32 CUDA tensor (updated in place)")
        K, T, nu = p.K, p.T, p.nu
        D = None
        out = None
        if diag:
            dev = self.device
            out = dict(d_min=torch.empty((K, T), device=dev),
                       argmin=torch.empty((K, T), dtype=torch.int32, device=dev),
                       J=torch.empty(K, device=dev), w=torch.empty(K, device=dev),
                       poses=torch.empty((K, T, 4), device=dev),
                       eps=torch.empty((K, T, nu), device=dev),
                       u=torch.empty((K, T, nu), device=dev),
                       U_upd=torch.empty((T, nu), device=dev),
                       d_nom=torch.full((T,), math.nan, device=dev),
                       J_nom=torch.full((1,), math.nan, device=dev))
            if diag is not True:
                out = {k: v for k, v in out.items() if k in set(diag)}
            D = MppiDiag(*[out[k].data_ptr() if k in out else None for k in MppiDiag.names()])
        # per-context argument buffers (a context serves one step at a time)
        q, u_out, valid = self._step_bufs
        q[0], q[1], q[2] = float(q0[0]), float(q0[1]), float(q0[2])
        self._check(self.lib.mppi_step(self.h, ctypes.byref(p), q, U.data_ptr(), int(seed), int(step),
                                       u_out, ctypes.byref(valid),
                                       ctypes.byref(D) if D is not None else None))
        return np.array(u_out[:nu], dtype=np.float32), bool(valid.value), out


def _scene_diag(lib, h, p, s, device, check):
    K, T, nu = p.K, p.T, p.nu
    out = dict(d_min=torch.empty((K, T), device=device), poses=torch.empty((K, T, 4), device=device),
               eps=torch.empty((K, T, nu), device=device), J=torch.empty(K, device=device),
               U_upd=torch.empty((T, nu), device=device), d_nom=torch.empty(T, device=device),
               J_nom=torch.empty(1, device=device))
    D = MppiDiag(*[out[k].data_ptr() if k in out else None for k in MppiDiag.names()])
    check(lib.mppi_batch_scene_diag(h, int(s), ctypes.byref(D)))
    return out


class Batch:
    """Batched step over several contexts (one scene each).

    The batch runs on its own (non-default) torch stream, which waits for the
    caller's current stream before every step.
    """

    def __init__(self, contexts, params_list):
        if len(contexts) != len(params_list) or not contexts:
            raise ValueError("one parameter set per context")
        self.lib = load()
        self.contexts = list(contexts)      # keep the contexts alive
        self.params = (MppiParams * len(contexts))(*[make_params(p) for p in params_list])
        self.n = len(contexts)
        self.device = contexts[0].device
        self.stream = torch.cuda.Stream(device=self.device)
        handles = (ctypes.c_void_p * self.n)(*[c.h.value for c in contexts])
        h = ctypes.c_void_p()
        rc = self.lib.mppi_batch_create(ctypes.byref(h), handles, self.params, self.n,
                                        ctypes.c_void_p(self.stream.cuda_stream))
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.mppi_batch_last_error(None).decode())
        self.h = h
        off = (ctypes.c_int * (self.n + 1))()
        self._check(self.lib.mppi_batch_u_offsets(self.h, off))
        self.u_offsets = list(off)

    def _check(self, rc):
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.mppi_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mppi_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mppi_batch_refresh(self):
        self._check(self.lib.mppi_batch_refresh(self.h))

    def mppi_batch_autotune(self, reps=3):
        w = ctypes.c_double()
        self._check(self.lib.mppi_batch_autotune(self.h, int(reps), ctypes.byref(w)))
        return w.value

    def mppi_batch_set_work(self, work_per_item=0.0):
        """Queue item size in point-primitive pairs (0: the default); re-plans."""
        self._check(self.lib.mppi_batch_set_work(self.h, float(work_per_item)))

    def mppi_batch_info(self):
        a, b, w = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_double()
        self._check(self.lib.mppi_batch_info(self.h, ctypes.byref(a), ctypes.byref(b),
                                             ctypes.byref(w)))
        return a.value, b.value, w.value

    def new_nominals(self):
        return torch.zeros(max(1, self.u_offsets[-1]), dtype=torch.float32, device=self.device)

    def nominal(self, U, s):
        p = self.params[s]
        return U[self.u_offsets[s]:self.u_offsets[s + 1]].view(p.T, p.nu)

    def mppi_step_batched(self, q0, U, seeds, steps, use_graph=True):
        """q0 (n, 3); U packed device nominals (updated in place); seeds, steps (n,).
        Returns (u_star (n, 3) ndarray, valid (n,) bool ndarray)."""
        q = np.ascontiguousarray(np.asarray(q0, dtype=np.float32).reshape(self.n, 3))
        sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(self.n))
        st = np.ascontiguousarray(np.asarray(steps, dtype=np.uint64).reshape(self.n))
        if not (U.is_cuda and U.dtype == torch.float32 and U.is_contiguous()):
            raise TypeError("U must be a contiguous float32 CUDA tensor")
        u_out = np.zeros((self.n, 3), dtype=np.float32)
        valid = np.zeros(self.n, dtype=np.int32)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        vp = ctypes.c_void_p
        self._check(self.lib.mppi_step_batched(
            self.h, q.ctypes.data_as(vp), _ptr(U), sd.ctypes.data_as(vp), st.ctypes.data_as(vp),
            u_out.ctypes.data_as(vp), valid.ctypes.data_as(vp), int(bool(use_graph))))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return u_out, valid.astype(bool)

    def set_profiling(self, enable=True):
        self._check(self.lib.mppi_batch_set_profiling(self.h, int(bool(enable))))

    def get_profile(self):
        """(total ms, timed eager steps) of the sampled-rollout distance pass."""
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(self.lib.mppi_batch_get_profile(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def scene_diag(self, s):
        """Diagnostics of scene s from the last step (see mppi_batch_scene_diag):
        dict of device tensors d_min (K, T), poses (K, T, 4), eps (K, T, nu),
        J (K,), U_upd (T, nu), d_nom (T,), J_nom (1,)."""
        return _scene_diag(self.lib, self.h, self.params[s], s, self.device, self._check)

    def nominal_costs(self):
        """J_nom of every scene from the last step (NaN where validation is off)."""
        J = np.zeros(self.n, dtype=np.float32)
        self._check(self.lib.mppi_batch_nominal_costs(self.h, J.ctypes.data_as(ctypes.c_void_p)))
        return J


class Hybrid:
    """Hybrid-mode cycle (Algorithm 2) over one context: one parameter set per
    motion mode.  Runs on its own torch stream, ordered after the caller's."""

    def __init__(self, context, mode_params):
        self.lib = load()
        self.context = context
        self.params = (MppiParams * len(mode_params))(*[make_params(p) for p in mode_params])
        self.n = len(mode_params)
        self.device = context.device
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        rc = self.lib.mppi_hybrid_create(ctypes.byref(h), context.h, self.params, self.n,
                                         ctypes.c_void_p(self.stream.cuda_stream))
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.mppi_hybrid_last_error(None).decode())
        self.h = h
        off = (ctypes.c_int * (self.n + 1))()
        rc = self.lib.mppi_batch_u_offsets(self.lib.mppi_hybrid_batch(self.h), off)
        self._check(rc)
        self.u_offsets = list(off)

    def _check(self, rc):
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.mppi_hybrid_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mppi_hybrid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_nominals(self):
        return torch.zeros(max(1, self.u_offsets[-1]), dtype=torch.float32, device=self.device)

    def autotune(self, reps=2):
        """Autotune the queue item size of the underlying batch (see
        mppi_batch_autotune); returns the chosen pairs per item."""
        w = ctypes.c_double()
        self._check(self.lib.mppi_batch_autotune(self.lib.mppi_hybrid_batch(self.h), int(reps),
                                                 ctypes.byref(w)))
        return w.value

    def nominal(self, U, m):
        p = self.params[m]
        return U[self.u_offsets[m]:self.u_offsets[m + 1]].view(p.T, p.nu)

    def mode_diag(self, m):
        """Diagnostics of mode m's Algorithm-1 cycle from the last hybrid step
        (the layout of Batch.scene_diag)."""
        return _scene_diag(self.lib, self.lib.mppi_hybrid_batch(self.h), self.params[m], m,
                           self.device, self._check)

    def step(self, q0, U, seed, step, hp, m_prev, tau_cool, use_graph=True):
        """One cycle.  hp: dict of mppi_hybrid_params fields.  U: packed per-mode
        nominals (updated in place).  Returns dict(u, mode, tau_cool, stopped,
        J (n,), valid (n,))."""
        if not (U.is_cuda and U.dtype == torch.float32 and U.is_contiguous()):
            raise TypeError("U must be a contiguous float32 CUDA tensor")
        hpar = HybridParams(float(hp.get("lambda_switch", 0.0)), int(hp.get("cool_max", 0)),
                            float(hp.get("v_min", 0.0)), float(hp.get("w_min", 0.0)),
                            float(hp.get("noise_v", 0.0)), float(hp.get("noise_w", 0.0)))
        q = (ctypes.c_float * 3)(*[float(v) for v in q0])
        m = ctypes.c_int(int(m_prev))
        tau = ctypes.c_int(int(tau_cool))
        stopped = ctypes.c_int(0)
        u = (ctypes.c_float * 3)()
        J = np.zeros(self.n, dtype=np.float32)
        valid = np.zeros(self.n, dtype=np.int32)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        vp = ctypes.c_void_p
        self._check(self.lib.mppi_hybrid_step(
            self.h, q, _ptr(U), int(seed), int(step), ctypes.byref(hpar), ctypes.byref(m),
            ctypes.byref(tau), u, ctypes.byref(stopped), J.ctypes.data_as(vp),
            valid.ctypes.data_as(vp), int(bool(use_graph))))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return dict(u=np.array(u[:], dtype=np.float32), mode=m.value, tau_cool=tau.value,
                    stopped=bool(stopped.value), J=J, valid=valid.astype(bool))


class Proposal:
    """Learned sampling proposal (MLP on the matrix cores), see exact_mppi.h."""

    BUFFERS = {"pre1": 0, "pre2": 1, "out": 2, "dout": 3, "dh2": 4, "dh1": 5, "grad": 6,
               "x": 10, "a1": 11, "a2": 12, "dout_b": 13, "dh2_b": 14, "dh1_b": 15}

    def __init__(self, T, nu, hidden=256, max_batch=1024, device=0, stream=None):
        self.lib = load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.lib.proposal_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream),
                                      int(T), int(nu), int(hidden), int(max_batch))
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.proposal_last_error(None).decode())
        self.h = h
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.proposal_shape(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        self.in_dim, self.hidden, self.out_dim = a.value, b.value, c.value
        self.T, self.nu = int(T), int(nu)
        self.n_params = int(self.lib.proposal_num_params(self.h))

    def _check(self, rc):
        if rc != MPPI_OK:
            raise MppiError(rc, self.lib.proposal_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.proposal_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_params(self, seed):
        """Glorot-uniform weights and zero biases drawn on the host from `seed`."""
        rng = np.random.default_rng(seed)
        parts = []
        for fi, fo in ((self.in_dim, self.hidden), (self.hidden, self.hidden),
                       (self.hidden, self.out_dim)):
            lim = math.sqrt(6.0 / (fi + fo))
            parts += [rng.uniform(-lim, lim, fi * fo), np.zeros(fo)]
        theta = np.concatenate(parts).astype(np.float32)
        self.set_params(theta)
        return theta

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(self.lib.proposal_set_params(self.h, a.ctypes.data_as(ctypes.c_void_p), a.size))

    def get_params(self):
        a = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.proposal_get_params(self.h, a.ctypes.data_as(ctypes.c_void_p), a.size))
        return a

    def set_scaling(self, prm, r_max=8.0):
        p = make_params(prm)
        self._check(self.lib.proposal_set_scaling(self.h, ctypes.byref(p), float(r_max)))

    def features(self, ctx, q0, U_prev):
        q0 = _dev_f32(q0, self.device, "q0").reshape(-1, 3).contiguous()
        U_prev = _dev_f32(U_prev, self.device, "U_prev").contiguous()
        M = q0.shape[0]
        out = torch.empty((M, self.in_dim), dtype=torch.float32, device=self.device)
        self._check(self.lib.proposal_features(self.h, ctx.h, _ptr(q0), _ptr(U_prev), M, _ptr(out)))
        return out

    def forward(self, feat):
        feat = _dev_f32(feat, self.device, "feat")
        out = torch.empty((feat.shape[0], self.out_dim), dtype=torch.float32, device=self.device)
        self._check(self.lib.proposal_forward(self.h, _ptr(feat), feat.shape[0], _ptr(out)))
        return out

    def mean(self, feat):
        feat = _dev_f32(feat, self.device, "feat")
        U = torch.empty((feat.shape[0], self.T, self.nu), dtype=torch.float32, device=self.device)
        self._check(self.lib.proposal_mean(self.h, _ptr(feat), feat.shape[0], _ptr(U)))
        return U

    def normalize(self, U, feat=None):
        """Training targets of the sequences U; feat (the same states'
        features) is needed in residual mode."""
        U = _dev_f32(U, self.device, "U")
        M = U.numel() // (self.T * self.nu)
        if feat is not None:
            feat = _dev_f32(feat, self.device, "feat")
        y = torch.empty((M, self.out_dim), dtype=torch.float32, device=self.device)
        self._check(self.lib.proposal_normalize(self.h, _ptr(U), _ptr(feat), M, _ptr(y)))
        return y

    def set_residual(self, scale):
        """0: outputs are sequences; > 0: corrections of the previous sequence."""
        self._check(self.lib.proposal_set_residual(self.h, float(scale)))

    def train_step(self, feat, target, lr, want_loss=True):
        feat = _dev_f32(feat, self.device, "feat")
        target = _dev_f32(target, self.device, "target")
        loss = ctypes.c_float()
        self._check(self.lib.proposal_train_step(self.h, _ptr(feat), _ptr(target), feat.shape[0],
                                                 float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def get_buffer(self, name, n):
        a = np.empty(int(n), dtype=np.float32)
        self._check(self.lib.proposal_get_buffer(self.h, self.BUFFERS[name],
                                                 a.ctypes.data_as(ctypes.c_void_p), a.size))
        return a

    def save(self, path):
        self._check(self.lib.proposal_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(self.lib.proposal_load(self.h, str(path).encode()))
