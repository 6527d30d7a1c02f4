"""ctypes binding of libxslam.so (include/xslam.h): argument marshalling only.

Every step of the frame runs in the library's HIP kernels; PyTorch provides the
device memory (one uint8 workspace tensor, input depth tensors) and the stream.
If the library is missing this module raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxslam.so")

# status codes
OK, WARN_TRACK_LOST = 0, 1
ERR_ARG, ERR_WORKSPACE, ERR_HIP, ERR_STATE, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
C64, C128 = 0, 1
# kernel classes of Slam.kernel_times()
TIMER_CLASSES = ("measure", "k_icp", "k_fuse", "k_raymarch", "other", "k_icp_finish", "k_rayhit", "k_brick_cull")
N_TIMER_CLASSES = len(TIMER_CLASSES)
(P_PHI_X, P_PHI_Y, P_PHI_Z, P_RHO_X, P_RHO_Y, P_RHO_Z, P_TRUNC, P_WCAP, P_DGATE, P_AGATE,
 P_ICPW0, P_ICPW1, P_ICPW2, P_FX, P_FY, P_CX, P_CY, P_DEPTH) = range(18)
(F_POSE, F_POSES, F_TSDF, F_WEIGHT, F_VMAP, F_NMAP, F_ZMAP, F_MVALID, F_MEAS_DEPTH, F_MEAS_V,
 F_MEAS_N, F_MEAS_VALID, F_COUNTERS, F_PREV_POSE, F_FRAME, F_SURF_V, F_SURF_N, F_SURF_R, F_SURF_C, F_SURF_T,
 F_SURF_COUNT) = range(21)
MAP_TSDF, MAP_SURFEL = 0, 1
N_COUNTERS = 40


class xslam_dir(C.Structure):
    _fields_ = [("param", C.c_int32), ("h", C.c_double)]


class xslam_pair(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32)]


class xslam_perturbation(C.Structure):
    _fields_ = [("n_dirs", C.c_int32), ("dirs", C.POINTER(xslam_dir)),
                ("n_pairs", C.c_int32), ("pairs", C.POINTER(xslam_pair))]


class xslam_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class xslam_volume(C.Structure):
    _fields_ = [("dim", C.c_int32 * 3), ("voxel", C.c_double), ("trunc", C.c_double), ("wcap", C.c_double)]


class xslam_icp(C.Structure):
    _fields_ = [("iters", C.c_int32 * 3), ("dgate", C.c_double), ("agate_deg", C.c_double),
                ("level_w", C.c_double * 3), ("disc_delta", C.c_double), ("init", C.c_int32),
                ("update", C.c_int32), ("solver", C.c_int32)]


class xslam_launch(C.Structure):
    _fields_ = [("ray_tile", C.c_int32 * 2), ("icp_blocks", C.c_int32 * 3), ("fuse_blocks", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class xslam_surfel(C.Structure):
    _fields_ = [("d_depth", C.c_double), ("d_norm_deg", C.c_double), ("d_dist", C.c_double), ("sigma", C.c_double),
                ("c_stable", C.c_double), ("capacity", C.c_int32)]


class xslam_config(C.Structure):
    _fields_ = [("prec", C.c_int32), ("cam", xslam_camera), ("vol", xslam_volume), ("icp", xslam_icp),
                ("bilateral_radius", C.c_int32), ("bilateral_sigma_px", C.c_double),
                ("bilateral_sigma_m", C.c_double), ("near_m", C.c_double), ("max_frames", C.c_int32),
                ("map", C.c_int32), ("surfel", xslam_surfel)]


_lib = None


def lib():
    """Load libxslam.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2405_02187_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
        cfgp, pertp = C.POINTER(xslam_config), C.POINTER(xslam_perturbation)
        sig = {
            "xslam_components": (C.c_int32, [pertp]),
            "xslam_workspace_bytes": (C.c_size_t, [cfgp, pertp]),
            "xslam_create": (C.c_int, [cfgp, pertp, vp, C.c_size_t, vp, dp, C.POINTER(vp)]),
            "xslam_measure": (C.c_int, [vp, vp, vp]),
            "xslam_integrate": (C.c_int, [vp, vp, vp, dp]),
            "xslam_raycast": (C.c_int, [vp, dp, vp, vp]),
            "xslam_track": (C.c_int, [vp, vp, vp, dp]),
            "xslam_step": (C.c_int, [vp, vp, vp, dp]),
            "xslam_icp_pass": (C.c_int, [vp, C.c_int32, dp]),
            "xslam_traj_err": (C.c_int, [vp, dp, C.c_int32, dp]),
            "xslam_icp_energy": (C.c_int, [vp, C.c_int32, C.c_int32, dp]),
            "xslam_reloc_energy": (C.c_int, [vp, dp, dp]),
            "xslam_get": (C.c_int, [vp, C.c_int32, vp, C.c_size_t]),
            "xslam_set": (C.c_int, [vp, C.c_int32, vp, C.c_size_t]),
            "xslam_set_timing": (C.c_int, [vp, C.c_int32]),
            "xslam_kernel_times": (C.c_int, [vp, dp, i64p]),
            "xslam_sync": (C.c_int, [vp]),
            "xslam_last_error": (C.c_char_p, [vp]),
            "xslam_destroy": (C.c_int, [vp]),
            "xslam_ctx_set_cnn": (C.c_int, [vp, vp]),
            "xslam_cnn_parts": (C.c_int, [vp, vp, vp]),
            "xslam_set_launch": (C.c_int, [vp, C.POINTER(xslam_launch)]),
            "xslam_get_launch": (C.c_int, [vp, C.POINTER(xslam_launch)]),
            "xslam_frame_graph": (C.c_int, [vp, C.POINTER(C.c_int32)]),
            "xslam_autotune": (C.c_int, [vp, C.c_int32, C.POINTER(xslam_launch), dp]),
            "xslam_batch_create": (C.c_int, [C.POINTER(vp), C.c_int32, C.POINTER(vp)]),
            "xslam_batch_create_grouped": (C.c_int, [C.POINTER(vp), C.c_int32, C.c_int32, C.POINTER(vp)]),
            "xslam_batch_step": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int32)]),
            "xslam_batch_latency": (C.c_int, [vp, C.POINTER(C.c_float)]),
            "xslam_batch_last_index": (C.c_int32, [vp]),
            "xslam_batch_destroy": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


EXPORTS_CORE = ["xslam_components", "xslam_workspace_bytes", "xslam_create", "xslam_measure", "xslam_integrate",
           "xslam_raycast", "xslam_track", "xslam_step", "xslam_icp_pass", "xslam_icp_energy", "xslam_reloc_energy", "xslam_traj_err", "xslam_get",
           "xslam_set", "xslam_set_timing", "xslam_kernel_times", "xslam_sync", "xslam_last_error",
           "xslam_destroy", "xslam_ctx_set_cnn", "xslam_cnn_parts", "xslam_set_launch", "xslam_get_launch",
           "xslam_autotune", "xslam_frame_graph", "xslam_batch_create", "xslam_batch_create_grouped", "xslam_batch_step", "xslam_batch_latency",
           "xslam_batch_last_index", "xslam_batch_destroy"]


class XslamError(RuntimeError):
    pass


# --------------------------------------------------------------------------
def make_config(prec=C64, width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5, dim=(512, 512, 512),
                voxel=0.01, trunc=0.06, wcap=64.0, iters=(10, 5, 4), dgate=0.1, agate_deg=20.0,
                level_w=(1.0, 1.0, 1.0), disc_delta=0.1, init=0, update=0, solver=0, bilateral_radius=3, sigma_px=4.5,
                sigma_m=0.03, near_m=0.1, max_frames=512, map=MAP_TSDF, surf_d_depth=0.03, surf_d_norm_deg=30.0,
                surf_d_dist=0.03, surf_sigma=0.015, surf_c_stable=0.0, surf_capacity=0) -> xslam_config:
    """surf_*: the surfel front end (map=MAP_SURFEL); capacity 0: 8 x the
    pixels of a frame."""
    c = xslam_config()
    c.prec = prec
    c.cam = xslam_camera(width, height, fx, fy, cx, cy)
    c.vol.dim[:] = list(dim)
    c.vol.voxel, c.vol.trunc, c.vol.wcap = voxel, trunc, wcap
    c.icp.iters[:] = list(iters)
    c.icp.dgate, c.icp.agate_deg = dgate, agate_deg
    c.icp.level_w[:] = list(level_w)
    c.icp.disc_delta, c.icp.init, c.icp.update, c.icp.solver = disc_delta, init, update, solver
    c.bilateral_radius, c.bilateral_sigma_px, c.bilateral_sigma_m = bilateral_radius, sigma_px, sigma_m
    c.near_m, c.max_frames = near_m, max_frames
    c.map = map
    c.surfel = xslam_surfel(surf_d_depth, surf_d_norm_deg, surf_d_dist, surf_sigma, surf_c_stable,
                            surf_capacity or 8 * width * height)
    return c


def config_from_preset(p: dict, prec=None, **kw) -> xslam_config:
    cam = p["camera"]
    args = dict(prec=(C128 if p["prec"] == "c128" else C64) if prec is None else prec,
                width=cam["width"], height=cam["height"], fx=cam["fx"], fy=cam["fy"], cx=cam["cx"], cy=cam["cy"],
                dim=(p["dim"],) * 3, voxel=p["voxel"], trunc=p["trunc"], wcap=p["wcap"],
                iters=tuple(p["icp"]["iters"]), dgate=p["icp"]["dgate"], agate_deg=p["icp"]["agate_deg"],
                max_frames=p["n_frames"])
    args.update(kw)
    return make_config(**args)


class Perturbation:
    """Directions [(param, h), ...] and Hessian size q (pairs over the first q)."""

    def __init__(self, dirs=(), q: int = 0):
        self.dirs = list(dirs)
        self.q = q
        self._d = (xslam_dir * max(1, len(self.dirs)))(*[xslam_dir(p, h) for p, h in self.dirs])
        pairs = [(a, b) for a in range(q) for b in range(a, q)]
        self._p = (xslam_pair * max(1, len(pairs)))(*[xslam_pair(a, b) for a, b in pairs])
        self.c = xslam_perturbation(len(self.dirs), self._d, len(pairs), self._p)

    @property
    def ncomp(self) -> int:
        return 1 + len(self.dirs) + self.q * (self.q + 1) // 2


def workspace_bytes(cfg: xslam_config, pert: Perturbation) -> int:
    return lib().xslam_workspace_bytes(C.byref(cfg), C.byref(pert.c))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Slam:
    """One context: workspace from torch, calls on torch's current stream."""

    def __init__(self, cfg: xslam_config, pert: Perturbation, T0, device="cuda:0"):
        import torch
        self.torch = torch
        self.cfg, self.pert = cfg, pert
        self.nc = pert.ncomp
        self.D, self.Q = len(pert.dirs), pert.q
        self.dtype = torch.float32 if cfg.prec == C64 else torch.float64
        self.np_dtype = np.float32 if cfg.prec == C64 else np.float64
        nbytes = workspace_bytes(cfg, pert)
        if nbytes == 0:
            raise XslamError("unsupported or invalid configuration / perturbation")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(device)
        T0 = np.ascontiguousarray(T0, dtype=np.float64).reshape(16)
        h = C.c_void_p()
        self._check(lib().xslam_create(C.byref(cfg), C.byref(pert.c), _ptr(self.ws), nbytes,
                                       C.c_void_p(self.stream.cuda_stream),
                                       T0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)), None)
        self.h = h
        W, H = cfg.cam.width, cfg.cam.height
        self.npx = [(W >> l) * (H >> l) for l in range(3)]
        self.nvox = cfg.vol.dim[0] * cfg.vol.dim[1] * cfg.vol.dim[2]

    def _check(self, rc, h="self", allow_warn=True):
        if rc < 0 or (rc > 0 and not allow_warn):
            msg = lib().xslam_last_error(self.h if h == "self" else None)
            raise XslamError(f"xslam error {rc}: {msg.decode() if msg else ''}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().xslam_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- calls -------------------------------------------------------------
    def _dd(self, depth_dot):
        return _ptr(depth_dot)

    def measure(self, depth, depth_dot=None):
        return self._check(lib().xslam_measure(self.h, _ptr(depth), self._dd(depth_dot)))

    def integrate(self, depth=None, depth_dot=None, pose=None):
        pp = None if pose is None else np.ascontiguousarray(pose, np.float64).reshape(16)
        return self._check(lib().xslam_integrate(self.h, _ptr(depth), self._dd(depth_dot),
                                                 None if pp is None else pp.ctypes.data_as(C.POINTER(C.c_double))))

    def raycast(self, pose=None):
        pp = None if pose is None else np.ascontiguousarray(pose, np.float64).reshape(16)
        return self._check(lib().xslam_raycast(self.h, None if pp is None else pp.ctypes.data_as(C.POINTER(C.c_double)),
                                               None, None))

    def track(self, depth=None, depth_dot=None, want_pose=True):
        """depth None: track the frame measured last (or set with set())."""
        out = np.zeros((self.nc, 16)) if want_pose else None
        rc = self._check(lib().xslam_track(self.h, None if depth is None else _ptr(depth), self._dd(depth_dot),
                                           None if out is None else out.ctypes.data_as(C.POINTER(C.c_double))))
        return rc, out

    def step(self, depth, depth_dot=None, want_pose=False):
        out = np.zeros((self.nc, 16)) if want_pose else None
        rc = self._check(lib().xslam_step(self.h, _ptr(depth), self._dd(depth_dot),
                                          None if out is None else out.ctypes.data_as(C.POINTER(C.c_double))))
        return rc, out

    def icp_pass(self, level):
        ns = 27 * self.nc + 2
        out = np.zeros(ns)
        self._check(lib().xslam_icp_pass(self.h, level, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out[:27 * self.nc].reshape(27, self.nc), out[27 * self.nc], out[27 * self.nc + 1]

    def icp_energy(self, level, through=False):
        """Newton objective of one ICP pass at the current pose, correspondences
        held fixed (or differentiated through the association): -> (E,
        gradient (6,), Hessian (6, 6), count)."""
        out = np.zeros(29)
        self._check(lib().xslam_icp_energy(self.h, int(level), int(bool(through)),
                                           out.ctypes.data_as(C.POINTER(C.c_double))))
        H = np.zeros((6, 6))
        iu = np.triu_indices(6)
        H[iu] = out[7:28]
        H = H + np.triu(H, 1).T
        return out[0], out[1:7].copy(), H, int(out[28])

    def reloc_energy(self, T):
        """Relocalisation objective at the camera-to-world pose T (4x4) against
        the context's volume, the last measured frame as the query: -> (E,
        gradient (6,), Hessian (6, 6), contributing voxels)."""
        T = np.ascontiguousarray(T, np.float64).reshape(16)
        out = np.zeros(29)
        self._check(lib().xslam_reloc_energy(self.h, T.ctypes.data_as(C.POINTER(C.c_double)),
                                             out.ctypes.data_as(C.POINTER(C.c_double))))
        H = np.zeros((6, 6))
        iu = np.triu_indices(6)
        H[iu] = out[7:28]
        H = H + np.triu(H, 1).T
        return out[0], out[1:7].copy(), H, int(out[28])

    def traj_err(self, gt):
        gt = np.ascontiguousarray(gt, np.float64).reshape(-1, 16)
        out = np.zeros(self.nc)
        self._check(lib().xslam_traj_err(self.h, gt.ctypes.data_as(C.POINTER(C.c_double)), len(gt),
                                         out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def sync(self):
        return self._check(lib().xslam_sync(self.h))

    def set_cnn(self, cnn):
        self._cnn = cnn
        return self._check(lib().xslam_ctx_set_cnn(self.h, None if cnn is None else cnn.h))

    def cnn_parts(self):
        """-> torch (1,60,80) depth channel and (4,60,80) model channels (device)."""
        W3, H3 = self.cfg.cam.width >> 3, self.cfg.cam.height >> 3
        d = self.torch.empty((1, H3, W3), dtype=self.torch.float32, device=self.ws.device)
        m = self.torch.empty((4, H3, W3), dtype=self.torch.float32, device=self.ws.device)
        self._check(lib().xslam_cnn_parts(self.h, C.c_void_p(d.data_ptr()), C.c_void_p(m.data_ptr())))
        return d, m

    def frame_graph(self) -> bool:
        """True if tracked frames replay the captured frame graph."""
        v = C.c_int32(0)
        self._check(lib().xslam_frame_graph(self.h, C.byref(v)))
        return bool(v.value)

    def get_launch(self) -> dict:
        lc = xslam_launch()
        self._check(lib().xslam_get_launch(self.h, C.byref(lc)))
        return dict(ray_tile=tuple(lc.ray_tile), icp_blocks=tuple(lc.icp_blocks), fuse_blocks=lc.fuse_blocks)

    def set_launch(self, ray_tile=None, icp_blocks=None, fuse_blocks=None):
        cur = self.get_launch()
        lc = xslam_launch()
        lc.ray_tile[:] = list(ray_tile or cur["ray_tile"])
        lc.icp_blocks[:] = list(icp_blocks or cur["icp_blocks"])
        lc.fuse_blocks = int(fuse_blocks or cur["fuse_blocks"])
        return self._check(lib().xslam_set_launch(self.h, C.byref(lc)))

    def autotune(self, reps=20):
        """Time candidate raycast tiles and ICP grids on the current state; keeps
        the fastest.  -> (shapes dict, ms of raycast and ICP levels 0, 1, 2)."""
        lc = xslam_launch()
        ms = np.zeros(4)
        self._check(lib().xslam_autotune(self.h, int(reps), C.byref(lc), ms.ctypes.data_as(C.POINTER(C.c_double))))
        return self.get_launch(), ms

    def set_timing(self, on=True):
        return self._check(lib().xslam_set_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        ms = np.zeros(N_TIMER_CLASSES)
        n = np.zeros(N_TIMER_CLASSES, dtype=np.int64)
        self._check(lib().xslam_kernel_times(self.h, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                             n.ctypes.data_as(C.POINTER(C.c_int64))))
        return ms, n

    # ---- state -------------------------------------------------------------
    def _field_shape(self, field):
        nc, n0 = self.nc, self.npx[0]
        tot = sum(self.npx)
        fl = self.np_dtype
        if field in (F_POSE, F_PREV_POSE):
            return (nc, 4, 4), np.float64
        if field == F_POSES:
            return (self.frame(), nc, 4, 4), np.float64
        if field in (F_TSDF, F_WEIGHT):
            return (nc, self.nvox), fl
        if field in (F_VMAP, F_NMAP):
            return (3, nc, n0), fl
        if field == F_ZMAP:
            return (n0,), fl
        if field == F_MVALID:
            return (n0,), np.uint8
        if field == F_MEAS_DEPTH:
            return (nc * tot,), fl
        if field in (F_MEAS_V, F_MEAS_N):
            return (3 * nc * tot,), fl
        if field == F_MEAS_VALID:
            return (tot,), np.uint8
        if field == F_COUNTERS:
            return (min(self.frame(), self.cfg.max_frames), N_COUNTERS), np.int32
        cap = self.cfg.surfel.capacity
        if field in (F_SURF_V, F_SURF_N):
            return (3, nc, cap), fl
        if field in (F_SURF_R, F_SURF_C):
            return (nc, cap), fl
        if field == F_SURF_T:
            return (cap,), np.int32
        if field == F_SURF_COUNT:
            return (1,), np.int32
        raise ValueError(field)

    def frame(self):
        v = np.zeros(1, np.int32)
        self._check(lib().xslam_get(self.h, F_FRAME, v.ctypes.data_as(C.c_void_p), 4))
        return int(v[0])

    def get(self, field):
        shape, dt = self._field_shape(field)
        out = np.zeros(shape, dtype=dt)
        self._check(lib().xslam_get(self.h, field, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def set(self, field, value):
        shape, dt = self._field_shape(field)
        if field in (F_POSES, F_COUNTERS):       # any number of history rows
            shape = (-1,) + shape[1:]
        v = np.ascontiguousarray(value, dtype=dt).reshape(shape)
        self._check(lib().xslam_set(self.h, field, v.ctypes.data_as(C.c_void_p), v.nbytes))

    STATE_FIELDS = (F_TSDF, F_WEIGHT, F_VMAP, F_NMAP, F_ZMAP, F_MVALID, F_POSE, F_PREV_POSE, F_POSES, F_COUNTERS)

    def save_state(self) -> dict:
        """Host copy of everything later frame steps read (checkpoint)."""
        st = {f: self.get(f) for f in self.STATE_FIELDS}
        st[F_FRAME] = self.frame()
        if self.cfg.map == MAP_SURFEL:
            st["surfels"] = self.surfels()
        return st

    def load_state(self, st: dict) -> None:
        """Resume from a checkpoint taken with save_state on a context of the
        same configuration and perturbation."""
        for f in self.STATE_FIELDS:
            self.set(f, st[f])
        if "surfels" in st:
            self.set_surfels(st["surfels"])
        self.set_frame(st[F_FRAME])

    def set_frame(self, k):
        v = np.array([k], np.int32)
        self._check(lib().xslam_set(self.h, F_FRAME, v.ctypes.data_as(C.c_void_p), 4))

    def surfels(self) -> dict:
        """The surfel map (map = MAP_SURFEL): dict(v (m, 3, nc), n, r (m, nc),
        c, t (m,)) over the m surfels in use."""
        m = int(self.get(F_SURF_COUNT)[0])
        V, N = self.get(F_SURF_V), self.get(F_SURF_N)
        return dict(v=np.transpose(V[:, :, :m], (2, 0, 1)), n=np.transpose(N[:, :, :m], (2, 0, 1)),
                    r=self.get(F_SURF_R)[:, :m].T, c=self.get(F_SURF_C)[:, :m].T, t=self.get(F_SURF_T)[:m])

    def set_surfels(self, S: dict) -> None:
        """Load a surfel map (as returned by ``surfels``)."""
        m = len(S["t"])
        self.set_raw(F_SURF_V, np.ascontiguousarray(np.transpose(S["v"], (1, 2, 0)), dtype=self.np_dtype))
        self.set_raw(F_SURF_N, np.ascontiguousarray(np.transpose(S["n"], (1, 2, 0)), dtype=self.np_dtype))
        self.set_raw(F_SURF_R, np.ascontiguousarray(np.asarray(S["r"]).T, dtype=self.np_dtype))
        self.set_raw(F_SURF_C, np.ascontiguousarray(np.asarray(S["c"]).T, dtype=self.np_dtype))
        self.set_raw(F_SURF_T, np.ascontiguousarray(S["t"], dtype=np.int32))
        self.set(F_SURF_COUNT, np.array([m], np.int32))

    def set_raw(self, field, value: np.ndarray) -> None:
        """xslam_set with the buffer as given (its size decides what is written)."""
        v = np.ascontiguousarray(value)
        self._check(lib().xslam_set(self.h, field, v.ctypes.data_as(C.c_void_p), v.nbytes))

    def measured(self):
        """-> per level dict(D (nc,H,W), V (3,nc,H,W), N, valid (H,W))."""
        W, H = self.cfg.cam.width, self.cfg.cam.height
        D = self.get(F_MEAS_DEPTH)
        V = self.get(F_MEAS_V)
        N = self.get(F_MEAS_N)
        M = self.get(F_MEAS_VALID)
        out, o1, o3 = [], 0, 0
        for l in range(3):
            n, h, w = self.npx[l], H >> l, W >> l
            out.append(dict(D=D[o1 * self.nc:(o1 + n) * self.nc].reshape(self.nc, h, w),
                            V=V[o3 * self.nc:(o3 + 3 * n) * self.nc].reshape(3, self.nc, h, w),
                            N=N[o3 * self.nc:(o3 + 3 * n) * self.nc].reshape(3, self.nc, h, w),
                            valid=M[o1:o1 + n].reshape(h, w)))
            o1 += n
            o3 += 3 * n
        return out


# --------------------------------------------------------------------------
# learned ICP initialiser
# --------------------------------------------------------------------------
CNN_EXPORTS = ["xslam_cnn_param_count", "xslam_cnn_workspace_bytes", "xslam_cnn_create", "xslam_cnn_set_weights",
               "xslam_cnn_get_weights", "xslam_cnn_get_grads", "xslam_cnn_forward", "xslam_cnn_forward_noalloc",
               "xslam_cnn_train_step",
               "xslam_cnn_last_error", "xslam_cnn_destroy"]


def _cnn_lib():
    L = lib()
    if not getattr(L, "_cnn_sig", False):
        vp, fp = C.c_void_p, C.POINTER(C.c_float)
        sig = {
            "xslam_cnn_param_count": (C.c_int32, []),
            "xslam_cnn_workspace_bytes": (C.c_size_t, [C.c_int32]),
            "xslam_cnn_create": (C.c_int, [vp, C.c_size_t, vp, C.c_int32, C.POINTER(vp)]),
            "xslam_cnn_set_weights": (C.c_int, [vp, fp, C.c_size_t]),
            "xslam_cnn_get_weights": (C.c_int, [vp, fp, C.c_size_t]),
            "xslam_cnn_get_grads": (C.c_int, [vp, fp, C.c_size_t]),
            "xslam_cnn_forward": (C.c_int, [vp, vp, C.c_int32, vp]),
            "xslam_cnn_forward_noalloc": (C.c_int, [vp, vp, C.c_int32, vp]),
            "xslam_cnn_train_step": (C.c_int, [vp, vp, vp, C.c_int32, C.c_float, fp]),
            "xslam_cnn_last_error": (C.c_char_p, [vp]),
            "xslam_cnn_destroy": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        L._cnn_sig = True
    return L


class Batch:
    """Independent contexts advanced together, one frame each per step (each on
    the stream it was created with).  grouped=True: contexts of one shape are
    stepped by grouped launches (they must share a stream); persist is the
    number of workgroups per grouped launch (0: one per work item)."""

    def __init__(self, slams, grouped: bool = False, persist: int = 0):
        self.slams = list(slams)
        n = len(self.slams)
        arr = (C.c_void_p * n)(*[s.h for s in self.slams])
        h = C.c_void_p()
        if grouped:
            rc = lib().xslam_batch_create_grouped(arr, n, persist, C.byref(h))
        else:
            rc = lib().xslam_batch_create(arr, n, C.byref(h))
        if rc != 0:
            msgs = "; ".join(lib().xslam_last_error(s.h).decode() for s in self.slams if lib().xslam_last_error(s.h))
            raise XslamError(f"xslam_batch_create{'_grouped' if grouped else ''}: error {rc}: {msgs}")
        self.h = h
        self.n = n

    def step(self, depths, depth_dots=None, active=None):
        """depths / depth_dots: per context a device tensor or None."""
        n = self.n
        d = (C.c_void_p * n)(*[None if x is None else x.data_ptr() for x in depths])
        dd = None
        if depth_dots is not None:
            dd = (C.c_void_p * n)(*[None if x is None else x.data_ptr() for x in depth_dots])
        act = None if active is None else (C.c_int32 * n)(*[1 if a else 0 for a in active])
        rc = lib().xslam_batch_step(self.h, d, dd, act)
        if rc < 0:
            i = lib().xslam_batch_last_index(self.h)
            msg = lib().xslam_last_error(self.slams[i].h) if i >= 0 else b""
            raise XslamError(f"batch step: context {i}: error {rc}: {msg.decode() if msg else ''}")
        return rc

    def latency(self):
        ms = np.zeros(self.n, dtype=np.float32)
        rc = lib().xslam_batch_latency(self.h, ms.ctypes.data_as(C.POINTER(C.c_float)))
        if rc != 0:
            raise XslamError(f"batch latency: error {rc}")
        return ms

    def close(self):
        if getattr(self, "h", None):
            lib().xslam_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cnn:
    """The initialiser network on one device (workspace from torch)."""

    def __init__(self, max_batch=256, device="cuda:0"):
        import torch
        self.torch = torch
        L = _cnn_lib()
        self.n_params = L.xslam_cnn_param_count()
        nbytes = L.xslam_cnn_workspace_bytes(max_batch)
        if nbytes == 0:
            raise XslamError("invalid batch size")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = L.xslam_cnn_create(C.c_void_p(self.ws.data_ptr()), nbytes, C.c_void_p(self.stream.cuda_stream),
                                max_batch, C.byref(h))
        if rc != 0:
            raise XslamError(f"xslam_cnn_create: {rc}")
        self.h = h
        self.max_batch = max_batch

    def _chk(self, rc):
        if rc != 0:
            raise XslamError(f"cnn error {rc}: {_cnn_lib().xslam_cnn_last_error(self.h)}")

    def set_weights(self, flat):
        w = np.ascontiguousarray(flat, dtype=np.float32)
        self._chk(_cnn_lib().xslam_cnn_set_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def get_weights(self):
        w = np.zeros(self.n_params, np.float32)
        self._chk(_cnn_lib().xslam_cnn_get_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))
        return w

    def get_grads(self):
        w = np.zeros(self.n_params, np.float32)
        self._chk(_cnn_lib().xslam_cnn_get_grads(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))
        return w

    def forward(self, x):
        """x: torch float32 (n,5,60,80) on the device -> torch (n,6)."""
        out = self.torch.empty((x.shape[0], 6), dtype=self.torch.float32, device=x.device)
        self._chk(_cnn_lib().xslam_cnn_forward(self.h, C.c_void_p(x.data_ptr()), x.shape[0], C.c_void_p(out.data_ptr())))
        return out

    def forward_noalloc(self, x, out):
        """xslam_cnn_forward_noalloc: x (n,5,60,80), out (n,6) float32 device
        tensors, n <= 32; the activations live in the library's fixed array."""
        return self._chk(_cnn_lib().xslam_cnn_forward_noalloc(self.h, C.c_void_p(x.data_ptr()), x.shape[0],
                                                               C.c_void_p(out.data_ptr())))

    def train_step(self, x, label, lr=1e-3, want_loss=True):
        loss = C.c_float(0)
        self._chk(_cnn_lib().xslam_cnn_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(label.data_ptr()),
                                                  x.shape[0], lr, C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "h", None):
            _cnn_lib().xslam_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


EXPORTS = EXPORTS_CORE + CNN_EXPORTS
