"""CPU oracle for the CSFD dense-SLAM frame step -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's ``cpu_baseline`` leg may
import this package.  The product path (the HIP library and its binding) never
touches it, and the two share no code.

The oracle is ``xslam_oracle.cpp`` (plain C++17 loops over one scalar type:
real, full ``std::complex<double>`` or bicomplex), built by :func:`build` into
``liboracle.so`` and called through ctypes.  Scalars cross the interface as
``ncomp`` doubles: 1 (real), 2 (re, im) or 4 (re, i1, i2, i1i2).

Parity pins live in ``tests/test_oracle_*.py``.  Parts without an independent
pin are marked "parity unpinned" there and in the design notes: the bilateral
and pyramid constants, the raycast march schedule and the discontinuity
threshold (pinned only by special cases).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "xslam_oracle.cpp")
LIB = os.path.join(_HERE, "liboracle.so")

# parameter ids (the perturbation targets)
P_PHI_X, P_PHI_Y, P_PHI_Z, P_RHO_X, P_RHO_Y, P_RHO_Z = range(6)
P_TRUNC, P_WCAP, P_DGATE, P_AGATE, P_ICPW0, P_ICPW1, P_ICPW2 = range(6, 13)
P_FX, P_FY, P_CX, P_CY, P_DEPTH = range(13, 18)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class OrcConfig(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("dim", C.c_int32 * 3), ("voxel", C.c_double), ("trunc", C.c_double), ("wcap", C.c_double),
                ("iters", C.c_int32 * 3), ("dgate", C.c_double), ("agate_deg", C.c_double),
                ("level_w", C.c_double * 3), ("disc_delta", C.c_double),
                ("bilateral_radius", C.c_int32), ("sigma_px", C.c_double), ("sigma_m", C.c_double),
                ("near_m", C.c_double), ("init", C.c_int32), ("update", C.c_int32), ("solver", C.c_int32),
                ("pf_d_depth", C.c_double), ("pf_d_norm_deg", C.c_double), ("pf_d_dist", C.c_double),
                ("pf_sigma", C.c_double), ("pf_c_stable", C.c_double), ("pf_capacity", C.c_int32)]


class OrcSeed(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pa", C.c_int32), ("pb", C.c_int32), ("h", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        i64 = C.POINTER(C.c_int64)
        i32 = C.POINTER(C.c_int32)
        cp, sp = C.POINTER(OrcConfig), C.POINTER(OrcSeed)
        L.orc_se3_exp.argtypes = [sp, dp, dp]
        L.orc_measure.argtypes = [cp, sp, dp, dp, dp, dp, dp, u8]
        L.orc_icp_reduce.argtypes = [cp, sp, C.c_int, dp, dp, u8, dp, dp, dp, u8, dp, dp, dp, dp, i64, dp]
        L.orc_solve.argtypes = [sp, dp, dp, dp, dp]
        L.orc_solve.restype = C.c_int
        L.orc_fuse.argtypes = [cp, sp, dp, dp, dp, dp, i64, C.c_int64]
        L.orc_fuse.restype = C.c_int64
        L.orc_raycast.argtypes = [cp, sp, dp, dp, dp, i32, C.c_int32, dp, dp, dp, u8, dp, dp]
        L.orc_track.argtypes = [cp, sp, dp, dp, dp, dp, dp, u8, dp, dp, dp, i64, dp]
        L.orc_track.restype = C.c_int
        L.orc_run_sequence.argtypes = [cp, sp, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_traj_err.argtypes = [sp, C.c_int, dp, dp, dp]
        L.orc_const_vel.argtypes = [sp, dp, dp, C.c_int32, dp]
        L.orc_small_angle_update.argtypes = [sp, dp, dp, dp]
        L.orc_icp_energy.argtypes = [cp, C.c_int, dp, dp, u8, dp, dp, dp, u8, dp, dp, C.c_int, C.c_int, dp]
        L.orc_reloc_energy.argtypes = [cp, dp, dp, dp, dp, C.c_int, dp]
        L.orc_frame_step.argtypes = [cp, sp, C.c_int32, dp, dp, dp, dp, dp, dp, dp, u8, dp, dp, i32, dp, u8]
        L.orc_pf_frame_step.argtypes = [cp, sp, C.c_int32, dp, dp, dp, dp, dp, dp, i32, i64, dp, dp, dp, u8, dp, dp,
                                        i32, dp, i64]
        L.orc_pf_run_sequence.argtypes = [cp, sp, C.c_int32, dp, dp, dp, dp, dp, i64, dp, dp, dp, dp, i32, i64]
        L.orc_pf_index_map.argtypes = [cp, dp, dp, C.c_int64, dp, C.c_int32, C.c_double, i64]
        fp = C.POINTER(C.c_float)
        L.orc_cnn_parts.argtypes = [cp, dp, dp, dp, u8, dp, fp, fp]
        L.orc_raycast_footprint.argtypes = [cp, sp, dp, dp, dp, u8]
        L.orc_raycast_footprint.restype = C.c_int64
        L.orc_fuse_margin.argtypes = [cp, sp, dp, dp, i64, C.c_int64, dp]
        L.orc_eval_f.argtypes = [sp, C.c_double, dp]
        L.orc_eval_g.argtypes = [sp, C.c_double, C.c_double, C.c_int, C.c_int, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads(1)
        _lib = L
    return _lib


# --------------------------------------------------------------------------
def config(p: dict | None = None, **kw) -> OrcConfig:
    """Build an OrcConfig from a scenegen preset dict (and keyword overrides)."""
    d = dict(width=160, height=120, fx=130.0, fy=130.0, cx=79.5, cy=59.5, dim=(128, 128, 128),
             voxel=0.02, trunc=0.06, wcap=64.0, iters=(10, 5, 4), dgate=0.1, agate_deg=20.0,
             level_w=(1.0, 1.0, 1.0), disc_delta=0.1, bilateral_radius=3, sigma_px=4.5,
             sigma_m=0.03, near_m=0.1, init=0, update=0, solver=0, pf_d_depth=0.03, pf_d_norm_deg=30.0,
             pf_d_dist=0.03, pf_sigma=0.015, pf_c_stable=0.0, pf_capacity=0)
    if p is not None:
        cam = p["camera"]
        d.update(width=cam["width"], height=cam["height"], fx=cam["fx"], fy=cam["fy"],
                 cx=cam["cx"], cy=cam["cy"], dim=(p["dim"],) * 3, voxel=p["voxel"],
                 trunc=p["trunc"], wcap=p["wcap"], iters=tuple(p["icp"]["iters"]),
                 dgate=p["icp"]["dgate"], agate_deg=p["icp"]["agate_deg"])
    d.update(kw)
    if not d["pf_capacity"]:
        d["pf_capacity"] = 8 * d["width"] * d["height"]
    c = OrcConfig()
    for k, v in d.items():
        if k in ("dim", "iters", "level_w"):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, k, v)
    return c


def seed(kind: int = 0, pa: int = -1, pb: int = -1, h: float = 1e-20) -> OrcSeed:
    return OrcSeed(kind, pa, pb, h)


def ncomp(s: OrcSeed) -> int:
    return {0: 1, 1: 2, 2: 4}[s.kind]


def _p(a, dtype=C.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(dtype))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def lift(x, s: OrcSeed) -> np.ndarray:
    """Real array -> scalars with zero imaginary parts (trailing ncomp axis)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape + (ncomp(s),))
    out[..., 0] = x
    return out


# --------------------------------------------------------------------------
def se3_exp(s: OrcSeed, xi) -> np.ndarray:
    xi = _f64(xi)
    out = np.zeros((4, 4, ncomp(s)))
    lib().orc_se3_exp(C.byref(s), _p(xi), _p(out))
    return out


def measure(c: OrcConfig, s: OrcSeed, depth, depth_dot=None):
    """-> list of 3 levels: dict(D (H,W,nc), V (H,W,3,nc), N, valid (H,W) uint8)."""
    nc = ncomp(s)
    W, H = c.width, c.height
    sizes = [(H >> l, W >> l) for l in range(3)]
    tot = sum(h * w for h, w in sizes)
    D = np.zeros((tot, nc)); V = np.zeros((tot, 3, nc)); N = np.zeros((tot, 3, nc))
    valid = np.zeros(tot, dtype=np.uint8)
    lib().orc_measure(C.byref(c), C.byref(s), _p(_f64(depth)), _p(_f64(depth_dot)), _p(D), _p(V), _p(N),
                      _p(valid, C.c_uint8))
    out, off = [], 0
    for h, w in sizes:
        n = h * w
        out.append(dict(D=D[off:off + n].reshape(h, w, nc), V=V[off:off + n].reshape(h, w, 3, nc),
                        N=N[off:off + n].reshape(h, w, 3, nc), valid=valid[off:off + n].reshape(h, w)))
        off += n
    return out


def icp_reduce(c, s, level, cur, model, Tprev, T):
    nc = ncomp(s)
    A = np.zeros((21, nc)); b = np.zeros((6, nc))
    cnt = C.c_int64(0); r2 = C.c_double(0)
    lib().orc_icp_reduce(C.byref(c), C.byref(s), level, _p(_f64(cur["V"])), _p(_f64(cur["N"])),
                         _p(np.ascontiguousarray(cur["valid"], np.uint8), C.c_uint8),
                         _p(_f64(model["V"])), _p(_f64(model["N"])), _p(_f64(model["Z"])),
                         _p(np.ascontiguousarray(model["valid"], np.uint8), C.c_uint8),
                         _p(_f64(Tprev)), _p(_f64(T)), _p(A), _p(b), C.byref(cnt), C.byref(r2))
    return A, b, cnt.value, r2.value


def solve(s, A, b, w=None):
    nc = ncomp(s)
    w = lift(1.0, s) if w is None else _f64(w)
    delta = np.zeros((6, nc))
    lost = lib().orc_solve(C.byref(s), _p(_f64(A)), _p(_f64(b)), _p(w), _p(delta))
    return delta, lost


def fuse(c, s, F, W, Df, T, idx=None):
    """In-place-free fusion: returns (F, W, n_updated).  F, W: (N, nc) for the
    whole volume (x-fastest) or for the listed voxels when ``idx`` is given."""
    F = np.array(F, dtype=np.float64, copy=True, order="C")
    W = np.array(W, dtype=np.float64, copy=True, order="C")
    idx_a = None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    n = lib().orc_fuse(C.byref(c), C.byref(s), _p(F), _p(W), _p(_f64(Df)), _p(_f64(T)),
                       _p(idx_a, C.c_int64), 0 if idx_a is None else len(idx_a))
    return F, W, n


def raycast(c, s, F, W, T, pix=None, sched_pose=None, sched_params=None):
    nc = ncomp(s)
    npx = c.width * c.height if pix is None else len(pix)
    V = np.zeros((npx, 3, nc)); N = np.zeros((npx, 3, nc)); Z = np.zeros(npx)
    valid = np.zeros(npx, dtype=np.uint8)
    pix_a = None if pix is None else np.ascontiguousarray(pix, dtype=np.int32)
    lib().orc_raycast(C.byref(c), C.byref(s), _p(_f64(F)), _p(_f64(W)), _p(_f64(T)),
                      _p(pix_a, C.c_int32), 0 if pix_a is None else len(pix_a),
                      _p(V), _p(N), _p(Z), _p(valid, C.c_uint8), _p(_f64(sched_pose)), _p(_f64(sched_params)))
    if pix is None:
        H, Wd = c.height, c.width
        return dict(V=V.reshape(H, Wd, 3, nc), N=N.reshape(H, Wd, 3, nc), Z=Z.reshape(H, Wd),
                    valid=valid.reshape(H, Wd))
    return dict(V=V, N=N, Z=Z, valid=valid)


def track(c, s, depth, depth_dot, model0, Tprev, Tinit):
    _check_solver(c, s)
    nc = ncomp(s)
    Tout = np.zeros((4, 4, nc))
    cnt = C.c_int64(0); r2 = C.c_double(0)
    lost = lib().orc_track(C.byref(c), C.byref(s), _p(_f64(depth)), _p(_f64(depth_dot)),
                           _p(_f64(model0["V"])), _p(_f64(model0["N"])), _p(_f64(model0["Z"])),
                           _p(np.ascontiguousarray(model0["valid"], np.uint8), C.c_uint8),
                           _p(_f64(Tprev)), _p(_f64(Tinit)), _p(Tout), C.byref(cnt), C.byref(r2))
    return Tout, lost, cnt.value, r2.value


def _check_solver(c, s):
    if c.solver >= 1 and s.kind != 0:
        raise ValueError("the Newton solver (solver=1) runs on real seeds only")


def run_sequence(c, s, depths, T0, depth_dots=None, want_volume=False, sched_poses=None,
                 sched_params=None):
    """-> dict(poses (n,4,4,nc), stats (n,6), F, W (N,nc) if want_volume)."""
    _check_solver(c, s)
    nc = ncomp(s)
    depths = _f64(depths)
    n = depths.shape[0]
    poses = np.zeros((n, 4, 4, nc))
    stats = np.zeros((n, 6))
    nv = c.dim[0] * c.dim[1] * c.dim[2]
    F = np.zeros((nv, nc)) if want_volume else None
    W = np.zeros((nv, nc)) if want_volume else None
    lib().orc_run_sequence(C.byref(c), C.byref(s), n, _p(depths), _p(_f64(depth_dots)), _p(_f64(T0)),
                           _p(poses), _p(stats), _p(F), _p(W), _p(_f64(sched_poses)),
                           _p(_f64(sched_params)))
    out = dict(poses=poses, stats=stats)
    if want_volume:
        out.update(F=F, W=W)
    return out


def traj_err(s, poses, gt):
    out = np.zeros(ncomp(s))
    poses = _f64(poses)
    lib().orc_traj_err(C.byref(s), poses.shape[0], _p(poses), _p(_f64(gt)), _p(out))
    return out


def const_vel(s: OrcSeed, T1, T2, both_tracked: bool = True) -> np.ndarray:
    """Constant-velocity initial estimate from the poses of the last two frames
    (arrays (4,4,nc)); T1 when not both were tracked."""
    out = np.zeros((4, 4, ncomp(s)))
    lib().orc_const_vel(C.byref(s), _p(_f64(T1)), _p(_f64(T2)), int(bool(both_tracked)), _p(out))
    return out


def icp_energy(c: OrcConfig, level: int, cur, model, Tprev, T, order: int = 2, through: bool = False):
    """Newton ICP objective of one pass (real run): E = sum r^2 at pose T (4x4
    real), its gradient g (6) and Hessian H (6x6) in the left increment, and
    the correspondence count, with the correspondences held fixed (the
    objective of one ICP pass) or, ``through``, differentiated through the
    projective association.  cur/model: maps of that level with one
    component (as from measure/raycast with a real seed, or lifted).  order
    0 / 1 skips the Hessian / both derivatives (returned as 0)."""
    out = np.zeros(29)
    f = lambda a: _f64(np.asarray(a)[..., :1] if np.asarray(a).ndim >= 3 else a)  # noqa: E731
    lib().orc_icp_energy(C.byref(c), int(level), _p(f(cur["V"])), _p(f(cur["N"])),
                         _p(np.ascontiguousarray(cur["valid"], np.uint8), C.c_uint8),
                         _p(f(model["V"])), _p(f(model["N"])), _p(_f64(model["Z"])),
                         _p(np.ascontiguousarray(model["valid"], np.uint8), C.c_uint8),
                         _p(_f64(np.asarray(Tprev)[..., 0] if np.asarray(Tprev).ndim == 3 else Tprev)),
                         _p(_f64(np.asarray(T)[..., 0] if np.asarray(T).ndim == 3 else T)), int(bool(through)),
                         int(order), _p(out))
    H = np.zeros((6, 6))
    iu = np.triu_indices(6)
    H[iu] = out[7:28]
    H = H + np.triu(H, 1).T
    return out[0], out[1:7].copy(), H, int(out[28])


def reloc_energy(c: OrcConfig, F, W, Df, T, order: int = 2):
    """Relocalisation objective (Sec. 5.2): E(T) = sum over the voxels of
    (F_r - F_q)^2, F_q the reference volume (F, W: real, (N,) or (N, nc),
    x-fastest) after fusing the query's filtered level-0 depth Df (H, W) at
    the real pose T (4x4), with its gradient g (6) and Hessian H (6x6) in the
    left increment exp(delta) T (6 complex-step and 21 bicomplex evaluations),
    and the number of contributing voxels.  order 0 / 1 skips the Hessian /
    both derivatives (returned as 0)."""
    F = np.asarray(F)
    W = np.asarray(W)
    f = lambda a: _f64(a[:, 0] if a.ndim == 2 else a)  # noqa: E731
    Df = np.asarray(Df)
    Df = Df[..., 0] if Df.ndim == 3 else Df
    out = np.zeros(29)
    lib().orc_reloc_energy(C.byref(c), _p(f(F)), _p(f(W)), _p(_f64(Df)),
                           _p(_f64(np.asarray(T)[..., 0] if np.asarray(T).ndim == 3 else T)), int(order), _p(out))
    H = np.zeros((6, 6))
    iu = np.triu_indices(6)
    H[iu] = out[7:28]
    H = H + np.triu(H, 1).T
    return out[0], out[1:7].copy(), H, int(out[28])


def small_angle_update(s: OrcSeed, xi, T) -> np.ndarray:
    """The original KinectFusion pose update: small-angle transform of the
    increment xi (6, nc) composed with T (4, 4, nc), rotation re-orthonormalised."""
    out = np.zeros((4, 4, ncomp(s)))
    lib().orc_small_angle_update(C.byref(s), _p(_f64(xi)), _p(_f64(T)), _p(out))
    return out


class State:
    """The state one frame step reads and writes (for state-loaded steps):
    volume F, W (N, nc) x-fastest; level-0 model maps of the previous frame
    (V, N (H, W, 3, nc), Z, valid (H, W)); poses of the last two frames T1, T2
    (4, 4, nc); lost flags of the last two frames; the next frame's index."""

    def __init__(self, c: OrcConfig, s: OrcSeed, T0=None):
        nc = ncomp(s)
        nv = c.dim[0] * c.dim[1] * c.dim[2]
        H, W = c.height, c.width
        self.F = np.zeros((nv, nc))
        self.W = np.zeros((nv, nc))
        self.V = np.zeros((H, W, 3, nc))
        self.N = np.zeros((H, W, 3, nc))
        self.Z = np.zeros((H, W))
        self.valid = np.zeros((H, W), np.uint8)
        self.T1 = np.zeros((4, 4, nc)) if T0 is None else np.array(_f64(T0), copy=True)
        self.T2 = self.T1.copy()
        self.lost = np.zeros(2, np.int32)
        self.frame = 0


def frame_step(c: OrcConfig, s: OrcSeed, st: State, depth, depth_dot=None, touch=None) -> np.ndarray:
    """One frame step of the sequence from state ``st`` (updated in place).
    -> stats (6,) as in run_sequence.  ``touch``: optional uint8 array over
    the volume, OR-ed with the raycast's footprint bits."""
    _check_solver(c, s)
    for name in ("F", "W", "V", "N", "Z", "T1", "T2"):
        a = getattr(st, name)
        if not (a.dtype == np.float64 and a.flags.c_contiguous):
            setattr(st, name, np.ascontiguousarray(a, dtype=np.float64))
    st.valid = np.ascontiguousarray(st.valid, dtype=np.uint8)
    st.lost = np.ascontiguousarray(st.lost, dtype=np.int32)
    stats = np.zeros(6)
    lib().orc_frame_step(C.byref(c), C.byref(s), int(st.frame), _p(_f64(depth)), _p(_f64(depth_dot)),
                         _p(st.F), _p(st.W), _p(st.V), _p(st.N), _p(st.Z), _p(st.valid, C.c_uint8),
                         _p(st.T1), _p(st.T2), _p(st.lost, C.c_int32), _p(stats), _p(touch, C.c_uint8))
    st.frame += 1
    return stats


def _surfel_arrays(cap: int, nc: int) -> dict:
    return dict(v=np.zeros((cap, 3, nc)), n=np.zeros((cap, 3, nc)), r=np.zeros((cap, nc)), c=np.zeros((cap, nc)),
                t=np.zeros(cap, np.int32))


def pf_run_sequence(c: OrcConfig, s: OrcSeed, depths, T0, depth_dots=None) -> dict:
    """Surfel pipeline (X-PointFusion front end, Sec. 4.2) over a sequence:
    frame 0 at exp(seed) T0.  -> dict(poses (n,4,4,nc), stats (n,6) as
    run_sequence's with surfel updates in column 3, pf (n,3) updated /
    inserted / dropped, surfels dict(v (m,3,nc), n, r (m,nc), c, t (m,)))."""
    _check_solver(c, s)
    nc = ncomp(s)
    depths = _f64(depths)
    n = depths.shape[0]
    poses = np.zeros((n, 4, 4, nc))
    stats = np.zeros((n, 6))
    pf = np.zeros((n, 3), np.int64)
    S = _surfel_arrays(c.pf_capacity, nc)
    cnt = np.zeros(1, np.int64)
    lib().orc_pf_run_sequence(C.byref(c), C.byref(s), n, _p(depths), _p(_f64(depth_dots)), _p(_f64(T0)),
                              _p(poses), _p(stats), _p(pf, C.c_int64), _p(S["v"]), _p(S["n"]), _p(S["r"]),
                              _p(S["c"]), _p(S["t"], C.c_int32), _p(cnt, C.c_int64))
    m = int(cnt[0])
    return dict(poses=poses, stats=stats, pf=pf, surfels={k: v[:m] for k, v in S.items()})


class PfState:
    """State of one surfel frame step: surfels (capacity c.pf_capacity, the
    first `count` in use), level-0 predicted maps, poses of the last two
    frames T1, T2 (4, 4, nc; frame 0 is taken at T1), their lost flags, the
    next frame's index."""

    def __init__(self, c: OrcConfig, s: OrcSeed, T0):
        nc = ncomp(s)
        H, W = c.height, c.width
        self.S = _surfel_arrays(c.pf_capacity, nc)
        self.count = np.zeros(1, np.int64)
        self.V = np.zeros((H, W, 3, nc))
        self.N = np.zeros((H, W, 3, nc))
        self.Z = np.zeros((H, W))
        self.valid = np.zeros((H, W), np.uint8)
        self.T1 = np.array(_f64(T0), copy=True)
        self.T2 = self.T1.copy()
        self.lost = np.zeros(2, np.int32)
        self.frame = 0

    def surfels(self) -> dict:
        m = int(self.count[0])
        return {k: v[:m] for k, v in self.S.items()}


def pf_frame_step(c: OrcConfig, s: OrcSeed, st: PfState, depth, depth_dot=None):
    """One surfel frame step from ``st`` (updated in place) -> (stats (6,),
    pf counts (3,): updated, inserted, dropped)."""
    _check_solver(c, s)
    stats = np.zeros(6)
    pf = np.zeros(3, np.int64)
    S = st.S
    lib().orc_pf_frame_step(C.byref(c), C.byref(s), int(st.frame), _p(_f64(depth)), _p(_f64(depth_dot)),
                            _p(S["v"]), _p(S["n"]), _p(S["r"]), _p(S["c"]), _p(S["t"], C.c_int32),
                            _p(st.count, C.c_int64), _p(st.V), _p(st.N), _p(st.Z), _p(st.valid, C.c_uint8),
                            _p(st.T1), _p(st.T2), _p(st.lost, C.c_int32), _p(stats), _p(pf, C.c_int64))
    st.frame += 1
    return stats, pf


def pf_index_map(c: OrcConfig, v, conf, T, sup: int = 4, c_min: float = -1e300) -> np.ndarray:
    """Index map of surfels at real positions v (m, 3) with confidences conf
    (m,) seen from the real pose T: (sup H, sup W) int64, -1 where empty."""
    v = _f64(np.asarray(v).reshape(-1, 3))
    conf = _f64(np.asarray(conf).reshape(-1))
    out = np.zeros((sup * c.height, sup * c.width), np.int64)
    lib().orc_pf_index_map(C.byref(c), _p(v), _p(conf), len(v), _p(_f64(T)), int(sup), float(c_min),
                           _p(out, C.c_int64))
    return out


def cnn_parts(c: OrcConfig, D2, Nm, Zm, validm, T):
    """Learned-initialiser input parts (real): level-3 depth from the level-2
    filtered depth D2 ((H/4, W/4)), and the level-0 model maps (Nm (H, W, 3),
    Zm (H, W), validm (H, W)) sampled at (8x, 8y) with the normal rotated into
    the camera frame of pose T.  -> (depth (H/8, W/8), model (4, H/8, W/8))
    float32."""
    H3, W3 = c.height // 8, c.width // 8
    d = np.zeros((H3, W3), np.float32)
    m = np.zeros((4, H3, W3), np.float32)
    Nm = np.asarray(Nm)
    Nm = Nm[..., 0] if Nm.ndim == 4 else Nm
    lib().orc_cnn_parts(C.byref(c), _p(_f64(D2)), _p(_f64(Nm)), _p(_f64(Zm)),
                        _p(np.ascontiguousarray(validm, np.uint8), C.c_uint8), _p(_f64(T)),
                        _p(d, C.c_float), _p(m, C.c_float))
    return d, m


def raycast_footprint(c: OrcConfig, s: OrcSeed, F, W, T, touch=None):
    """-> (touch (N,) uint8 with bits 1 = marched cells' corners, 2 = corners of
    cells evaluated at hits; number of hits)."""
    nv = c.dim[0] * c.dim[1] * c.dim[2]
    if touch is None:
        touch = np.zeros(nv, np.uint8)
    hits = lib().orc_raycast_footprint(C.byref(c), C.byref(s), _p(_f64(F)), _p(_f64(W)), _p(_f64(T)),
                                       _p(touch, C.c_uint8))
    return touch, int(hits)


def fuse_margin(c: OrcConfig, s: OrcSeed, Df, T, idx) -> np.ndarray:
    """re(eta) + re(mu) of fusion's update test for the listed voxels (NaN
    where the voxel is decided before that test)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(len(idx))
    lib().orc_fuse_margin(C.byref(c), C.byref(s), _p(_f64(Df)), _p(_f64(T)), _p(idx, C.c_int64), len(idx), _p(out))
    return out


def set_threads(n: int) -> None:
    """Threads for the oracle's per-voxel and per-ray loops (default 1)."""
    lib().orc_set_threads(int(n))


def eval_f(s, x):
    out = np.zeros(ncomp(s))
    lib().orc_eval_f(C.byref(s), float(x), _p(out))
    return out


def eval_g(s, x, y, x_on, y_on):
    out = np.zeros(ncomp(s))
    lib().orc_eval_g(C.byref(s), float(x), float(y), int(x_on), int(y_on), _p(out))
    return out
