"""Seeded synthetic inputs for the CSFD dense-SLAM frame step.

This module only *generates inputs*: analytic scenes, depth frames rendered from
them, depth noise and ground-truth camera trajectories.  It holds none of the
SLAM method's arithmetic (no filtering, no fusion, no ray marching of a TSDF, no
ICP), so both the CPU oracle and the GPU path can consume its output without
sharing any of the method's code.

The workloads stand in for the RGB-D sequences the paper evaluates on
(Sec. 5.1: TUM RGB-D fr1/desk, fr1/xyz and ICL-NUIM), which are not available:
640x480 depth at fx=fy=525 with noise growing as z^2, smooth hand-held-like
trajectories at 30 Hz, and a room-sized scene made of a floor, spheres and
boxes.  No dataset content is reproduced.

Randomness: ``SeedSequence(seed)`` children ``(0,)`` scene, ``(1,)``
trajectory, ``(2, k)`` the depth noise of frame ``k``; every stream is PCG64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Scene", "make_scene", "render_depth", "render_maps", "look_at", "circle_trajectory",
    "spline_trajectory", "Sequence", "make_sequence", "PRESETS", "preset",
]


# --------------------------------------------------------------------------
# Scene
# --------------------------------------------------------------------------
@dataclass
class Scene:
    L: float                       # cube edge in metres; world origin at cube centre
    floor_y: float                 # floor plane y = floor_y (solid below)
    spheres: np.ndarray            # (n, 4): cx, cy, cz, r
    boxes: np.ndarray              # (n, 6): cx, cy, cz, hx, hy, hz

    def sdf(self, p: np.ndarray) -> np.ndarray:
        """Signed distance of points p (..., 3) to the union of primitives."""
        p = np.asarray(p, dtype=np.float64)
        d = p[..., 1] - self.floor_y
        for cx, cy, cz, r in self.spheres:
            ds = np.linalg.norm(p - np.array([cx, cy, cz]), axis=-1) - r
            d = np.minimum(d, ds)
        for cx, cy, cz, hx, hy, hz in self.boxes:
            q = np.abs(p - np.array([cx, cy, cz])) - np.array([hx, hy, hz])
            outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
            inside = np.minimum(np.max(q, axis=-1), 0.0)
            d = np.minimum(d, outside + inside)
        return d

    def centroid(self) -> np.ndarray:
        c = [s[:3] for s in self.spheres] + [b[:3] for b in self.boxes]
        return np.mean(np.array(c), axis=0)


def _children(seed: int):
    return (np.random.SeedSequence(seed, spawn_key=(0,)),
            np.random.SeedSequence(seed, spawn_key=(1,)))


def noise_stream(seed: int, k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(2, k))))


def make_scene(seed: int, L: float, n_spheres: int = 3, n_boxes: int = 2,
               centre_frac: float = 0.7) -> Scene:
    """Floor at y=-0.3L, spheres r~U(0.2,0.5) m, boxes half-extents ~U(0.1,0.4) m,
    all resting on the floor with non-overlapping xz footprints, centres
    uniform over the central ``centre_frac`` of the cube in x and z."""
    rng = np.random.Generator(np.random.PCG64(_children(seed)[0]))
    floor_y = -0.3 * L
    half = 0.5 * centre_frac * L
    placed = []  # (x, z, footprint radius)
    spheres, boxes = [], []
    kinds = ["s"] * n_spheres + ["b"] * n_boxes
    for kind in kinds:
        for _ in range(100000):
            if kind == "s":
                r = rng.uniform(0.2, 0.5)
                size = (r,)
                foot = r
            else:
                hx, hy, hz = rng.uniform(0.1, 0.4, size=3)
                size = (hx, hy, hz)
                foot = float(np.hypot(hx, hz))
            x, z = rng.uniform(-half, half, size=2)
            if all(np.hypot(x - px, z - pz) > foot + pf + 0.05 for px, pz, pf in placed):
                break
        else:  # pragma: no cover - generator cannot place objects
            raise RuntimeError("scene generator failed to place objects")
        placed.append((x, z, foot))
        if kind == "s":
            spheres.append((x, floor_y + size[0], z, size[0]))
        else:
            boxes.append((x, floor_y + size[1], z, size[0], size[1], size[2]))
    return Scene(L=L, floor_y=floor_y, spheres=np.array(spheres, dtype=np.float64).reshape(-1, 4),
                 boxes=np.array(boxes, dtype=np.float64).reshape(-1, 6))


# --------------------------------------------------------------------------
# Rendering (analytic first hit of the union; exact equivalent of sphere tracing)
# --------------------------------------------------------------------------
def _rays(pose: np.ndarray, W: int, H: int, fx: float, fy: float, cx: float, cy: float):
    xs = (np.arange(W, dtype=np.float64) - cx) / fx
    ys = (np.arange(H, dtype=np.float64) - cy) / fy
    dc = np.stack(np.broadcast_arrays(xs[None, :], ys[:, None], np.ones((1, 1))), axis=-1)  # (H,W,3), z=1
    R = pose[:3, :3]
    d = dc @ R.T
    o = pose[:3, 3]
    return o, d


def render_depth(scene: Scene, pose: np.ndarray, W: int, H: int, fx: float, fy: float,
                 cx: float, cy: float, max_range: float = 10.0) -> np.ndarray:
    """Noise-free camera-z depth (FP64) of the first surface hit; 0 on a miss.
    The ray through pixel u is o + t R K^-1 (u,1): t is the camera z depth."""
    o, d = _rays(pose, W, H, fx, fy, cx, cy)
    t = np.full(d.shape[:2], np.inf)
    # floor: y = floor_y
    with np.errstate(divide="ignore", invalid="ignore"):
        tf = (scene.floor_y - o[1]) / d[..., 1]
    t = np.where((tf > 0) & np.isfinite(tf), np.minimum(t, tf), t)
    a = np.einsum("hwi,hwi->hw", d, d)
    for cx_, cy_, cz_, r in scene.spheres:
        oc = o - np.array([cx_, cy_, cz_])
        b = 2.0 * (d @ oc)
        c = oc @ oc - r * r
        disc = b * b - 4 * a * c
        ok = disc >= 0
        ts = np.where(ok, (-b - np.sqrt(np.where(ok, disc, 0.0))) / (2 * a), np.inf)
        t = np.where((ts > 0) & ok, np.minimum(t, ts), t)
    for cx_, cy_, cz_, hx, hy, hz in scene.boxes:
        lo = np.array([cx_ - hx, cy_ - hy, cz_ - hz]) - o
        hi = np.array([cx_ + hx, cy_ + hy, cz_ + hz]) - o
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = lo / d
            t2 = hi / d
        tn = np.nanmax(np.minimum(t1, t2), axis=-1)
        tx = np.nanmin(np.maximum(t1, t2), axis=-1)
        ok = (tn <= tx) & (tn > 0)
        t = np.where(ok, np.minimum(t, tn), t)
    t = np.where(np.isfinite(t) & (t <= max_range), t, 0.0)
    return t


def render_maps(scene: Scene, pose: np.ndarray, W: int, H: int, fx: float, fy: float,
                cx: float, cy: float, max_range: float = 10.0):
    """Noise-free analytic surface maps: camera-z depth (H,W), world hit points
    (H,W,3) and outward surface normals (H,W,3); zeros on a miss."""
    o, d = _rays(pose, W, H, fx, fy, cx, cy)
    z = render_depth(scene, pose, W, H, fx, fy, cx, cy, max_range)
    P = o + z[..., None] * d
    N = np.zeros_like(P)
    best = np.full(z.shape, np.inf)
    # classify by the primitive whose signed distance is smallest in magnitude
    cand = [("floor", None)] + [("s", s) for s in scene.spheres] + [("b", b) for b in scene.boxes]
    for kind, prm in cand:
        if kind == "floor":
            dist = np.abs(P[..., 1] - scene.floor_y)
            n = np.broadcast_to(np.array([0.0, 1.0, 0.0]), P.shape)
        elif kind == "s":
            q = P - prm[:3]
            dist = np.abs(np.linalg.norm(q, axis=-1) - prm[3])
            n = q / np.maximum(np.linalg.norm(q, axis=-1, keepdims=True), 1e-300)
        else:
            q = (P - prm[:3]) / prm[3:]
            ax = np.argmax(np.abs(q), axis=-1)
            n = np.zeros_like(P)
            np.put_along_axis(n, ax[..., None], np.sign(np.take_along_axis(q, ax[..., None], -1)), -1)
            qa = np.abs(P - prm[:3]) - prm[3:]
            dist = np.abs(np.max(qa, axis=-1))
        upd = dist < best
        best = np.where(upd, dist, best)
        N = np.where(upd[..., None], n, N)
    hit = z > 0
    return z, np.where(hit[..., None], P, 0.0), np.where(hit[..., None], N, 0.0)


def add_noise(z: np.ndarray, seed: int, k: int, sigma2: float = 0.0012):
    """Returns (noisy depth, noise-scale tangent) with noise sigma2*z^2*n, n~N(0,1)."""
    n = noise_stream(seed, k).standard_normal(z.shape)
    tangent = np.where(z > 0, sigma2 * z * z * n, 0.0)
    return np.where(z > 0, z + tangent, 0.0), tangent


# --------------------------------------------------------------------------
# Trajectories (camera-to-world 4x4; camera x right, y down, z forward)
# --------------------------------------------------------------------------
def look_at(eye, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, y, f, eye
    return T


def _look_at_many(eye: np.ndarray, target: np.ndarray) -> np.ndarray:
    f = target - eye
    f /= np.linalg.norm(f, axis=-1, keepdims=True)
    x = np.cross(f, np.array([0.0, 1.0, 0.0]))
    x /= np.linalg.norm(x, axis=-1, keepdims=True)
    y = np.cross(f, x)
    return np.stack([x, y, f], axis=-1)


def circle_trajectory(n_frames: int, radius: float, height: float = 0.0,
                      deg_per_frame: float = 2.0) -> np.ndarray:
    poses = []
    for k in range(n_frames):
        a = np.deg2rad(deg_per_frame * k)
        eye = (radius * np.sin(a), height, -radius * np.cos(a))
        poses.append(look_at(eye, (0.0, height, 0.0)))
    return np.array(poses)


def _catmull_rom(P: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Uniform Catmull-Rom through control points P (n,3) at parameters s in [0, n-1]."""
    n = len(P)
    Q = np.concatenate([P[:1], P, P[-1:]], axis=0)
    i = np.clip(np.floor(s).astype(int), 0, n - 2)
    t = (s - i)[:, None]
    p0, p1, p2, p3 = Q[i], Q[i + 1], Q[i + 2], Q[i + 3]
    return 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t ** 2
                  + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3)


def _rot_angle(Ra: np.ndarray, Rb: np.ndarray) -> np.ndarray:
    # ||Ra - Rb||_F = 2 sqrt(2) sin(theta/2): accurate for small angles too
    f = np.sqrt(np.einsum("nij,nij->n", Ra - Rb, Ra - Rb))
    return 2.0 * np.arcsin(np.clip(f / (2.0 * np.sqrt(2.0)), 0.0, 1.0))


def spline_trajectory(seed: int, scene: Scene, n_frames: int, v_max: float = 0.5,
                      w_max_deg: float = 30.0, fps: float = 30.0, n_ctrl: int = 8,
                      clearance: float = 0.3) -> np.ndarray:
    """Catmull-Rom position spline through ``n_ctrl`` points in the central 50% of
    the cube, 0.8-1.8 m above the floor and >= ``clearance`` from every surface,
    looking at a second spline through points near the object centroid; retimed
    so speed <= v_max and angular rate <= w_max at ``fps`` with a smooth speed
    profile (no jumps in velocity) that slows down towards the path's ends;
    ping-pongs along the path if it is shorter than the requested number of
    frames."""
    rng = np.random.Generator(np.random.PCG64(_children(seed)[1]))
    L = scene.L
    half = 0.25 * L
    cen = scene.centroid()
    for _attempt in range(200):
        ctrl = []
        while len(ctrl) < n_ctrl:
            p = np.array([rng.uniform(-half, half), scene.floor_y + rng.uniform(0.8, 1.8),
                          rng.uniform(-half, half)])
            if scene.sdf(p[None])[0] >= clearance + 0.05:
                ctrl.append(p)
        ctrl = np.array(ctrl)
        tgt = cen[None, :] + rng.uniform(-0.3, 0.3, size=(n_ctrl, 3))
        s = np.linspace(0.0, n_ctrl - 1.0, 20001)
        pos = _catmull_rom(ctrl, s)
        if np.min(scene.sdf(pos)) < clearance:
            continue
        tg = _catmull_rom(tgt, s)
        if np.min(np.linalg.norm(tg - pos, axis=-1)) < 0.5:
            continue
        break
    else:  # pragma: no cover
        raise RuntimeError("trajectory generator failed")
    Rs = _look_at_many(pos, tg)
    dl = np.linalg.norm(np.diff(pos, axis=0), axis=-1)
    da = _rot_angle(Rs[:-1], Rs[1:])
    # seconds per segment at the limits (5% margin for the within-segment nonlinearity)
    cost = np.maximum(dl / (0.95 * v_max), da / np.deg2rad(0.95 * w_max_deg))
    # a smooth speed profile: the running maximum over +-W samples, averaged
    # over +-W samples, bounds every sample's own cost (so the limits still
    # hold) and changes continuously; towards both ends of the path the speed
    # ramps down to a tenth, so that the ping-pong turnaround is gentle
    W = 400
    pad = np.pad(cost, W, mode="edge")
    win = np.lib.stride_tricks.sliding_window_view(pad, 2 * W + 1)
    env = win.max(axis=1)
    ker = np.ones(2 * W + 1) / (2 * W + 1)
    cost = np.convolve(np.pad(env, W, mode="edge"), ker, mode="valid")
    ramp = 3 * W
    u = np.minimum(np.arange(len(cost)), np.arange(len(cost))[::-1]) / ramp
    cost = cost / np.maximum(0.1, np.sin(0.5 * np.pi * np.minimum(u, 1.0)))
    tcum = np.concatenate([[0.0], np.cumsum(cost)])
    total = tcum[-1]
    period = 2.0 * total
    tk = (np.arange(n_frames) / fps) % period
    tk = np.where(tk > total, period - tk, tk)
    j = np.clip(np.searchsorted(tcum, tk, side="right") - 1, 0, len(s) - 2)
    w = ((tk - tcum[j]) / np.maximum(cost[j], 1e-300))[:, None]
    eye = (1 - w) * pos[j] + w * pos[j + 1]
    tgt_k = (1 - w) * tg[j] + w * tg[j + 1]
    poses = np.array([look_at(e, t) for e, t in zip(eye, tgt_k)])
    # assert the motion limits (the spline sampling makes them hold to within the grid)
    dpos = np.linalg.norm(np.diff(poses[:, :3, 3], axis=0), axis=-1) * fps
    dang = np.rad2deg(_rot_angle(poses[:-1, :3, :3], poses[1:, :3, :3])) * fps
    assert dpos.max(initial=0) <= v_max and dang.max(initial=0) <= w_max_deg
    return poses


# --------------------------------------------------------------------------
# Sequences and presets
# --------------------------------------------------------------------------
@dataclass
class Sequence:
    scene: Scene
    poses_gt: np.ndarray          # (K, 4, 4) FP64 camera-to-world
    camera: dict                  # width, height, fx, fy, cx, cy
    seed: int
    depth_dtype: type = np.float32
    sigma2: float = 0.0012
    _cache: dict = field(default_factory=dict, repr=False)

    def __len__(self):
        return len(self.poses_gt)

    def frame(self, k: int, noise: bool = True):
        """Depth of frame k in ``depth_dtype`` and the noise-scale tangent."""
        key = (k, noise)
        if key not in self._cache:
            c = self.camera
            z = render_depth(self.scene, self.poses_gt[k], c["width"], c["height"],
                             c["fx"], c["fy"], c["cx"], c["cy"])
            if noise:
                d, tan = add_noise(z, self.seed, k, self.sigma2)
            else:
                d, tan = z, np.zeros_like(z)
            self._cache[key] = (d.astype(self.depth_dtype), tan.astype(self.depth_dtype))
        return self._cache[key]

    def depths(self, n: int | None = None, noise: bool = True, workers: int = 1) -> np.ndarray:
        """Depth frames 0..n-1 (``workers`` > 1 renders them in a process pool)."""
        n = len(self) if n is None else n
        if workers > 1 and n > 1:
            from concurrent.futures import ProcessPoolExecutor
            args = [(self.scene, self.poses_gt[k], self.camera, self.seed, k, noise, self.sigma2,
                     self.depth_dtype) for k in range(n)]
            with ProcessPoolExecutor(workers) as ex:
                return np.stack(list(ex.map(_render_one, args, chunksize=4)))
        return np.stack([self.frame(k, noise)[0] for k in range(n)])

    def depths_and_tangents(self, n: int | None = None, workers: int = 1):
        """Noisy depth frames 0..n-1 and their noise-scale tangents."""
        n = len(self) if n is None else n
        if workers > 1 and n > 1:
            from concurrent.futures import ProcessPoolExecutor
            args = [(self.scene, self.poses_gt[k], self.camera, self.seed, k, True, self.sigma2,
                     self.depth_dtype, True) for k in range(n)]
            with ProcessPoolExecutor(workers) as ex:
                out = list(ex.map(_render_one, args, chunksize=4))
        else:
            out = [self.frame(k) for k in range(n)]
        return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def _render_one(a):
    scene, pose, c, seed, k, noise, sigma2, dt = a[:8]
    with_tangent = len(a) > 8 and a[8]
    z = render_depth(scene, pose, c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"])
    if noise:
        d, tan = add_noise(z, seed, k, sigma2)
    else:
        d, tan = z, np.zeros_like(z)
    return (d.astype(dt), tan.astype(dt)) if with_tangent else d.astype(dt)


PRESETS = {
    # 128^3 at 2 cm in a 2.56 m cube; 160x120; 20 frames on a circle; FP64-complex
    "c0": dict(seed=0, L=2.56, dim=128, voxel=0.02, trunc=0.06, wcap=64.0,
               camera=dict(width=160, height=120, fx=130.0, fy=130.0, cx=79.5, cy=59.5),
               n_frames=20, traj="circle", radius=1.5, prec="c128",
               icp=dict(iters=(10, 5, 4), dgate=0.1, agate_deg=20.0), h=1e-20),
    # 512^3 at 1 cm in a 5.12 m cube; 640x480 at fx=fy=525; 500 frames on a spline; FP32-complex
    "c1": dict(seed=1, L=5.12, dim=512, voxel=0.01, trunc=0.06, wcap=64.0,
               camera=dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5),
               n_frames=500, traj="spline", prec="c64",
               icp=dict(iters=(10, 5, 4), dgate=0.1, agate_deg=20.0), h=2.0 ** -20),
    # 256^3 at 2 cm (config 1 generator), 300 frames
    "c2": dict(seed=2, L=5.12, dim=256, voxel=0.02, trunc=0.06, wcap=64.0,
               camera=dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5),
               n_frames=300, traj="spline", prec="c64",
               icp=dict(iters=(10, 5, 4), dgate=0.1, agate_deg=20.0), h=2.0 ** -20),
}


# The 16 parameters of the batched-direction workload: initial pose (6),
# truncation, weight cap, ICP distance and angle gates, the three per-level ICP
# step weights, the depth-noise scale, fx, fy (library parameter ids).
PARAMS16 = (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 17, 13, 14)


def instance_presets(n: int = 24, seed0: int = 100) -> list:
    """Uneven independent sequences: TSDF of 128^3..384^3 voxels at 1 or 2 cm
    (cubes below 2.56 m are redrawn: the scene generator places its objects in
    the central 70% of a cube of at least that size), 320x240 (fx=fy=262.5) or
    640x480 (fx=fy=525) depth, 60..400 frames, 1..6 complex directions drawn
    from PARAMS16.  Instance i uses scene seed seed0 + i; the draws come from
    PCG64 stream SeedSequence(seed0 + i, spawn_key=(3,)).  Cubes of at least
    3.84 m use the spline trajectory, smaller ones the 1.5 m circle."""
    out = []
    for i in range(n):
        seed = seed0 + i
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(3,))))
        while True:
            dim = int(rng.choice([128, 192, 256, 320, 384]))
            voxel = float(rng.choice([0.01, 0.02]))
            if dim * voxel >= 2.56 - 1e-9:
                break
        if rng.random() < 0.5:
            cam = dict(width=320, height=240, fx=262.5, fy=262.5, cx=159.5, cy=119.5)
        else:
            cam = dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5)
        frames = int(rng.integers(60, 401))
        nd = int(rng.integers(1, 7))
        dirs = [int(x) for x in rng.choice(PARAMS16, size=nd, replace=False)]
        L = dim * voxel
        out.append(dict(seed=seed, L=L, dim=dim, voxel=voxel, trunc=0.06, wcap=64.0, camera=cam,
                        n_frames=frames, traj="spline" if L >= 3.84 - 1e-9 else "circle", radius=1.5,
                        prec="c64", icp=dict(iters=(10, 5, 4), dgate=0.1, agate_deg=20.0), h=2.0 ** -20,
                        dirs=dirs))
    return out


def preset(name: str, **overrides) -> dict:
    p = {**PRESETS[name]}
    for k, v in overrides.items():
        p[k] = v
    return p


def make_sequence(p: dict, n_frames: int | None = None) -> Sequence:
    n = p["n_frames"] if n_frames is None else n_frames
    scene = make_scene(p["seed"], p["L"])
    if p["traj"] == "circle":
        poses = circle_trajectory(n, p.get("radius", 1.5), 0.0, 2.0)
    else:
        poses = spline_trajectory(p["seed"], scene, n)
    dt = np.float64 if p["prec"] == "c128" else np.float32
    return Sequence(scene=scene, poses_gt=poses, camera=dict(p["camera"]), seed=p["seed"],
                    depth_dtype=dt)
