"""Launch-shape autotuner with a JSON cache.

The library times the stages it can re-run without changing state (raycast
tile, ICP grid per level; ``Slam.autotune``).  The fusion grid changes the
TSDF when it runs, so it is tuned here on real frames: consecutive steps of
the sequence with different grids, timed by the library's per-kernel event
timer (no result depends on the fusion grid).  The library's ICP choice per
level is then checked on real frames too, against the one-pixel-per-thread
grid: passes timed back to back in isolation do not always rank the grids as
the frame step, where each pass follows a finish launch and the levels
alternate, does.  (The ICP grid changes the order of the FP64 partial sums,
so the poses of those frames may differ by rounding.)  Chosen shapes are
cached per workload shape (image size, volume, precision, directions, Hessian
size).
"""
from __future__ import annotations

import json
import os

from . import xslam as X

FUSE_GRIDS = (4096, 2048, 1024, 512)
# shapes the tuner chose on an MI355X, per workload key (used when there is no
# time to tune, e.g. a short benchmark warm-up)
SHAPES_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "launch_shapes.json")
ICP_FULL = 0          # ICP workgroups value of the one-pixel-per-thread grid
ICP_PREFER = 0.95     # a grid other than the one-pixel-per-thread one must be 5% faster


def key(slam: "X.Slam") -> str:
    c = slam.cfg
    prec = "c128" if c.prec == X.C128 else "c64"
    dims = "x".join(str(int(d)) for d in c.vol.dim)
    return f"{c.cam.width}x{c.cam.height}_{dims}_{prec}_D{slam.D}_Q{slam.Q}"


def load(path: str) -> dict:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(slam: "X.Slam", shapes: dict) -> None:
    slam.set_launch(ray_tile=tuple(shapes["ray_tile"]), icp_blocks=tuple(shapes["icp_blocks"]),
                    fuse_blocks=int(shapes["fuse_blocks"]))


def _icp_ms(slam: "X.Slam") -> float:
    """Event-timed ms so far of the ICP passes and their finish launches (the
    finish reduces one partial per workgroup, so it depends on the grid too)."""
    ms = slam.kernel_times()[0]
    return float(ms[X.TIMER_CLASSES.index("k_icp")] + ms[X.TIMER_CLASSES.index("k_icp_finish")])


def _icp_on_steps(slam: "X.Slam", take, frames_per_cand: int) -> dict:
    """Per level (0, 1, 2 in turn): if the library chose a grid other than the
    one-pixel-per-thread one, step ``frames_per_cand`` frames with each of the
    two, alternating, and keep the other grid only if its ICP time (passes
    and finish launches) over those frames is 5% lower.  -> {level: {grid: ms per frame}}."""
    out = {}
    for lvl in range(3):
        cur = list(slam.get_launch()["icp_blocks"])
        full = list(cur)
        full[lvl] = ICP_FULL
        slam.set_launch(icp_blocks=full)
        full_g = slam.get_launch()["icp_blocks"][lvl]
        if full_g == cur[lvl]:
            continue
        cands = {cur[lvl]: 0.0, full_g: 0.0}
        for _ in range(frames_per_cand):
            for g in cands:
                cfg = list(cur)
                cfg[lvl] = g
                slam.set_launch(icp_blocks=cfg)
                before = _icp_ms(slam)
                slam.step(take())
                cands[g] += _icp_ms(slam) - before
        keep = cur[lvl] if cands[cur[lvl]] < ICP_PREFER * cands[full_g] else full_g
        cfg = list(cur)
        cfg[lvl] = keep
        slam.set_launch(icp_blocks=cfg)
        out[lvl] = {str(g): t / frames_per_cand for g, t in cands.items()}
    return out


def tune(slam: "X.Slam", frames, reps: int = 20, fuse_frames_per_grid: int = 2,
         icp_frames_per_grid: int | None = None) -> dict:
    """Tune on a context that has stepped at least one frame.  ``frames`` is an
    iterable of device depth frames that continue the sequence, at least
    ``frames_needed(fuse_frames_per_grid, icp_frames_per_grid)`` of them
    (fusion grid: len(FUSE_GRIDS) * fuse_frames_per_grid; ICP grids on steps:
    up to 3 levels x 2 grids x icp_frames_per_grid, default
    fuse_frames_per_grid; 0 skips that check).
    -> dict(ray_tile, icp_blocks, fuse_blocks, ms, frames): ``frames`` is the
    number of frames stepped (the ICP check skips a level whose grid is
    already the one-pixel-per-thread one), so the sequence continues with
    the frame after them."""
    if icp_frames_per_grid is None:
        icp_frames_per_grid = fuse_frames_per_grid
    shapes, ms = slam.autotune(reps)
    it = iter(frames)
    used = 0

    def take():
        nonlocal used
        try:
            f = next(it)
        except StopIteration:
            raise ValueError(f"autotune.tune: ran out of frames after {used}; pass "
                             f"frames_needed({fuse_frames_per_grid}, {icp_frames_per_grid}) of them") from None
        used += 1
        return f

    i_fuse = X.TIMER_CLASSES.index("k_fuse")
    t_fuse = {g: 0.0 for g in FUSE_GRIDS}
    slam.set_timing(True)
    try:
        for _ in range(fuse_frames_per_grid):
            for g in FUSE_GRIDS:
                slam.set_launch(fuse_blocks=g)
                before = slam.kernel_times()[0][i_fuse]
                slam.step(take())
                t_fuse[g] += slam.kernel_times()[0][i_fuse] - before
        best_fuse = min(FUSE_GRIDS, key=lambda g: t_fuse[g])
        slam.set_launch(fuse_blocks=best_fuse)
        icp_steps = _icp_on_steps(slam, take, icp_frames_per_grid) if icp_frames_per_grid > 0 else {}
    finally:
        slam.set_timing(False)
    out = slam.get_launch()
    out["ms"] = dict(raycast=float(ms[0]), icp=[float(x) for x in ms[1:]],
                     fuse={str(g): t_fuse[g] / fuse_frames_per_grid for g in FUSE_GRIDS},
                     icp_steps={str(k): v for k, v in icp_steps.items()})
    out["ray_tile"] = list(out["ray_tile"])
    out["icp_blocks"] = list(out["icp_blocks"])
    out["frames"] = used
    return out


def tuned(slam: "X.Slam", frames, cache_path: str | None = None, reps: int = 20) -> dict:
    """Cached shapes for this workload if present (applied), else tune, store
    and return them."""
    cache = load(cache_path) if cache_path else {}
    k = key(slam)
    if k in cache:
        apply(slam, cache[k])
        return cache[k]
    out = tune(slam, frames, reps=reps)
    if cache_path:
        cache[k] = out
        save(cache_path, cache)
    return out


def frames_needed(fuse_frames_per_grid: int = 2, icp_frames_per_grid: int | None = None) -> int:
    if icp_frames_per_grid is None:
        icp_frames_per_grid = fuse_frames_per_grid
    return len(FUSE_GRIDS) * fuse_frames_per_grid + 3 * 2 * icp_frames_per_grid


__all__ = ["key", "load", "save", "apply", "tune", "tuned", "frames_needed", "FUSE_GRIDS"]
