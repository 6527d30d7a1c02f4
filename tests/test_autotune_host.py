"""Host logic of the launch-shape autotuner (no GPU): the fusion grid is
taken from timed frame steps, the library's ICP grid per level is checked on
frame steps against the one-pixel-per-thread grid with a 5% preference for the
latter, and the tuner reports how many frames it stepped.  A stand-in context
gives each launch shape a fixed kernel time per frame."""
import numpy as np
import pytest

from paper_2405_02187_amd import autotune as AT
from paper_2405_02187_amd import xslam as X

FULL = (1200, 300, 75)    # one pixel per thread at 640x480 and its two pyramid levels
I_ICP, I_FIN, I_FUSE = (X.TIMER_CLASSES.index(k) for k in ("k_icp", "k_icp_finish", "k_fuse"))


class FakeSlam:
    """What ``AT.tune`` uses of ``X.Slam``: the library tuner's choice is
    given; per frame, ICP time = sum over levels of icp_ms[level][grid] (split
    between the pass and finish classes), fusion time = fuse_ms[grid]."""

    def __init__(self, lib_choice, icp_ms, fuse_ms):
        self.lib_choice = list(lib_choice)
        self.icp_ms, self.fuse_ms = icp_ms, fuse_ms
        self.icp = [0, 0, 0]
        self.fuse = 2048
        self.ms = np.zeros(X.N_TIMER_CLASSES)
        self.n = np.zeros(X.N_TIMER_CLASSES, dtype=np.int64)
        self.timing = False
        self.stepped = []

    def autotune(self, reps):
        self.icp = list(self.lib_choice)
        return self.get_launch(), np.array([0.1, 0.02, 0.015, 0.013])

    def get_launch(self):
        return dict(ray_tile=(16, 4), icp_blocks=tuple(g if g > 0 else f for g, f in zip(self.icp, FULL)),
                    fuse_blocks=self.fuse)

    def set_launch(self, ray_tile=None, icp_blocks=None, fuse_blocks=None):
        if icp_blocks is not None:
            assert all(0 <= g <= 1200 for g in icp_blocks)
            self.icp = list(icp_blocks)
        if fuse_blocks is not None:
            self.fuse = int(fuse_blocks)

    def set_timing(self, on=True):
        self.timing = on

    def kernel_times(self):
        return self.ms.copy(), self.n.copy()

    def step(self, frame):
        self.stepped.append(frame)
        if not self.timing:
            return
        shapes = self.get_launch()["icp_blocks"]
        t = sum(self.icp_ms[lvl][g] for lvl, g in enumerate(shapes))
        self.ms[I_ICP] += 0.6 * t
        self.ms[I_FIN] += 0.4 * t
        self.ms[I_FUSE] += self.fuse_ms[self.fuse]


FUSE_MS = {4096: 0.031, 2048: 0.027, 1024: 0.030, 512: 0.032}


def _icp_ms(l0, l1, l2):
    return [l0, l1, l2]


def test_frames_needed_counts_fusion_and_icp_checks():
    assert AT.frames_needed(2) == 4 * 2 + 3 * 2 * 2
    assert AT.frames_needed(1) == 4 + 6
    assert AT.frames_needed(2, 0) == 8


def test_icp_check_keeps_faster_smaller_grid_and_reverts_slower_one():
    # level 0: the library's 512 is much faster in frame steps than 1200 -> kept;
    # level 1: the library's 96 is slower in frame steps than 300 -> full grid;
    # level 2: already the full grid -> not checked, no frames spent
    icp = _icp_ms({512: 0.16, 1200: 0.21}, {96: 0.075, 300: 0.048}, {75: 0.031})
    s = FakeSlam((512, 96, 0), icp, FUSE_MS)
    frames = list(range(100, 100 + AT.frames_needed(2)))
    out = AT.tune(s, frames, reps=1)
    assert out["icp_blocks"] == [512, 300, 75]
    assert out["fuse_blocks"] == 2048
    assert out["frames"] == 8 + 4 + 4
    assert s.stepped == frames[:out["frames"]]          # in order, none skipped
    steps = out["ms"]["icp_steps"]
    assert set(steps) == {"0", "1"}
    assert steps["0"]["512"] < steps["0"]["1200"]
    assert not s.timing


def test_icp_check_prefers_full_grid_within_five_percent():
    # the rule compares the frames' whole ICP time (all levels; here only level
    # 1 takes time): 3% lower is not enough to keep the smaller grid, 6% is
    for gain, keep in ((0.97, 300), (0.94, 128)):
        icp = _icp_ms({1200: 0.0}, {128: 0.05 * gain, 300: 0.05}, {75: 0.0})
        s = FakeSlam((0, 128, 0), icp, FUSE_MS)
        out = AT.tune(s, range(AT.frames_needed(2)), reps=1)
        assert out["icp_blocks"][1] == keep, (gain, out)
        assert out["frames"] == 8 + 4


def test_icp_check_can_be_skipped():
    icp = _icp_ms({512: 0.16, 1200: 0.21}, {96: 0.075, 300: 0.048}, {32: 0.05, 75: 0.031})
    s = FakeSlam((512, 96, 32), icp, FUSE_MS)
    out = AT.tune(s, range(AT.frames_needed(1, 0)), reps=1, fuse_frames_per_grid=1, icp_frames_per_grid=0)
    assert out["icp_blocks"] == [512, 96, 32]            # the library's choice stands
    assert out["frames"] == 4


def test_too_few_frames_is_an_error():
    icp = _icp_ms({512: 0.16, 1200: 0.21}, {300: 0.048}, {75: 0.031})
    s = FakeSlam((512, 0, 0), icp, FUSE_MS)
    with pytest.raises(ValueError, match="ran out of frames after 9"):
        AT.tune(s, range(8 + 1), reps=1)
    assert not s.timing
