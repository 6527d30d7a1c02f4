"""MI355X-native CSFD dense-SLAM frame step (X-SLAM, Sec. 3-4.1).

The hot path lives in ``libxslam.so`` (hand-written HIP for gfx950 behind the C
ABI of ``include/xslam.h``); :mod:`paper_2405_02187_amd.xslam` is its ctypes
binding and :mod:`paper_2405_02187_amd.build` compiles it.
"""
