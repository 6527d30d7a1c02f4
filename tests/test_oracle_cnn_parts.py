"""Pins of the oracle's learned-initialiser input parts: the level-3 depth is
the pyramid's gated binomial applied once more (a linear ramp stays a linear
ramp sampled at the even positions; a depth step beyond the gate is not
averaged across), and the model channels are the level-0 maps at (8x, 8y)
with the normal rotated into the camera frame (R^T n in closed form; invalid
pixels 0)."""
import numpy as np

import oracle as O

W, H = 64, 48


def cfg():
    return O.config(None, width=W, height=H, fx=50.0, fy=50.0, cx=31.5, cy=23.5, dim=(32,) * 3, voxel=0.02,
                    sigma_m=0.03)


def rot(axis, ang):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
    T[:3, 3] = (0.1, -0.2, 0.3)
    return T


def test_level3_depth_of_a_ramp_and_of_a_step():
    c = cfg()
    y, x = np.mgrid[0:H // 4, 0:W // 4].astype(float)
    ramp = 1.0 + 0.001 * x + 0.0005 * y                 # gradients far below the 9 cm gate
    d, _ = O.cnn_parts(c, ramp, np.zeros((H, W, 3)), np.zeros((H, W)), np.zeros((H, W), np.uint8), np.eye(4))
    # away from the border the symmetric binomial reproduces the linear ramp at (2x, 2y)
    inner = d[1:-1, 1:-1]
    exp = (1.0 + 0.001 * (2 * x[:H // 8, :W // 8]) + 0.0005 * (2 * y[:H // 8, :W // 8]))[1:-1, 1:-1]
    assert np.abs(inner - exp.astype(np.float32)).max() < 2e-7
    step = np.where(x < 8, 1.0, 1.5)
    d, _ = O.cnn_parts(c, step, np.zeros((H, W, 3)), np.zeros((H, W)), np.zeros((H, W), np.uint8), np.eye(4))
    assert np.all(d[:, :4] == np.float32(1.0)) and np.all(d[:, 4:] == np.float32(1.5))


def test_model_channels_rotate_normals_into_the_camera():
    c = cfg()
    rng = np.random.default_rng(3)
    N = rng.standard_normal((H, W, 3))
    N /= np.linalg.norm(N, axis=-1, keepdims=True)
    Z = 1.0 + rng.random((H, W))
    valid = (rng.random((H, W)) < 0.7).astype(np.uint8)
    T = rot([0.3, -1.0, 0.4], 0.7)
    _, m = O.cnn_parts(c, np.zeros((H // 4, W // 4)), N, Z, valid, T)
    Ns = N[::8, ::8]
    ref = Ns @ T[:3, :3]                                # R^T n as row vectors
    v = valid[::8, ::8].astype(bool)
    assert np.all(m[:, ~v] == 0)
    assert np.abs(m[0][v] - Z[::8, ::8][v].astype(np.float32)).max() == 0
    for k in range(3):
        assert np.abs(m[1 + k][v] - ref[..., k][v]).max() < 1e-6
