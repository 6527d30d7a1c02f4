"""Pins of the FP64 CNN oracle of the learned ICP initialiser: the strided
convolution against a brute-force loop, every parameter gradient against
central finite differences, the parameter count, and one Adam step against its
closed form on a quadratic."""
import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, w, b):
    N, Ci, H, W = x.shape
    Co = w.shape[0]
    Ho, Wo = cnn.out_size(H), cnn.out_size(W)
    y = np.zeros((N, Co, Ho, Wo))
    for n in range(N):
        for o in range(Co):
            for i in range(Ho):
                for j in range(Wo):
                    s = b[o]
                    for c in range(Ci):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xx = 2 * i - 1 + ky, 2 * j - 1 + kx
                                if 0 <= yy < H and 0 <= xx < W:
                                    s += w[o, c, ky, kx] * x[n, c, yy, xx]
                    y[n, o, i, j] = s
    return y


def test_parameter_count():
    assert cnn.n_params() == 106374


@pytest.mark.parametrize("H,W", [(7, 9), (8, 6), (15, 10)])
def test_strided_conv_matches_brute_force(H, W):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, H, W))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.allclose(cnn.conv_s2(x, w, b), brute_conv(x, w, b), atol=1e-12)


def test_shapes_through_the_network():
    p = cnn.init_params(0)
    x = np.random.default_rng(2).standard_normal((3, 5, 60, 80))
    xi, cache = cnn.forward(p, x)
    assert xi.shape == (3, 6)
    assert [a.shape[2:] for a in cache["acts"]] == [(60, 80), (30, 40), (15, 20), (8, 10), (4, 5)]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(3)
    p = cnn.init_params(1)
    p = [q + 0.05 * rng.standard_normal(q.shape) for q in p]   # biases nonzero too
    x = rng.standard_normal((2, 5, 60, 80))
    xi, cache = cnn.forward(p, x)
    label = xi + 0.01 * rng.standard_normal((2, 6))      # a loss of order 1 keeps FD rounding low
    g = cnn.backward(p, cache, xi, label)
    for k in range(12):
        flat = p[k].reshape(-1)
        idxs = rng.choice(flat.size, size=min(4, flat.size), replace=False)
        for i in idxs:
            an = g[k].reshape(-1)[i]
            best = np.inf
            for eps in (1e-4, 1e-5, 1e-6):   # the smallest error over a step sweep (ReLU kinks)
                old = flat[i]
                flat[i] = old + eps
                lp = cnn.loss(cnn.forward(p, x)[0], label)
                flat[i] = old - eps
                lm = cnn.loss(cnn.forward(p, x)[0], label)
                flat[i] = old
                best = min(best, abs((lp - lm) / (2 * eps) - an))
            assert best <= 1e-7 * max(1.0, abs(an)), (k, i, best, an)


def test_adam_first_step_is_sign_step():
    # first bias-corrected Adam step moves every coordinate by lr * g/(|g| + eps)
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    P, M, V = cnn.adam_step(p, g, [np.zeros(3)], [np.zeros(3)], t=1, lr=0.1)
    assert np.allclose(P[0], p[0] - 0.1 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)


def test_bf16_round_ties_to_even_and_matches_torch():
    one = 1.0
    u = 2.0 ** -7                       # bf16 spacing at 1
    vals = np.array([one, one + u / 2, one + 3 * u / 2, one + u / 2 + 2.0 ** -20, -2.5 - u / 4, 3.0e-5, 1e30])
    r = cnn.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == one + 2 * u and r[3] == one + u
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    a = np.concatenate([vals, rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000)])
    tb = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a), tb)


def test_bf16_storage_mode_stays_close_to_fp64():
    p = cnn.init_params(0)
    rng = np.random.default_rng(0)
    x = 1.0 + rng.random((2, 5, 60, 80))
    a, _ = cnn.forward(p, x)
    b, cache = cnn.forward(p, x, quant=cnn.bf16_round)
    assert np.abs(a - b).max() <= 3e-2 * np.abs(a).max()
    assert all(np.array_equal(cnn.bf16_round(h), h) for h in cache["acts"])
