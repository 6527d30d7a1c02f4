"""The allocation-free forward of the initialiser network
(xslam_cnn_forward_noalloc: activations in the library's fixed device array)
against the existing forward (xslam_cnn_forward, activations in the handle's
workspace): the same kernels, so the outputs are equal bit for bit, on two
calls in a row (the second with a smaller batch), on a handle whose own
workspace only fits one sample, and a batch beyond the array's maximum is
refused with a clear error."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_02187_amd import xslam as X  # noqa: E402


def _weights(n, seed=11):
    rng = np.random.default_rng(seed)
    return (0.1 * rng.standard_normal(n)).astype(np.float32)


def _inputs(n, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.rand((n, 5, 60, 80), generator=g, dtype=torch.float32) * 3.0
    return x.to("cuda:0")


def test_noalloc_forward_equals_forward_on_two_calls():
    cnn = X.Cnn(max_batch=32)
    cnn.set_weights(_weights(cnn.n_params))
    for n, seed in ((32, 1), (5, 2)):
        x = _inputs(n, seed)
        ref = cnn.forward(x)
        out = torch.full((n, 6), float("nan"), dtype=torch.float32, device="cuda:0")
        cnn.forward_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert torch.equal(out, ref), (n, (out - ref).abs().max().item())
    cnn.close()


def test_noalloc_forward_serves_batches_beyond_the_handle_workspace():
    big = X.Cnn(max_batch=32)
    small = X.Cnn(max_batch=1)
    w = _weights(big.n_params, seed=3)
    big.set_weights(w)
    small.set_weights(w)
    x = _inputs(16, 7)
    ref = big.forward(x)
    out = torch.empty((16, 6), dtype=torch.float32, device="cuda:0")
    small.forward_noalloc(x, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    with pytest.raises(X.XslamError, match="-2"):
        small.forward_noalloc(_inputs(33, 8), torch.empty((33, 6), dtype=torch.float32, device="cuda:0"))
    big.close()
    small.close()
