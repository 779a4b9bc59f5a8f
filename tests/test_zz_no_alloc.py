"""The closure's forward pass without allocation (mdf_cnn_forward_noalloc, on
the library's fixed device scratch) against mdf_cnn_forward on a caller
workspace, through the C ABI: identical outputs on two calls in a row, the
second with a smaller input; inputs past the fixed limit are rejected."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _forward_ws(L, torch, params, uv, B, H, W, stream):
    nb = L.mdf_cnn_workspace_size(B, H, W)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    out = torch.empty((B, 2, H, W), dtype=torch.float64, device="cuda:0")
    L.mdf_cnn_forward(ws.data_ptr(), nb, params.data_ptr(), B, H, W, uv.data_ptr(), 20.0, 1e-4, out.data_ptr(),
                      stream)
    return out


def test_noalloc_forward_matches_workspace_forward():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08216_amd import _lib as L
    npar = L.mdf_cnn_param_count()
    rng = np.random.default_rng(5)
    params = torch.from_numpy(rng.standard_normal(npar).astype(np.float32) * 0.2).to("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    for B, H, W in ((1, 128, 128), (2, 40, 64)):          # the full limit, then a smaller input
        say(f"[gpu no-alloc] forward B={B} H={H} W={W}")
        uv = torch.from_numpy(rng.standard_normal((B, 2, H, W)) * 0.02).to("cuda:0")
        ref = _forward_ws(L, torch, params, uv, B, H, W, stream)
        out = torch.full((B, 2, H, W), float("nan"), dtype=torch.float64, device="cuda:0")
        L.mdf_cnn_forward_noalloc(params.data_ptr(), B, H, W, uv.data_ptr(), 20.0, 1e-4, out.data_ptr(), stream)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        say(f"    max|d| = {np.abs(a - b).max():.3e}, max|ref| = {np.abs(b).max():.3e}")
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)


def test_noalloc_forward_rejects_inputs_past_its_limit():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08216_amd import _lib as L
    params = torch.zeros(L.mdf_cnn_param_count(), dtype=torch.float32, device="cuda:0")
    uv = torch.zeros((2, 2, 128, 128), dtype=torch.float64, device="cuda:0")
    out = torch.zeros_like(uv)
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(L.MdfError):
        L.mdf_cnn_forward_noalloc(params.data_ptr(), 2, 128, 128, uv.data_ptr(), 1.0, 1.0, out.data_ptr(), stream)
    with pytest.raises(L.MdfError):
        L.mdf_cnn_forward_noalloc(params.data_ptr(), 1, 128, 100, uv.data_ptr(), 1.0, 1.0, out.data_ptr(), stream)
    assert float(out.abs().max()) == 0.0
