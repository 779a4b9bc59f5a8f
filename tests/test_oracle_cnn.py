"""Pins of the closure network's CPU oracle against definitions it does not
share code with: a library periodic correlation, central finite differences
of its own loss, torch's bfloat16 rounding, and the moment identities of the
MDF equilibrium (eq. 2.2.5) for the correction step."""
import numpy as np
import pytest

from oracle import orc


def _params(seed=0, scale=0.2):
    rng = np.random.default_rng(seed)
    p = np.zeros(orc.cnn_param_count())
    for ws, bs, cin, cout in orc.cnn_layer_slices():
        p[ws] = rng.normal(size=ws.stop - ws.start) * scale / np.sqrt(9 * cin)
        p[bs] = rng.normal(size=bs.stop - bs.start) * 0.05
    return p


def test_param_count():
    assert orc.cnn_param_count() == 9 * (2 * 32 + 32 * 32 + 32 * 32 + 32 * 2) + 32 + 32 + 32 + 2


def test_conv_matches_library_periodic_correlation():
    """z[y, x, co] = b + sum_{dy, dx, ci} w a[y + dy, x + dx, ci] with wrap-around:
    per (ci, co) a periodic cross-correlation (scipy.ndimage, mode 'wrap')."""
    from scipy import ndimage
    rng = np.random.default_rng(1)
    B, H, W, cin, cout = 2, 7, 9, 3, 4
    a = rng.normal(size=(B, H, W, cin))
    w = rng.normal(size=(9, cin, cout))
    b = rng.normal(size=cout)
    z = orc.cnn_conv3x3(a, w, b)
    ref = np.zeros_like(z)
    for bb in range(B):
        for ci in range(cin):
            for co in range(cout):
                k = w[:, ci, co].reshape(3, 3)          # k[dy + 1, dx + 1]
                ref[bb, :, :, co] += ndimage.correlate(a[bb, :, :, ci], k, mode="wrap")
    ref += b
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


def test_centre_tap_identity():
    """A kernel with only the centre tap = I copies the input."""
    rng = np.random.default_rng(2)
    a = rng.normal(size=(1, 5, 6, 3))
    w = np.zeros((9, 3, 3))
    w[4] = np.eye(3)
    assert np.array_equal(orc.cnn_conv3x3(a, w), a)


def test_gradient_matches_central_differences():
    """Backpropagation against FP64 central differences of the same loss."""
    rng = np.random.default_rng(3)
    p = _params(3)
    B, H, W = 1, 6, 5
    x = rng.normal(size=(B, H, W, 2))
    t = rng.normal(size=(B, H, W, 2)) * 0.1
    loss, g = orc.cnn_loss_grad(p, x, t)
    assert loss == pytest.approx(np.mean((orc.cnn_forward(p, x) - t) ** 2), rel=1e-14)
    idx = []
    for ws, bs, _, _ in orc.cnn_layer_slices():
        idx += list(rng.choice(np.arange(ws.start, ws.stop), 6, replace=False)) + [bs.start, bs.stop - 1]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (orc.cnn_loss_grad(pp, x, t)[0] - orc.cnn_loss_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-8) + 1e-11, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(4)
    v = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.uniform(-8, 8, size=2000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, 3.0e38, 1e-40]])
    mine = orc.cnn_bf16_array(v)
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mine, ref)


def test_correction_sets_velocity_and_keeps_pressure():
    """f + f^eq(u + du, P) - f^eq(u, P): the zeroth moments become u + du and
    v + dv exactly (sum_j f^eq_j = u_a) and the pressure identity returns P."""
    rng = np.random.default_rng(5)
    ny, nx = 6, 7
    f = rng.normal(size=(10, ny, nx)) * 0.05
    du = rng.normal(size=(ny, nx)) * 1e-3
    dv = rng.normal(size=(ny, nx)) * 1e-3
    g = orc.cnn_apply_correction(f, du, dv, c=1.0)

    def mom(ff):
        u = ff[0:5].sum(0)
        v = ff[5:10].sum(0)
        P = 0.5 * ((ff[1] - ff[3] + ff[7] - ff[9]) - (u * u + v * v))
        return u, v, P
    u0, v0, P0 = mom(f)
    u1, v1, P1 = mom(g)
    assert np.abs(u1 - (u0 + du)).max() <= 1e-15 and np.abs(v1 - (v0 + dv)).max() <= 1e-15
    assert np.abs(P1 - P0).max() <= 1e-15
    # no correction, no change
    assert np.array_equal(orc.cnn_apply_correction(f, 0 * du, 0 * dv), f)
