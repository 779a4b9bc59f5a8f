"""GPU checks of the learned closure against the CPU oracle (oracle/cnn_oracle.c):
each convolution layer on identical BF16 operands (FP32-accumulation bound),
the whole network and its gradient against FP64 at BF16 accuracy, Adam, the
correction step of eq. 2.2.5 on an MDF state, the guard, and training."""
import sys

import numpy as np
import pytest

from paper_2306_08216_amd import problems as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08216_amd import closure
    return closure


def _uv(B, H, W, seed=0, amp=0.05):
    rng = np.random.default_rng(seed)
    x = np.arange(W) * 2 * np.pi / W
    y = np.arange(H) * 2 * np.pi / H
    X, Y = np.meshgrid(x, y, indexing="xy")
    uv = np.zeros((B, 2, H, W))
    for b in range(B):
        for _ in range(5):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi, size=2)
            uv[b, 0] += amp / 3 * np.sin(kx * X + ky * Y + ph[0])
            uv[b, 1] += amp / 3 * np.cos(kx * X - ky * Y + ph[1])
        uv[b] += rng.normal(size=(2, H, W)) * amp * 0.05
    return uv


def _bf16_to_f64(a16):
    """int16 BF16 patterns -> float64."""
    u = (np.asarray(a16).astype(np.int32) & 0xFFFF).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("B,H,W", [(1, 8, 32), (2, 5, 64)])
def test_each_layer_matches_oracle_on_identical_bf16_operands(gpu, B, H, W):
    import torch
    from oracle import orc
    say(f"[gpu closure] layers B={B} H={H} W={W}")
    net = gpu.ClosureNet(H, W, B, seed=3)
    p = gpu.init_params(3, last_scale=1.0)
    rng = np.random.default_rng(9)
    for ws, bs, _, _ in gpu.layer_slices():
        p[bs] = rng.normal(size=bs.stop - bs.start).astype(np.float32) * 0.1
    net.params.copy_(torch.as_tensor(p))
    uv = torch.as_tensor(_uv(B, H, W, seed=1)).cuda()
    net.forward(uv)
    torch.cuda.synchronize()
    for layer, (ws, bs, cin, cout) in enumerate(gpu.layer_slices(), start=1):
        a16, z, _, _ = net.layer_io(layer)
        a = _bf16_to_f64(a16.cpu().numpy())[:, :cin].reshape(B, H, W, cin)
        w = orc.cnn_bf16_array(p[ws].astype(np.float64)).reshape(9, cin, cout)
        bias = p[bs].astype(np.float64)
        ref = orc.cnn_conv3x3(a, w, bias)
        mag = orc.cnn_conv3x3(np.abs(a), np.abs(w), np.abs(bias))
        zg = z.cpu().numpy().astype(np.float64)[:, :cout].reshape(B, H, W, cout)
        K = 9 * cin
        bound = 2 * K * 2.0 ** -24 * mag + 1e-30
        err = np.abs(zg - ref)
        say(f"    layer {layer}: max err {err.max():.3e}, max err/bound {(err / bound).max():.3f}")
        assert np.all(err <= bound)


def _shift(a, B, H, W, dy, dx):
    """a[p + (dy, dx)] per image (periodic), a: [P, C] channels last."""
    A = a.reshape(B, H, W, -1)
    return np.roll(A, shift=(-dy, -dx), axis=(1, 2)).reshape(B * H * W, -1)


def _run_net(gpu, B, H, W, seed):
    import torch
    net = gpu.ClosureNet(H, W, B, seed=seed)
    p = gpu.init_params(seed, last_scale=1.0)
    rng = np.random.default_rng(seed + 100)
    for ws, bs, _, _ in gpu.layer_slices():
        p[bs] = rng.normal(size=bs.stop - bs.start).astype(np.float32) * 0.05
    net.params.copy_(torch.as_tensor(p))
    uv = torch.as_tensor(_uv(B, H, W, seed=seed + 1)).cuda()
    target = torch.as_tensor(_uv(B, H, W, seed=seed + 2, amp=1e-3)).cuda()
    duv = net.forward(uv)
    loss = net.backward(target)
    torch.cuda.synchronize()
    return net, p, uv, target, duv, loss


def test_backward_kernels_on_identical_operands(gpu):
    """Each backward GEMM against the oracle's sums on the GPU's own BF16
    operands: weight gradient sum_p a[p + o_t][ci] g[p][co], bias gradient
    sum_p g[p][co], and the data gradient through the mirrored taps times
    the ReLU mask; FP32-accumulation bounds 2 K 2^-24 sum|terms|."""
    from oracle import orc
    B, H, W = 2, 6, 32
    Pn = B * H * W
    say("[gpu closure] backward kernels on identical operands")
    net, p, uv, target, duv, loss = _run_net(gpu, B, H, W, 21)
    grad = net.grad.cpu().numpy().astype(np.float64)
    io = {l: [t.cpu().numpy() for t in net.layer_io(l)] for l in (1, 2, 3, 4)}
    u = 2.0 ** -24
    for l, (ws, bs, cin, cout) in enumerate(gpu.layer_slices(), start=1):
        a16, _, g16, g32 = io[l]
        a = _bf16_to_f64(a16)[:, :cin]
        g = _bf16_to_f64(g16)[:, :cout]
        gw = grad[ws].reshape(9, cin, cout)
        for t in range(9):
            at = _shift(a, B, H, W, t // 3 - 1, t % 3 - 1)
            ref = at.T @ g
            mag = np.abs(at).T @ np.abs(g)
            err = np.abs(gw[t] - ref)
            assert np.all(err <= 2 * Pn * u * mag + 1e-30), (l, t, (err / (2 * Pn * u * mag + 1e-30)).max())
        gb = grad[bs]
        refb = g32[:, :cout].astype(np.float64).sum(0)
        magb = np.abs(g32[:, :cout].astype(np.float64)).sum(0)
        assert np.all(np.abs(gb - refb) <= 2 * Pn * u * magb + 1e-30)
        if l == 1:
            continue
        # data gradient into layer l-1's output
        _, zprev, _, gprev32 = io[l - 1]
        wbf = orc.cnn_bf16_array(p[ws].astype(np.float64)).reshape(9, cin, cout)
        wm = np.ascontiguousarray(wbf[::-1].transpose(0, 2, 1))        # [t][co][ci] = W[8 - t][ci][co]
        gin = g.reshape(B, H, W, cout)
        ref = orc.cnn_conv3x3(gin, wm).reshape(Pn, cin)
        mag = orc.cnn_conv3x3(np.abs(gin), np.abs(wm)).reshape(Pn, cin)
        mask = zprev[:, :cin] > 0
        ref = np.where(mask, ref, 0.0)
        got = gprev32[:, :cin].astype(np.float64)
        bound = 2 * 9 * cout * u * mag + 1e-30
        err = np.abs(got - ref)
        say(f"    layer {l}: data grad max err/bound {(err / bound).max():.3f}")
        assert np.all(err <= bound)


def test_network_end_to_end_bf16_accuracy(gpu):
    """The whole BF16 network and its gradient against the FP64 oracle on the
    unrounded parameters: BF16 operands (8 significant bits) through four
    layers give forward errors near 1e-2; gradients are compared normwise
    and by direction."""
    from oracle import orc
    B, H, W = 2, 6, 32
    say("[gpu closure] forward + backward vs FP64 oracle")
    net, p, uv, target, duv, loss = _run_net(gpu, B, H, W, 5)
    x = (gpu.IN_SCALE * uv.cpu().numpy()).transpose(0, 2, 3, 1)
    t = (target.cpu().numpy() / gpu.OUT_SCALE).transpose(0, 2, 3, 1)
    y_ref = orc.cnn_forward(p.astype(np.float64), x)
    y_gpu = (duv.cpu().numpy() / gpu.OUT_SCALE).transpose(0, 2, 3, 1)
    rel = np.linalg.norm(y_gpu - y_ref) / np.linalg.norm(y_ref)
    say(f"    forward normwise rel err {rel:.3e}")
    assert rel <= 2e-2
    l_ref, g_ref = orc.cnn_loss_grad(p.astype(np.float64), x, t)
    assert float(loss.item()) == pytest.approx(l_ref, rel=2e-2)
    g = net.grad.cpu().numpy().astype(np.float64)
    for l, (ws, bs, _, _) in enumerate(gpu.layer_slices(), start=1):
        for sl, nm in ((ws, "W"), (bs, "b")):
            a, r = g[sl], g_ref[sl]
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = a @ r / (np.linalg.norm(a) * np.linalg.norm(r))
            say(f"    layer {l} grad {nm}: rel {rel:.3e} cos {cos:.6f}")
            assert rel <= 5e-2 and cos >= 0.999
    # determinism: the same backward twice gives the same bits
    g1 = net.grad.clone()
    net.forward(uv)
    net.backward(target)
    import torch
    torch.cuda.synchronize()
    assert torch.equal(g1, net.grad)


def test_adam_step(gpu):
    import torch
    net = gpu.ClosureNet(4, 32, 1, seed=1)
    rng = np.random.default_rng(0)
    p0 = net.params.cpu().numpy().copy()
    g = rng.normal(size=net.n).astype(np.float32)
    net.grad.copy_(torch.as_tensor(g))
    net.adam(lr=1e-2)
    torch.cuda.synchronize()
    m = 0.1 * g
    v = 0.001 * g * g
    ref = p0 - 1e-2 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert np.allclose(net.params.cpu().numpy(), ref, rtol=1e-5, atol=1e-7)


def test_correction_step_and_guard(gpu):
    import torch
    from oracle import orc
    from paper_2306_08216_amd.solver import Solver
    prob = P.random_vortex(64, 3, 1e-3, kmax=6, urms=0.05)
    s = Solver(prob)
    s.step(10)
    f0 = s.save().cpu().numpy()
    u0, v0, _ = (t.cpu().numpy() for t in s.moments())
    rng = np.random.default_rng(1)
    du = torch.as_tensor(rng.normal(size=(64, 64)) * 1e-4).cuda()
    dv = torch.as_tensor(rng.normal(size=(64, 64)) * 1e-4).cuda()
    ke, div, fb = gpu.apply_correction(s, None, None, 0.0, 0.0)          # measure only
    assert not fb and ke == pytest.approx(0.5 * np.sum(u0 * u0 + v0 * v0), rel=1e-13) and div > 0
    dun, dvn = du.cpu().numpy(), dv.cpu().numpy()
    ke_c = 0.5 * np.sum((u0 + dun) ** 2 + (v0 + dvn) ** 2)
    # energy above the reference: no change at all
    ke1, div1, fb1 = gpu.apply_correction(s, du, dv, ke_ref=0.5 * ke_c, div_factor=1e9)
    assert fb1 and ke1 == ke and div1 == div and np.array_equal(s.save().cpu().numpy(), f0)
    # divergence limit below the corrected field's: no change
    _, _, fb2 = gpu.apply_correction(s, du, dv, ke_ref=2 * ke_c, div_factor=1e-6)
    assert fb2 and np.array_equal(s.save().cpu().numpy(), f0)
    # accepted: f + f^eq(u + du, P) - f^eq(u, P) as the oracle computes it
    ke3, div3, fb3 = gpu.apply_correction(s, du, dv, ke_ref=2 * ke_c, div_factor=1e9)
    assert not fb3 and ke3 == pytest.approx(ke_c, rel=1e-12)
    ref = orc.cnn_apply_correction(f0, dun, dvn, c=prob.c)
    got = s.save().cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-15
    u, v, _ = (t.cpu().numpy() for t in s.moments())
    assert np.abs(u - (u0 + dun)).max() <= 1e-15 and np.abs(v - (v0 + dvn)).max() <= 1e-15
    s.close()


def test_training_reduces_loss(gpu):
    """Fit the corrections of a fixed smooth map on a few fields: the loss falls."""
    import torch
    B, H, W = 4, 32, 32
    net = gpu.ClosureNet(H, W, B, seed=11)
    uv = torch.as_tensor(_uv(B, H, W, seed=7)).cuda()
    target = (torch.roll(uv, 1, dims=3) - uv) * 0.02       # a local linear map of the input
    losses = []
    for it in range(150):
        net.forward(uv)
        losses.append(float(net.backward(target).item()))
        net.adam(lr=2e-3)
    torch.cuda.synchronize()
    say(f"[gpu closure] training loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.2 * losses[0]


def test_trained_closure_gains_over_plain_coarse_run(gpu):
    """What the trained network gains: an under-resolved coarse run (64^2,
    nu = 1e-4, modes |k| <= 24, u_rms 0.1) against the same flow on 256^2
    restricted to the coarse nodes.  Trained on 8 seeds of runs the method
    generates, tested on 2 others over 800 coarse steps with the guarded
    correction every 4 steps; the closure must cut the relative L2 error of
    (u, v) by at least 15 % on each test seed."""
    res = gpu.experiment(list(range(8)), [1000, 1001], n_coarse=64, ratio=4, nu=1e-4, K=4, windows=200,
                         horizon=800, kmax=24, urms=0.1, batch=8, iters=1500, lr=1e-3)
    for row in res["test"]:
        say(f"[gpu closure] seed {row['seed']}: plain {row['plain_rel_l2']:.4f} closure {row['closure_rel_l2']:.4f} "
            f"fallbacks {row['fallbacks']}/{row['windows']} t_fine {row['t_fine_s']:.3f}s t_closure "
            f"{row['t_closure_s']:.3f}s")
        assert row["closure_rel_l2"] < 0.85 * row["plain_rel_l2"]
        assert row["windows"] == 200


def test_device_guard_matches_host_guard(gpu):
    """The guarded correction decided on the device (mdf_closure_begin /
    mdf_closure_apply_async / mdf_closure_stats, no host synchronisation)
    leaves the same state and counts the same fall-backs as the host-decided
    mdf_closure_apply over the same windows, accepted and refused ones alike."""
    import torch
    from paper_2306_08216_amd import _lib as L
    from paper_2306_08216_amd.solver import Solver
    prob = P.random_vortex(64, 5, 1e-3, kmax=6, urms=0.05)
    a, b = Solver(prob), Solver(prob)
    ke_ref, _, _ = gpu.apply_correction(a, None, None, 0.0, 0.0)
    L.mdf_closure_begin(b.ctx)
    fallbacks = 0
    for w in range(12):
        for s in (a, b):
            s.step(3)
        u, v, _ = a.moments()
        sign = -1.0 if w % 3 != 1 else 1.0            # damping corrections pass, amplifying ones are refused
        du = (sign * 1e-3 * u).contiguous()
        dv = (sign * 1e-3 * v).contiguous()
        ke_ref, _, fb = gpu.apply_correction(a, du, dv, ke_ref, 2.0)
        fallbacks += int(fb)
        L.mdf_closure_apply_async(b.ctx, du.data_ptr(), dv.data_ptr(), 2.0)
    ke_b, fb_b, windows = L.mdf_closure_stats(b.ctx)
    say(f"[gpu closure] device guard: fallbacks host {fallbacks} device {fb_b} of {windows}")
    assert windows == 12 and fb_b == fallbacks and 0 < fallbacks < 12
    assert ke_b == ke_ref
    assert np.array_equal(a.save().cpu().numpy(), b.save().cpu().numpy())
    a.close()
    b.close()
    del torch


def test_captured_window_replays_match_eager_windows(gpu):
    """A closure window captured as a HIP graph (K steps, the velocity, the
    network, the guarded apply) and replayed gives, after every replay, exactly
    the state and fall-back count of the same window launched eagerly on a
    twin run; eager work on the replayed run's stream and synchronisations sit
    between the replays.  The two runs take turns (they share the network's
    fixed scratch array)."""
    import torch
    from paper_2306_08216_amd import _lib as L
    from paper_2306_08216_amd.solver import Solver
    prob = P.random_vortex(64, 11, 1e-4, kmax=24, urms=0.1)
    net = gpu.ClosureNet(64, 64, 1, params=gpu.init_params(3, last_scale=1.0))
    a = Solver(prob, stream=torch.cuda.Stream())
    b = Solver(prob, stream=torch.cuda.Stream())
    wa = gpu._Window(a, net, 4, 1.0, 2.0, graph=False)
    wb = gpu._Window(b, net, 4, 1.0, 2.0, graph=True)
    L.mdf_closure_begin(a.ctx)
    L.mdf_closure_begin(b.ctx)
    torch.cuda.synchronize()
    for w in range(6):
        wa()
        torch.cuda.synchronize()
        wb()
        torch.cuda.synchronize()
        fa, fb = a.save().cpu().numpy(), b.save().cpu().numpy()
        say(f"[gpu closure] replay {w}: max|f_graph - f_eager| = {np.abs(fa - fb).max():.3e}")
        assert np.array_equal(fa, fb), w
        assert L.mdf_closure_stats(a.ctx)[:2] == L.mdf_closure_stats(b.ctx)[:2]
        b.moments()                      # eager work on the replayed run's stream
        torch.cuda.synchronize()
    a.close()
    b.close()


def test_graph_rollout_matches_eager_rollout(gpu):
    """The evaluation rollout replaying captured graphs (fine run, plain coarse
    run and closure windows) ends on the same fields as the eager rollout."""
    net = gpu.ClosureNet(64, 64, 1, params=gpu.init_params(5, last_scale=0.3))
    kw = dict(n_coarse=64, ratio=2, nu=1e-4, K=4, steps=40, kmax=16, urms=0.05)
    for model in (None, net):
        r_e = gpu.rollout(21, model, graph=False, **kw)
        r_g = gpu.rollout(21, model, graph=True, **kw)
        say(f"[gpu closure] rollout {'closure' if model else 'plain'}: eager {r_e['rel_l2']:.6e} graph {r_g['rel_l2']:.6e}")
        assert r_e["rel_l2"] == r_g["rel_l2"]
        assert r_e["fallbacks"] == r_g["fallbacks"]
        for x, y in zip(r_e["fine_ref"][:2], r_g["fine_ref"][:2]):
            assert bool((x == y).all())
