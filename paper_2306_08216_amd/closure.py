"""Learned coarse-grid closure (a project addition): a small periodic CNN,
evaluated and trained through the library's BF16 matrix-core kernels, that
corrects the velocity of a coarse MDF-FDLBM run toward the fine-grid solution.

Every arithmetic step runs in libmdf.so; this module allocates device memory
(PyTorch), marshals arguments and orchestrates data generation and training.
"""
from __future__ import annotations

import math
import sys
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from . import problems as P
from .solver import Solver

CHANNELS = (2, 32, 32, 32, 2)
NOALLOC_MAX_PIXELS = 16384   # batch*h*w limit of mdf_cnn_forward_noalloc (MDF_CNN_NOALLOC_MAX_PIXELS)
IN_SCALE = 20.0      # (u, v) ~ 0.05 -> O(1) inputs
OUT_SCALE = 1.0e-4   # one-window corrections ~ 1e-5 .. 1e-4 -> O(1) outputs


def layer_slices():
    out, o = [], 0
    for l in range(4):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        nw = 9 * cin * cout
        out.append((slice(o, o + nw), slice(o + nw, o + nw + cout), cin, cout))
        o += nw + cout
    return out


def init_params(seed: int = 0, last_scale: float = 0.1) -> np.ndarray:
    """He-normal weights, zero biases; the last layer starts small so the
    untrained closure is a near-zero correction."""
    rng = np.random.default_rng(seed)
    p = np.zeros(L.mdf_cnn_param_count(), dtype=np.float32)
    for l, (ws, bs, cin, cout) in enumerate(layer_slices()):
        std = math.sqrt(2.0 / (9 * cin)) * (last_scale if l == 3 else 1.0)
        p[ws] = rng.normal(size=ws.stop - ws.start) * std
    return p


class ClosureNet:
    """The network on one device, with a workspace for batches of (batch, h, w)."""

    def __init__(self, h: int, w: int, batch: int = 1, params: Optional[np.ndarray] = None, device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, seed: int = 0):
        L.lib()
        self.device = torch.device(device)
        self.h, self.w, self.batch = h, w, batch
        self.n = L.mdf_cnn_param_count()
        self.ws_bytes = L.mdf_cnn_workspace_size(batch, h, w)
        if self.ws_bytes == 0:
            raise L.MdfError(L.MDF_EINVAL, "closure needs w a multiple of 32 and h >= 3")
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws = (self._ws.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.as_tensor(p.copy()).to(self.device)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.adam_steps = 0

    def forward(self, uv: torch.Tensor) -> torch.Tensor:
        """uv: [batch, 2, h, w] FP64 device -> (du, dv) [batch, 2, h, w] FP64."""
        assert uv.dtype == torch.float64 and uv.is_contiguous() and tuple(uv.shape) == (self.batch, 2, self.h, self.w)
        out = torch.empty_like(uv)
        L.mdf_cnn_forward(self.ws, self.ws_bytes, self.params.data_ptr(), self.batch, self.h, self.w, uv.data_ptr(),
                          IN_SCALE, OUT_SCALE, out.data_ptr(), self.stream.cuda_stream)
        return out

    def backward(self, target: torch.Tensor) -> float:
        """Gradient of the mean squared error against target corrections
        [batch, 2, h, w] for the last forward call; returns the loss."""
        assert target.dtype == torch.float64 and target.is_contiguous()
        L.mdf_cnn_backward(self.ws, self.ws_bytes, self.params.data_ptr(), self.batch, self.h, self.w,
                           target.data_ptr(), OUT_SCALE, self.grad.data_ptr(), self.loss_dev.data_ptr(),
                           self.stream.cuda_stream)
        return self.loss_dev

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.adam_steps += 1
        L.mdf_cnn_adam(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.n,
                       lr, beta1, beta2, eps, self.adam_steps, self.stream.cuda_stream)

    def layer_io(self, layer: int):
        """(BF16 input, FP32 pre-activation, BF16 and FP32 loss gradient at it) of a layer."""
        P_ = self.batch * self.h * self.w
        cin = 8 if layer == 1 else 32
        a = torch.empty((P_, cin), dtype=torch.int16, device=self.device)
        z = torch.empty((P_, 2 if layer == 4 else 32), dtype=torch.float32, device=self.device)
        g16 = torch.empty((P_, 32), dtype=torch.int16, device=self.device)
        g32 = torch.empty((P_, 32), dtype=torch.float32, device=self.device)
        L.mdf_cnn_layer_io(self.ws, self.ws_bytes, self.batch, self.h, self.w, layer, a.data_ptr(), z.data_ptr(),
                           g16.data_ptr(), g32.data_ptr(), self.stream.cuda_stream)
        return a, z, g16, g32

    def save(self, path: str):
        np.savez(path, params=self.params.cpu().numpy())

    @staticmethod
    def load_params(path: str) -> np.ndarray:
        with np.load(path, allow_pickle=False) as d:
            return d["params"].astype(np.float32)


def apply_correction(solver: Solver, du: Optional[torch.Tensor], dv: Optional[torch.Tensor], ke_ref: float,
                     div_factor: float):
    """Guarded correction of a periodic run; returns (ke, div, fell_back) of the field it leaves."""
    return L.mdf_closure_apply(solver.ctx, du.data_ptr() if du is not None else None,
                               dv.data_ptr() if dv is not None else None, ke_ref, div_factor)


# ---- experiment: data from the method itself, training, guarded rollout ------

def restrict(a: torch.Tensor, r: int) -> torch.Tensor:
    """Coincident-node injection: fine node r*I is coarse node I."""
    return a[::r, ::r].contiguous()


def _coarse_problem(fine: P.Problem, r: int) -> P.Problem:
    n = fine.nx // r
    return P.Problem(nx=n, ny=n, lx=fine.lx, ly=fine.ly, nu=fine.nu, u0=fine.u0[::r, ::r].copy(),
                     v0=fine.v0[::r, ::r].copy(), p0=fine.p0[::r, ::r].copy(), cfl=fine.cfl, eta=fine.eta,
                     s_ratio=fine.s_ratio, name=f"coarse_of_{fine.name}")


def make_pairs(seeds: Sequence[int], n_coarse: int = 128, ratio: int = 4, nu: float = 1e-3, K: int = 4,
               windows: int = 100, kmax: int = 16, urms: float = 0.05):
    """Training pairs generated by the method, as the closure meets them in a
    run: the coarse run keeps its own state and, at the start of every
    window, has its velocity set to the restricted fine velocity through the
    same correction step the closure uses (non-equilibrium parts kept); it
    then takes K steps (the same physical time as K*ratio fine steps at fixed
    CFL) and its velocity is paired with the restricted fine velocity minus it."""
    inputs, targets = [], []
    nf = n_coarse * ratio
    for si, sd in enumerate(seeds):
        if si % 8 == 0:
            print(f"closure pairs: seed {si + 1}/{len(seeds)}", file=sys.stderr, flush=True)
        pf = P.random_vortex(nf, sd, nu, kmax=kmax, urms=urms)
        fine = Solver(pf)
        coarse = Solver(_coarse_problem(pf, ratio))
        for w in range(windows):
            if w > 0:
                uf, vf, _ = fine.moments()
                uc, vc, _ = coarse.moments()
                apply_correction(coarse, (restrict(uf, ratio) - uc).contiguous(),
                                 (restrict(vf, ratio) - vc).contiguous(), math.inf, math.inf)
            coarse.step(K)
            fine.step(K * ratio)
            uc, vc, _ = coarse.moments()
            uf2, vf2, _ = fine.moments()
            inputs.append(torch.stack([uc, vc]))
            targets.append(torch.stack([restrict(uf2, ratio) - uc, restrict(vf2, ratio) - vc]))
        fine.close()
        coarse.close()
    return torch.stack(inputs).contiguous(), torch.stack(targets).contiguous()


def train(net: ClosureNet, inputs: torch.Tensor, targets: torch.Tensor, iters: int = 2000, lr: float = 1e-3,
          seed: int = 0, log_every: int = 100):
    """Minibatch Adam on the mean squared correction error; returns the loss history."""
    rng = np.random.default_rng(seed)
    n = inputs.shape[0]
    hist = []
    for it in range(iters):
        idx = torch.as_tensor(rng.choice(n, size=net.batch, replace=n < net.batch), device=inputs.device)
        x = inputs.index_select(0, idx).contiguous()
        t = targets.index_select(0, idx).contiguous()
        net.forward(x)
        loss = net.backward(t)
        frac = it / max(iters - 1, 1)
        net.adam(lr=lr * (0.1 if frac > 0.7 else 1.0))
        if log_every and (it % log_every == 0 or it == iters - 1):
            hist.append((it, float(loss.item())))
            if it % (10 * log_every) == 0:
                print(f"closure training: iteration {it}/{iters} loss {hist[-1][1]:.4e}", file=sys.stderr, flush=True)
    return hist


class _Window:
    """One closure window on a coarse run: K steps, the velocity, the network's
    correction and the guarded apply, all on the run's stream (nothing waits
    for the device or allocates).  With graph=True the first call launches the
    window eagerly (every kernel and the network's scratch array are then set
    up), the second captures it as a HIP graph and every later call replays
    it; the step counter of the context counts the captured window once, and K
    must be even so that the state's ping-pong buffer is the same after every
    window."""

    def __init__(self, coarse: Solver, net: "ClosureNet", K: int, gain: float, div_factor: float, graph: bool):
        n = coarse.nx
        assert net.h == n and net.w == n
        self.coarse, self.net, self.K, self.gain, self.div_factor = coarse, net, K, gain, div_factor
        self.uv = torch.empty((1, 2, n, n), dtype=torch.float64, device=coarse.device)
        self.duv = torch.empty_like(self.uv)
        self.noalloc = n * n <= NOALLOC_MAX_PIXELS
        self.want_graph, self.graph, self.calls = graph, None, 0
        if graph and (K % 2 or not coarse.stream.cuda_stream):
            raise ValueError("a captured window needs an even K and a run on its own stream")

    def _launch(self):
        c, n, sc = self.coarse, self.coarse.nx, self.coarse.stream.cuda_stream
        c.step(self.K)
        L.mdf_moments(c.ctx, self.uv[0, 0].data_ptr(), self.uv[0, 1].data_ptr(), None)
        if self.noalloc:
            L.mdf_cnn_forward_noalloc(self.net.params.data_ptr(), 1, n, n, self.uv.data_ptr(), IN_SCALE,
                                      OUT_SCALE * self.gain, self.duv.data_ptr(), sc)
        else:
            L.mdf_cnn_forward(self.net.ws, self.net.ws_bytes, self.net.params.data_ptr(), 1, n, n,
                              self.uv.data_ptr(), IN_SCALE, OUT_SCALE * self.gain, self.duv.data_ptr(), sc)
        # guard: energy must not exceed the last check's, divergence at most div_factor x the plain field's
        L.mdf_closure_apply_async(c.ctx, self.duv[0, 0].data_ptr(), self.duv[0, 1].data_ptr(), self.div_factor)

    def __call__(self):
        self.calls += 1
        if not self.want_graph or self.calls == 1:
            self._launch()
            return
        if self.graph is None:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.coarse.stream):
                self._launch()
            self.graph = g
        with torch.cuda.stream(self.coarse.stream):
            self.graph.replay()


def _advance(solver: Solver, steps: int, chunk: int, graph: bool):
    """steps steps of a run; with graph=True the first `chunk` steps (even)
    eagerly, then replays of one captured graph of `chunk` steps, and the
    remainder eagerly."""
    if not graph or steps < 2 * chunk:
        solver.step(steps)
        return
    assert chunk % 2 == 0
    solver.step(chunk)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=solver.stream):
        solver.step(chunk)
    with torch.cuda.stream(solver.stream):
        for _ in range(steps // chunk - 1):
            g.replay()
    solver.step(steps % chunk)


def rollout(seed: int, net: Optional[ClosureNet], n_coarse: int = 128, ratio: int = 4, nu: float = 1e-3,
            K: int = 4, steps: int = 2000, kmax: int = 16, urms: float = 0.05, div_factor: float = 2.0,
            fine_ref: Optional[Tuple[torch.Tensor, torch.Tensor, float]] = None, gain: float = 1.0,
            graph: bool = False):
    """Coarse run from the restricted initial field, with the guarded closure
    every K steps when `net` is given, against the fine run restricted to the
    coarse nodes.  With graph=True every run (fine, plain coarse, coarse with
    the closure) replays captured graphs of K coarse (K * ratio fine) steps
    (the same fields; on one MI355X the wall times move by under 8 %: these
    runs are bound by the kernels' own duration, not by launching them).
    Returns a dict with
    the relative L2 error of (u, v) at the horizon, wall times, fall-backs and
    the fine reference for reuse."""
    nf = n_coarse * ratio
    pf = P.random_vortex(nf, seed, nu, kmax=kmax, urms=urms)
    if fine_ref is None:
        fine = Solver(pf, stream=torch.cuda.Stream() if graph else None)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(fine.stream)
        _advance(fine, steps * ratio, K * ratio, graph)
        t1.record(fine.stream)
        torch.cuda.synchronize()
        t_fine = t0.elapsed_time(t1) / 1e3
        uf, vf, _ = fine.moments()
        fine_ref = (restrict(uf, ratio), restrict(vf, ratio), t_fine)
        fine.close()
    ufr, vfr, t_fine = fine_ref
    coarse = Solver(_coarse_problem(pf, ratio), stream=torch.cuda.Stream() if graph else None)
    fallbacks = 0
    # the window (and its graph) is built before the timing: the loop itself
    # allocates nothing and never waits for the device
    window = _Window(coarse, net, K, gain, div_factor, graph) if net is not None else None
    torch.cuda.synchronize()
    w0 = torch.cuda.Event(enable_timing=True)
    w1 = torch.cuda.Event(enable_timing=True)
    w0.record(coarse.stream)
    if net is None:
        _advance(coarse, steps, K, graph)
    else:
        L.mdf_closure_begin(coarse.ctx)
        for _ in range(steps // K):
            window()
        coarse.step(steps % K)
    w1.record(coarse.stream)
    torch.cuda.synchronize()
    t_coarse = w0.elapsed_time(w1) / 1e3
    if net is not None:
        _, fallbacks, _ = L.mdf_closure_stats(coarse.ctx)
    uc, vc, _ = coarse.moments()
    err = math.sqrt(float(((uc - ufr) ** 2 + (vc - vfr) ** 2).sum()) / float((ufr ** 2 + vfr ** 2).sum()))
    coarse.close()
    return {"seed": seed, "rel_l2": err, "t_coarse_s": t_coarse, "t_fine_s": t_fine, "fallbacks": fallbacks,
            "windows": steps // K if net is not None else 0, "fine_ref": fine_ref}


def experiment(train_seeds: Sequence[int], test_seeds: Sequence[int], n_coarse: int = 128, ratio: int = 4,
               nu: float = 1e-3, K: int = 4, windows: int = 100, horizon: int = 2000, kmax: int = 16,
               urms: float = 0.05, batch: int = 8, iters: int = 2000, lr: float = 1e-3, seed: int = 0,
               params_out: Optional[str] = None, val_seeds: Sequence[int] = (), gains: Sequence[float] = (1.0,),
               graph: bool = False):
    """Generate pairs, train, pick the correction gain on validation seeds (if
    any), and evaluate plain coarse vs coarse + closure vs fine on held-out seeds."""
    x, t = make_pairs(train_seeds, n_coarse, ratio, nu, K, windows, kmax, urms)
    net = ClosureNet(n_coarse, n_coarse, batch, seed=seed)
    hist = train(net, x, t, iters, lr, seed)
    del x, t
    if params_out:
        net.save(params_out)
    infer = ClosureNet(n_coarse, n_coarse, 1, params=net.params.cpu().numpy())
    gain, val = 1.0, []
    if val_seeds and len(gains) > 1:
        refs = {sd: rollout(sd, None, n_coarse, ratio, nu, K, horizon, kmax, urms, graph=graph) for sd in val_seeds}
        for g in gains:
            e = [rollout(sd, infer if g != 0.0 else None, n_coarse, ratio, nu, K, horizon, kmax, urms,
                         fine_ref=refs[sd]["fine_ref"], gain=g, graph=graph)["rel_l2"] for sd in val_seeds]
            val.append((g, float(np.mean(e))))
        gain = min(val, key=lambda r: r[1])[0]
    print(f"closure validation: {val} -> gain {gain}", file=sys.stderr, flush=True)
    rows = []
    for sd in test_seeds:
        plain = rollout(sd, None, n_coarse, ratio, nu, K, horizon, kmax, urms, graph=graph)
        # gain 0 (chosen when the closure does not help on validation) switches it off
        corr = rollout(sd, infer if gain != 0.0 else None, n_coarse, ratio, nu, K, horizon, kmax, urms,
                       fine_ref=plain["fine_ref"], gain=gain, graph=graph)
        rows.append({"seed": sd, "plain_rel_l2": plain["rel_l2"], "closure_rel_l2": corr["rel_l2"],
                     "t_fine_s": plain["t_fine_s"], "t_plain_s": plain["t_coarse_s"],
                     "t_closure_s": corr["t_coarse_s"], "fallbacks": corr["fallbacks"], "windows": corr["windows"]})
    return {"pairs": len(train_seeds) * windows, "loss_history": hist, "validation": val, "gain": gain,
            "test": rows}


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and evaluate the learned coarse-grid closure")
    ap.add_argument("--n-coarse", type=int, default=128)
    ap.add_argument("--ratio", type=int, default=4)
    ap.add_argument("--nu", type=float, default=1e-3)
    ap.add_argument("--K", type=int, default=4)
    ap.add_argument("--windows", type=int, default=100, help="training windows per seed")
    ap.add_argument("--horizon", type=int, default=2000, help="coarse steps of each evaluation run")
    ap.add_argument("--kmax", type=int, default=16)
    ap.add_argument("--urms", type=float, default=0.05)
    ap.add_argument("--train-seeds", type=int, default=64)
    ap.add_argument("--test-seeds", type=int, default=8)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--params-out", default=None)
    ap.add_argument("--val-seeds", type=int, default=0, help="validation seeds for choosing the correction gain")
    ap.add_argument("--gains", default="1.0", help="comma-separated correction gains tried on the validation seeds")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured graphs in the evaluation runs instead of launching every kernel")
    a = ap.parse_args()
    res = experiment(list(range(a.train_seeds)), [1000 + i for i in range(a.test_seeds)], a.n_coarse, a.ratio, a.nu,
                     a.K, a.windows, a.horizon, a.kmax, a.urms, a.batch, a.iters, a.lr, params_out=a.params_out,
                     val_seeds=[2000 + i for i in range(a.val_seeds)],
                     gains=[float(g) for g in a.gains.split(",")], graph=a.graph)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
