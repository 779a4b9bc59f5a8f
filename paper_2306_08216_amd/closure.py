"""Learned coarse-grid closure (a project addition): a small periodic CNN,
evaluated and trained through the library's BF16 matrix-core kernels, that
corrects the velocity of a coarse MDF-FDLBM run toward the fine-grid solution.

Every arithmetic step runs in libmdf.so; this module allocates device memory
(PyTorch), marshals arguments and orchestrates data generation and training.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from . import problems as P
from .solver import Solver

CHANNELS = (2, 32, 32, 32, 2)
IN_SCALE = 20.0      # (u, v) ~ 0.05 -> O(1) inputs
OUT_SCALE = 1.0e-3   # corrections ~ 1e-4 .. 1e-3 -> O(1) outputs


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
                     div_tol: float):
    """Guarded correction of a periodic run; returns (ke, div, fell_back)."""
    return L.mdf_closure_apply(solver.ctx, du.data_ptr() if du is not None else None,
                               dv.data_ptr() if dv is not None else None, ke_ref, div_tol)
