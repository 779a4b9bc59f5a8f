"""Solver: one MDF-FDLBM run on the GPU through the C ABI.

PyTorch provides the device memory (workspace, field tensors) and the stream;
all arithmetic runs in the HIP kernels of libmdf.so.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .problems import Problem

DERIVED_NAMES = ["ux", "uy", "vx", "vy", "div", "Sxx", "Sxy", "Syy", "sig_xx", "sig_xy", "sig_yy",
                 "Omega_xy", "omega", "nu"]
DIAG_NAMES = ["sum_u", "sum_v", "ke", "enstrophy", "max_speed", "max_fd_div", "nonfinite", "area"]


def params_of(prob: Problem, keep: list) -> L.mdf_params:
    """Marshal a Problem into the C parameter struct (metric arrays stay owned by `keep`)."""
    def arr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))
    for f in (prob.force_x, prob.force_y):
        if f is not None and np.shape(f) != (prob.ny, prob.nx):
            raise ValueError("force fields must have shape (ny, nx)")
    if prob.metric is not None and np.shape(prob.metric) != (4, prob.ny, prob.nx):
        raise ValueError("a general mapping's metric must have shape (4, ny, nx)")
    if prob.mass_source is not None and np.shape(prob.mass_source) != (prob.ny, prob.nx):
        raise ValueError("a mass source must have shape (ny, nx)")
    return L.mdf_params(prob.nx, prob.ny, prob.lx, prob.ly, prob.nu, prob.pl_n, prob.nu_min, prob.nu_max,
                        prob.cfl, prob.c, prob.eta, prob.s_ratio, prob.bc_x, prob.bc_y, prob.lid_u,
                        prob.fx, prob.fy, arr(prob.inv_dx_x), arr(prob.inv_dx_y), prob.dx_min,
                        arr(prob.force_x), arr(prob.force_y), prob.force_omega, prob.force_phase,
                        int(prob.force_harmonic), arr(prob.metric), arr(prob.mass_source))


class Solver:
    def __init__(self, prob: Problem, device: str = "cuda:0", stream: Optional[torch.cuda.Stream] = None):
        L.lib()
        self.prob = prob
        self.device = torch.device(device)
        self.nx, self.ny = prob.nx, prob.ny
        keep: list = []
        self._p = params_of(prob, keep)
        nbytes = L.mdf_workspace_size(self._p)
        if nbytes == 0:
            raise L.MdfError(L.MDF_EINVAL, "invalid problem parameters")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.stream(self.stream):
            u0 = torch.as_tensor(np.ascontiguousarray(prob.u0), dtype=torch.float64).to(self.device)
            v0 = torch.as_tensor(np.ascontiguousarray(prob.v0), dtype=torch.float64).to(self.device)
            p0 = torch.as_tensor(np.ascontiguousarray(prob.p0), dtype=torch.float64).to(self.device)
        self.stream.synchronize()
        self.ctx = L.mdf_init(self._p, u0.data_ptr(), v0.data_ptr(), p0.data_ptr(), self.workspace.data_ptr(),
                              nbytes, self.stream.cuda_stream)
        del keep

    # -- life cycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            L.mdf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C calls ---------------------------------------------------------
    @property
    def dt(self) -> float:
        return L.mdf_dt(self.ctx)

    @property
    def steps(self) -> int:
        return L.mdf_steps(self.ctx)

    def set_kernel(self, variant: int, tile_w: int = 0, seg_h: int = 0, prefetch: int = 0):
        L.mdf_set_kernel(self.ctx, variant, tile_w, seg_h, prefetch)
        return self

    def autotune(self, steps: int = 10):
        """Pick the fastest fused kernel and partition for this run (state restored);
        returns (variant, prefetch, x-wall scale, y-wall scale, ms per step, tile_w)."""
        return L.mdf_autotune(self.ctx, steps)

    def signature(self) -> str:
        """Key of a tuning cache: grid, boundaries, fluid model, mapping and device
        (architecture and compute-unit count)."""
        p = self.prob
        props = torch.cuda.get_device_properties(self.device)
        dev = [str(getattr(props, "gcnArchName", "")).split(":")[0], int(props.multi_processor_count)]
        key = [p.nx, p.ny, p.bc_x, p.bc_y, p.pl_n, p.inv_dx_x is None and p.inv_dx_y is None, dev]
        return f"{p.nx}x{p.ny}-" + hashlib.sha256(json.dumps(key).encode()).hexdigest()[:16]

    def apply_choice(self, choice):
        """Select (variant, tile_w, prefetch, x-wall scale, y-wall scale) without timing anything."""
        variant, tile_w, prefetch, sx, sy = choice
        self.set_kernel(int(variant), int(tile_w), -1, int(prefetch))
        self.set_partition_costs(float(sx), float(sy))
        return self

    def tuned(self, cache_path: Optional[str] = None, steps: int = 10, retune: bool = False):
        """The kernel choice for this run from the tuning cache at `cache_path`
        (same signature), else from the autotuner, whose choice is then stored
        there.  Returns ((variant, tile_w, prefetch, x scale, y scale), cached)."""
        key = self.signature()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        if key in cache and not retune:
            choice = tuple(cache[key]["choice"])
            self.apply_choice(choice)
            return choice, True
        c = self.autotune(steps)
        choice = (int(c[0]), int(c[5]), int(c[1]), float(c[2]), float(c[3]))
        if cache_path:
            cache[key] = {"choice": list(choice), "nx": self.nx, "ny": self.ny, "ms_per_step": c[4]}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return choice, False

    def set_partition_costs(self, x_wall_scale: float, y_wall_scale: float):
        L.mdf_set_partition_costs(self.ctx, x_wall_scale, y_wall_scale)
        return self

    def set_fields(self, u: torch.Tensor, v: torch.Tensor, p: torch.Tensor):
        """Restart from (u, v, p) (device FP64 [ny, nx]): f_hat = f^eq at every node."""
        for t in (u, v, p):
            assert t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (self.ny, self.nx)
        L.mdf_set_fields(self.ctx, u.data_ptr(), v.data_ptr(), p.data_ptr())
        return self

    def step(self, n: int = 1):
        L.mdf_step(self.ctx, n)
        return self

    def moments(self):
        u = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        v = torch.empty_like(u)
        p = torch.empty_like(u)
        L.mdf_moments(self.ctx, u.data_ptr(), v.data_ptr(), p.data_ptr())
        return u, v, p

    def derived(self, mask: int = (1 << 14) - 1) -> torch.Tensor:
        k = bin(mask).count("1")
        out = torch.empty((k, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.mdf_derived(self.ctx, out.data_ptr(), mask)
        return out

    def diagnostics(self):
        buf = (C.c_double * 8)()
        status = L.mdf_diagnostics(self.ctx, buf)
        return np.array(buf[:]), status

    def save(self) -> torch.Tensor:
        f = torch.empty((10, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.mdf_save(self.ctx, f.data_ptr())
        return f

    def load(self, f: torch.Tensor):
        assert f.dtype == torch.float64 and f.is_contiguous() and tuple(f.shape) == (10, self.ny, self.nx)
        L.mdf_load(self.ctx, f.data_ptr())
        return self

    def synchronize(self):
        self.stream.synchronize()
