"""Batched MDF-FDLBM: many independent periodic instances advanced by one
kernel launch per step, through the batch calls of the C ABI.

PyTorch provides the device memory and the stream; the arithmetic runs in
libmdf.so.  `BatchSolver.autotune` picks the step kernel with the library's
autotuner and caches the choice in a JSON file keyed by the batch's shape.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .problems import Problem
from .solver import params_of


class BatchSolver:
    def __init__(self, probs: Sequence[Problem], device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        L.lib()
        self.probs = list(probs)
        self.count = len(self.probs)
        self.device = torch.device(device)
        keep: list = []
        arr = (L.mdf_params * self.count)(*[params_of(p, keep) for p in self.probs])
        self._ps = arr
        nbytes = L.mdf_batch_workspace_size(arr, self.count)
        if nbytes == 0:
            raise L.MdfError(L.MDF_EINVAL, "invalid batch parameters: " + L.mdf_batch_last_error(None))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # 256 extra bytes so the workspace can be aligned to 256
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        ws = (base + 255) & ~255
        fields = []
        with torch.cuda.stream(self.stream):
            for p in self.probs:
                fields.append(tuple(torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(self.device)
                                    for a in (p.u0, p.v0, p.p0)))
        self.stream.synchronize()
        self.b = L.mdf_batch_init(arr, self.count, [f[0].data_ptr() for f in fields],
                                  [f[1].data_ptr() for f in fields], [f[2].data_ptr() for f in fields],
                                  ws, nbytes, self.stream.cuda_stream)
        del fields, keep

    @property
    def nodes(self) -> int:
        return sum(p.nx * p.ny for p in self.probs)

    def close(self):
        if getattr(self, "b", None):
            L.mdf_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        L.mdf_batch_step(self.b, n)
        return self

    def step_graph(self, n: int):
        L.mdf_batch_step_graph(self.b, n)
        return self

    def set_kernel(self, variant: int, prefetch: int = 2, rounds: int = 1, tile_w: int = 64):
        L.mdf_batch_set_kernel(self.b, variant, tile_w, prefetch, rounds)
        return self

    def signature(self) -> str:
        """Key of the autotuner cache: the instance sizes, the fluid model and the
        device (architecture and compute-unit count)."""
        sizes = sorted((p.nx, p.ny) for p in self.probs)
        props = torch.cuda.get_device_properties(self.device)
        dev = [str(getattr(props, "gcnArchName", "")).split(":")[0], int(props.multi_processor_count)]
        h = hashlib.sha256(json.dumps([sizes, self.probs[0].pl_n, dev]).encode()).hexdigest()[:16]
        return f"{self.count}x-{h}"

    def autotune(self, cache_path: Optional[str] = None, steps: int = 5, retune: bool = False):
        """Pick the fastest (variant, prefetch, rounds, tile_w); reuse a cached choice for the same signature."""
        key = self.signature()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        if key in cache and len(cache[key]["choice"]) == 4 and not retune:
            v, pf, r, tw = cache[key]["choice"]
            self.set_kernel(v, pf, r, tw)
            return tuple(cache[key]["choice"]), True
        choice = L.mdf_batch_autotune(self.b, steps)
        if cache_path:
            cache[key] = {"choice": list(choice), "count": self.count}
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return choice, False

    def moments(self, i: int):
        p = self.probs[i]
        u = torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device)
        v = torch.empty_like(u)
        pr = torch.empty_like(u)
        L.mdf_batch_moments(self.b, i, u.data_ptr(), v.data_ptr(), pr.data_ptr())
        return u, v, pr

    def derived(self, i: int, mask: int = (1 << 14) - 1) -> torch.Tensor:
        """Instance i's local quantities of Sec. 2.4 (planes as Solver.derived)."""
        p = self.probs[i]
        out = torch.empty((bin(mask).count("1"), p.ny, p.nx), dtype=torch.float64, device=self.device)
        L.mdf_batch_derived(self.b, i, out.data_ptr(), mask)
        return out

    def diagnostics(self, i: int):
        """Instance i's eight diagnostics (as Solver.diagnostics) and the status."""
        buf = (C.c_double * 8)()
        status = L.mdf_batch_diagnostics(self.b, i, buf)
        return np.array(buf[:]), status

    def save(self, i: int) -> torch.Tensor:
        p = self.probs[i]
        f = torch.empty((10, p.ny, p.nx), dtype=torch.float64, device=self.device)
        L.mdf_batch_save(self.b, i, f.data_ptr())
        return f

    def dt(self, i: int) -> float:
        return L.mdf_batch_dt(self.b, i)

    @property
    def steps(self) -> int:
        return L.mdf_batch_steps(self.b)

    @property
    def workgroups(self) -> int:
        return L.mdf_batch_workgroups(self.b)

    def synchronize(self):
        self.stream.synchronize()
