"""Growth matrix of the oracle's time step -- TEST INFRASTRUCTURE ONLY.

The von Neumann analysis of Sec. 3.1 asks for the amplification of a small
Fourier-mode perturbation of a uniform state over one time step.  Here that
matrix is measured from the oracle itself: for each of the 10 distributions
q, the perturbations +-eps e_q cos(theta . i) and +-eps e_q sin(theta . i) of
the uniform equilibrium on a small periodic grid are advanced by one oracle
step (Steps (1)-(4) of Sec. 2.2), the central difference gives the linear
response, and its discrete Fourier coefficient at theta is column q of the
growth matrix.  The spectral radius is that of numpy's eigenvalues.  No code
is shared with the HIP library's analytic construction of the same matrix.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import orc


def growth_matrix(prob, u0: float, v0: float, mx: int, my: int, eps: float = 1e-5) -> np.ndarray:
    """10 x 10 complex growth matrix of mode (mx, my) of the periodic grid of
    prob (nx, ny nodes), linearised about the uniform state (u0, v0, P = 0)."""
    nx, ny = prob.nx, prob.ny
    fe = orc.feq(prob.c, u0, v0, 0.0)
    base = np.broadcast_to(fe[:, None, None], (10, ny, nx)).copy()
    o = orc.Oracle(prob)
    ix = np.arange(nx)[None, :]
    iy = np.arange(ny)[:, None]
    phase = 2.0 * math.pi * (mx * ix / nx + my * iy / ny)
    waves = (np.cos(phase), np.sin(phase))
    M = np.zeros((10, 10), dtype=complex)
    kernel = np.exp(-1j * phase) / (nx * ny)
    for q in range(10):
        resp = []
        for wv in waves:
            out = []
            for sgn in (1.0, -1.0):
                f = base.copy()
                f[q] += sgn * eps * wv
                o.set_f(f)
                o.step(1)
                out.append(o.f())
            resp.append((out[0] - out[1]) / (2.0 * eps))
        r = resp[0] + 1j * resp[1]            # response to e_q exp(i theta . x)
        M[:, q] = (r * kernel[None]).sum(axis=(1, 2))
    return M


def spectral_radius(M: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(M))))
