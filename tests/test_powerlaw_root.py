"""CPU check of the kernels' n = 3/2 viscosity root (no GPU).

The kernels solve nu^3 + theta nu^2 = r (r = K^2 g, the local power-law
equation of the shear-thickening index) with three Halley steps from an upper
bound of the root: min of a cube root read from the exponent bits and the raw
hardware estimate of sqrt(r/theta).  The first two steps divide by the raw
hardware reciprocal, the last by a reciprocal refined once.  This test runs the
same arithmetic in float64 with every hardware estimate perturbed by +-2^-20
(the gfx950 estimates measure within 2^-24 of the correctly rounded values)
and compares the result with a 50-digit root."""
import struct
from decimal import Decimal, getcontext

import numpy as np

getcontext().prec = 60
EST = 2.0 ** -20


def _cbrt_bits(r):
    b = struct.unpack("<Q", struct.pack("<d", r))[0]
    return struct.unpack("<d", struct.pack("<Q", b // 3 + (682 << 52)))[0]


def _kernel_root(r, th, d_rcp, d_rsq):
    rt = r * (1.0 / th)
    x = min(_cbrt_bits(r), rt * (1.0 / np.sqrt(rt)) * (1.0 + d_rsq))
    for it in range(3):
        f = x * x * (x + th) - r
        d1 = x * (3.0 * x + 2.0 * th)
        d2 = 6.0 * x + 2.0 * th
        den = 2.0 * d1 * d1 - f * d2
        y = (1.0 / den) * (1.0 + d_rcp)
        if it == 2:
            y = y + y * (1.0 - den * y)
        x -= 2.0 * f * d1 * y
    return x


def _exact_root(r, th):
    R, T = Decimal(r), Decimal(th)
    x = min(R ** (Decimal(1) / 3), (R / T).sqrt())
    for _ in range(200):
        nx = x - (x * x * (x + T) - R) / (x * (3 * x + 2 * T))
        if abs(nx - x) <= Decimal(10) ** -55 * abs(x):
            return nx
        x = nx
    return x


def test_halley_root_with_raw_estimates_reaches_rounding():
    rng = np.random.default_rng(7)
    worst = 0.0
    for th in (1e-8, 1e-6, 1e-4, 1e-2, 1.0):
        for lg in np.linspace(-20.0, 20.0, 81):
            r = th ** 3 * 10.0 ** lg * (1.0 + 0.1 * rng.random())
            ex = _exact_root(r, th)
            for d_rcp in (-EST, 0.0, EST):
                for d_rsq in (-EST, EST):
                    x = _kernel_root(r, th, d_rcp, d_rsq)
                    worst = max(worst, float(abs((Decimal(x) - ex) / ex)))
    assert worst <= 2.5e-16, worst
