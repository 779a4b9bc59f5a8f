"""Pins of the oracle's general (non-separable) coordinate transformation (no
GPU): the grid is any smooth map of the node indices, x = X(i, j), y = Y(i, j),
and c_j . grad becomes U d/di + V d/dj with the contravariant components of c_j,
each index derivative by the mixed scheme (eqs. 2.2.12-2.2.13) upwinded by its
own component's sign."""
import math
import os

import numpy as np

from paper_2306_08216_amd import problems as P

THREADS = max(1, min(8, os.cpu_count() or 1))   # OpenMP build of the oracle: identical results


def _warped_error(orc, n, shear, eps, t_end=20.0):
    prob = P.warped_taylor_green(n, shear=shear, eps=eps)
    o = orc.Oracle(prob, threads=THREADS)
    steps = int(round(t_end / o.dt))
    o.step(steps)
    u, v, _ = o.moments()
    X, Y = prob.node_xy
    A = 0.01 * math.exp(-2.0 * 0.01 * steps * o.dt)
    g = max(P.gre(u, A * np.sin(X) * np.cos(Y)), P.gre(v, -A * np.cos(X) * np.sin(Y)))
    return g, o.diagnostics(), A


def test_warped_taylor_green_decay(orc):
    """The physical Taylor-Green vortex on sheared and warped periodic grids
    (warped_taylor_green): the error against the closed form falls by more than
    4 from 32^2 to 64^2 nodes (second order or better at fixed CFL), the node
    areas add up to the (2 pi)^2 of the torus, and the kinetic energy follows
    pi^2 A^2 with A = u0 exp(-2 nu t)."""
    for shear, eps in ((1, 0.0), (1, 0.2), (0, 0.2)):
        g32, _, _ = _warped_error(orc, 32, shear, eps)
        g64, d, A = _warped_error(orc, 64, shear, eps)
        assert g64 < 6e-3, (shear, eps, g64)
        assert g32 / g64 > 4.0, (shear, eps, g32, g64)
        assert abs(d[7] - 4.0 * math.pi ** 2) < 1e-12 * 4.0 * math.pi ** 2
        assert abs(d[2] - math.pi ** 2 * A * A) < 1e-2 * math.pi ** 2 * A * A


def test_identity_mapping_equals_the_separable_path(orc):
    """The general transport with the metric of a uniform grid (no shear, no
    warp) reproduces the separable scheme to rounding."""
    a = orc.Oracle(P.warped_taylor_green(32, shear=0, eps=0.0))
    b = orc.Oracle(P.taylor_green(32))
    assert a.dt == b.dt
    a.step(200)
    b.step(200)
    assert np.abs(a.f() - b.f()).max() <= 1e-15


def test_sheared_channel_poiseuille(orc):
    """Walls on index lines of a slanted grid: the channel of Sec. 4.3 on a grid
    whose i-lines cross it at 63 degrees reaches the Poiseuille profile
    (eq. 4.3.1) with no transverse velocity, as accurately as the aligned grid
    does (Table 2's MDF-FDLBM error at this size is 6.2e-4)."""
    errs = []
    for shear in (0.0, 0.5):
        prob = P.sheared_channel(32, shear=shear)
        o = orc.Oracle(prob, threads=THREADS)
        o.step(20000)
        u, v, _ = o.moments()
        _, Y = prob.node_xy
        errs.append(P.gre(u, P.poiseuille_exact(Y, 0.01, 1e-4)))
        assert np.abs(v).max() < 1e-9
    assert errs[1] < 2e-4 and errs[0] < 2e-4, errs


def test_divergence_of_a_mapped_field(orc):
    """Diagnostics on a warped grid: the central-difference divergence of the
    compressive field u = sin x, v = sin y (div = cos x + cos y) takes both
    index differences by the chain rule; its largest value is 2 up to O(dx^2)."""
    prob = P.warped_taylor_green(64, shear=1, eps=0.2)
    X, Y = prob.node_xy
    prob.u0, prob.v0, prob.p0 = 1e-3 * np.sin(X), 1e-3 * np.sin(Y), np.zeros_like(X)
    d = orc.Oracle(prob).diagnostics()
    assert abs(d[5] - 2e-3) < 2e-3 * 2e-2, d[5]
