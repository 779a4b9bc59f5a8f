"""GPU parity of the general (non-separable) coordinate transformation through
the C ABI against the oracle, element by element, to 1e-12: sheared and warped
periodic grids, a channel on a slanted grid, the trapezoidal cavity (Newtonian
and power law), a time-dependent force on a warped grid; derived quantities
and diagnostics on the mapped grid; the kernel limits of a general mapping."""
import functools
import sys

import numpy as np
import pytest

from paper_2306_08216_amd import problems as P

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08216_amd.solver import Solver
    return Solver


def _pl_trapezoid(n=40):
    prob = P.trapezoidal_cavity(n, re=100.0)
    prob.pl_n, prob.nu = 0.5, 3.162e-4 * 10.0
    prob.nu_min, prob.nu_max = 1e-5, 1e-1
    return prob


def _forced_warped(n=40):
    prob = P.warped_taylor_green(n, shear=1, eps=0.2)
    prob.fx, prob.fy = 2e-3, -1e-3
    prob.force_harmonic, prob.force_omega, prob.force_phase = True, 0.3, 0.1
    return prob


CASES = {
    "warped_tg40": lambda: (P.warped_taylor_green(40, shear=1, eps=0.2), 300),
    "warped_tg_ragged36x28": lambda: (_ragged_warped(), 200),
    "sheared_channel32": lambda: (P.sheared_channel(32, shear=0.5), 500),
    "trapezoid48": lambda: (P.trapezoidal_cavity(48), 400),
    "trapezoid_pl40": lambda: (_pl_trapezoid(40), 300),
    "forced_warped40": lambda: (_forced_warped(40), 300),
}


def _ragged_warped():
    """A warped grid with different node counts per axis (36 x 28)."""
    import math
    nx, ny = 36, 28
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    xi, et = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dy, indexing="xy")
    X = xi + 0.15 * np.sin(et)
    Y = et + 0.1 * np.sin(xi)
    met, dxm = P.mapping_metric(np.ones_like(xi) * dx, 0.15 * np.cos(et) * dy, 0.1 * np.cos(xi) * dx,
                                np.ones_like(xi) * dy)
    u0 = 0.01 * np.sin(X) * np.cos(Y)
    return P.Problem(nx=nx, ny=ny, lx=2 * math.pi, ly=2 * math.pi, nu=0.01, u0=u0, v0=-0.01 * np.cos(X) * np.sin(Y),
                     p0=0.25e-4 * (np.cos(2 * X) + np.cos(2 * Y)), metric=met, dx_min=dxm, node_xy=(X, Y))


@functools.lru_cache(maxsize=None)
def oracle_run(key):
    from oracle.orc import Oracle
    prob, steps = CASES[key]()
    o = Oracle(prob)
    o.step(steps)
    return o, prob, steps


@pytest.mark.parametrize("key", sorted(CASES))
def test_general_mapping_parity(gpu, key):
    o, prob, steps = oracle_run(key)
    say(f"[gpu mapping] case={key} nx={prob.nx} ny={prob.ny} steps={steps}")
    s = gpu(prob, device="cuda:0")
    s.step(steps // 2)
    s.step(steps - steps // 2)
    f = s.save().cpu().numpy()
    u, v, p = (t.cpu().numpy() for t in s.moments())
    d = s.derived().cpu().numpy()
    diag, status = s.diagnostics()
    s.close()
    fo = o.f()
    err = np.abs(f - fo).max()
    say(f"    max|df|={err:.3e} max|f|={np.abs(fo).max():.3e}")
    assert np.all(np.isfinite(f))
    assert err <= TOL, (key, err)
    uo, vo, po = o.moments()
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max(), np.abs(p - po).max()) <= TOL
    do = o.derived()
    assert np.abs(d[:13] - do[:13]).max() <= 1e-9 * max(1.0, np.abs(do[:13]).max())
    dio = o.diagnostics()
    assert status == 0
    n = prob.nodes
    assert diag[7] == pytest.approx(dio[7], rel=n * 2.0 ** -52)          # mapped area
    assert abs(diag[2] - dio[2]) <= 1e-9 * dio[2] + 1e-30                 # kinetic energy
    assert abs(diag[5] - dio[5]) <= 1e-9 * max(dio[5], 1e-12) + 1e-14     # mapped divergence


def test_identity_mapping_reproduces_the_separable_step(gpu):
    """The general transport with the metric of a uniform grid (d i/dx = d j/dy
    = 1/dx, the cross terms 0) computes the same products as the separable
    tiled step; only the compiler's fusing of subtractions into
    multiply-adds differs, so after 100 steps the two agree to rounding
    (1e-14 of the largest value; measured 1.2e-15)."""
    ident = P.taylor_green(32)
    inv = 1.0 / (ident.lx / ident.nx)
    met = np.zeros((4, 32, 32))
    met[0] = met[3] = inv
    ident.metric, ident.dx_min = met, ident.lx / ident.nx
    a = gpu(ident, device="cuda:0")
    b = gpu(P.taylor_green(32), device="cuda:0")
    b.set_kernel(0)
    a.step(100)
    b.step(100)
    fa, fb = a.save().cpu().numpy(), b.save().cpu().numpy()
    a.close()
    b.close()
    assert np.abs(fa - fb).max() <= 1e-14 * np.abs(fb).max()


def test_general_mapping_kernel_limits(gpu):
    """A general mapping runs on the tiled step: the fused kernels are
    rejected and the autotuner reports variant 0 without changing the state."""
    from paper_2306_08216_amd._lib import MdfError
    o, prob, steps = oracle_run("warped_tg40")
    s = gpu(prob, device="cuda:0")
    for v in (1, 2):
        with pytest.raises(MdfError):
            s.set_kernel(v)
    choice = s.autotune(2)
    assert int(choice[0]) == 0 and s.steps == 0
    s.step(steps)
    err = np.abs(s.save().cpu().numpy() - o.f()).max()
    s.close()
    assert err <= TOL
