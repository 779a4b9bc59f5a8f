"""GPU parity of body forces through the C ABI against the oracle, element by
element, to 1e-12: the steady force field F(x) (eq. 2.2.6; the four-roll mill
of Sec. 4.1, the periodic flow of Sec. 4.2, forced walled and power-law flows)
and forces with harmonic time dependence, whose full step carries the
(dt^2/2) d_t F term of eq. 2.3.24."""
import functools
import math
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


def _forced_channel(n=40, pl_n=1.0):
    """Channel (walls in y, periodic x) driven by a force that varies along the
    channel and across it, started from a smooth field."""
    prob = P.poiseuille(n, nu=0.01, force=0.0) if pl_n == 1.0 else \
        P.poiseuille(n, nu=5e-4, force=0.0, pl_n=pl_n, nu_min=1e-5, nu_max=0.05)
    x, y = prob.node_x(), prob.node_y()
    X, Y = np.meshgrid(x, y, indexing="xy")
    prob.force_x = 1e-4 * (1.0 + 0.5 * np.sin(2 * math.pi * X)) * (0.5 + Y)
    prob.force_y = 3e-5 * np.cos(2 * math.pi * X) * np.sin(math.pi * Y)
    prob.u0 = 0.01 * np.sin(math.pi * Y) * (1 + 0.2 * np.cos(2 * math.pi * X))
    return prob


def _forced_cavity(n=48):
    prob = P.cavity(n, re=400.0)
    x, y = prob.node_x(), prob.node_y()
    X, Y = np.meshgrid(x, y, indexing="xy")
    prob.force_x = 2e-4 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    prob.force_y = -1e-4 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    prob.fy = 1e-5
    return prob


def _oscillating_channel(n=32, pl_n=1.0):
    """Channel (walls in y) driven by a uniform force oscillating in time
    (Womersley-type flow), Newtonian or power law."""
    prob = P.poiseuille(n, nu=0.01, force=2e-4) if pl_n == 1.0 else \
        P.poiseuille(n, nu=5e-4, force=2e-4, pl_n=pl_n, nu_min=1e-5, nu_max=0.05)
    prob.force_harmonic, prob.force_omega, prob.force_phase = True, 0.7, 0.4
    return prob


def _pulsed_cavity(n=40):
    """Lid-driven cavity with a harmonic force field on top of the lid."""
    prob = _forced_cavity(n)
    prob.force_harmonic, prob.force_omega, prob.force_phase = True, 0.3, -0.2
    return prob


def _periodic_mapped():
    pos, g, dxm = P.sine_mapping(64, 0.2, 1.0)
    return P.periodic_flow(64, 32, nu=0.005, inv_dx_x=g, x_nodes=pos, dx_min=dxm)


CASES = {
    "four_roll64": lambda: (P.four_roll_mill(64), 1000),
    "four_roll_rest48": lambda: (P.four_roll_mill(48, start="rest", u0=0.01), 400),
    "periodic64x32": lambda: (P.periodic_flow(64, 32, nu=0.005), 1000),
    "periodic_mapped64x32": lambda: (_periodic_mapped(), 500),
    "channel40": lambda: (_forced_channel(40), 400),
    "channel_pl0.5": lambda: (_forced_channel(24, 0.5), 300),
    "channel_pl1.5": lambda: (_forced_channel(24, 1.5), 300),
    "cavity48": lambda: (_forced_cavity(48), 300),
    "pulsed_vortex48": lambda: (P.pulsed_vortex(48, a0=0.01, omega=0.4), 400),
    "pulsed_cavity40": lambda: (_pulsed_cavity(40), 300),
}

# uniform forces with harmonic time dependence: every kernel variant takes them
UNIFORM_HARMONIC = {
    "swept_vortex40": lambda: (P.swept_vortex(40, f0=2e-3, omega=0.3, phase=0.5), 400),
    "oscillating_channel32": lambda: (_oscillating_channel(32), 400),
    "oscillating_channel_pl1.5": lambda: (_oscillating_channel(24, 1.5), 300),
}


@functools.lru_cache(maxsize=None)
def oracle_run(key):
    from oracle.orc import Oracle
    prob, steps = {**CASES, **UNIFORM_HARMONIC}[key]()
    o = Oracle(prob)
    o.step(steps)
    return o, prob, steps


@pytest.mark.parametrize("key", sorted(CASES))
@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, -1, 2)), (1, (64, 7, 2))])
def test_force_field_parity(gpu, key, variant, shape):
    o, prob, steps = oracle_run(key)
    say(f"[gpu forced] case={key} nx={prob.nx} ny={prob.ny} steps={steps} variant={variant} shape={shape}")
    s = gpu(prob, device="cuda:0")
    s.set_kernel(variant, *shape)
    s.step(steps)
    f = s.save().cpu().numpy()
    u, v, p = (t.cpu().numpy() for t in s.moments())
    s.close()
    err = np.abs(f - o.f()).max()
    uo, vo, po = o.moments()
    say(f"    max|df|={err:.3e} max|f|={np.abs(o.f()).max():.3e}")
    assert np.all(np.isfinite(f))
    assert err <= TOL, (key, err)
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max(), np.abs(p - po).max()) <= TOL


def test_force_field_default_kernel_and_limits(gpu):
    """A run with a force field defaults to the one-wave-per-strip kernel;
    the per-component kernel and other strip shapes are rejected; the
    autotuner keeps to the force-field kernel; parity holds after it."""
    from paper_2306_08216_amd._lib import MdfError
    o, prob, steps = oracle_run("four_roll64")
    s = gpu(prob, device="cuda:0")
    with pytest.raises(MdfError):
        s.set_kernel(2)
    with pytest.raises(MdfError):
        s.set_kernel(1, 128, -1, 2)
    with pytest.raises(MdfError):
        s.set_kernel(1, 64, -1, 3)
    choice = s.autotune(3)
    assert int(choice[0]) == 1 and int(choice[5]) == 64 and int(choice[1]) == 2
    assert s.steps == 0
    s.step(steps)
    err = np.abs(s.save().cpu().numpy() - o.f()).max()
    s.close()
    say(f"[gpu forced] default kernel after autotune: max|df|={err:.3e}")
    assert err <= TOL


def test_force_field_derived_quantities(gpu):
    """Derived planes of the four-roll mill follow the oracle (eqs. 2.4.1-2.4.5)."""
    o, prob, steps = oracle_run("four_roll64")
    s = gpu(prob, device="cuda:0")
    s.step(steps)
    d = s.derived().cpu().numpy()
    s.close()
    do = o.derived()
    theta = 0.2 * prob.c ** 2 * o.dt
    bound = 8 * TOL * prob.c / (prob.nu + theta)
    for k in range(13):
        scale = 2 * prob.nu if k in (8, 9, 10) else 1.0
        assert np.abs(d[k] - do[k]).max() <= bound * scale + 1e-18, k


@pytest.mark.parametrize("key", sorted(UNIFORM_HARMONIC))
@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, -1, 2)), (1, (256, -1, 3)), (1, (64, 7, 2)),
                                           (2, (64, -1, 2))])
def test_harmonic_uniform_force_parity(gpu, key, variant, shape):
    """F(t) = F cos(omega t + phase) on every kernel variant and strip shape,
    with the step's time taken from the run's own step count."""
    o, prob, steps = oracle_run(key)
    say(f"[gpu forced] harmonic case={key} nx={prob.nx} ny={prob.ny} steps={steps} variant={variant} shape={shape}")
    s = gpu(prob, device="cuda:0")
    s.set_kernel(variant, *shape)
    s.step(steps // 3)            # several calls: the force's time runs on across them
    s.step(steps - steps // 3)
    f = s.save().cpu().numpy()
    s.close()
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e} max|f|={np.abs(o.f()).max():.3e}")
    assert np.all(np.isfinite(f))
    assert err <= TOL, (key, err)


def test_harmonic_force_time_survives_autotune(gpu):
    """The autotuner times candidates on the run itself and restores its state
    and step count, so the force's phase after tuning is the untuned one."""
    o, prob, steps = oracle_run("swept_vortex40")
    s = gpu(prob, device="cuda:0")
    s.autotune(3)
    assert s.steps == 0
    s.step(steps)
    err = np.abs(s.save().cpu().numpy() - o.f()).max()
    s.close()
    say(f"[gpu forced] harmonic after autotune: max|df|={err:.3e}")
    assert err <= TOL
