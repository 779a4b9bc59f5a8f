"""GPU parity at the benchmark's full sizes and in the launch configuration
the benchmark times (the kernel choice the tuning cache holds for the
workload on this device, applied through Solver.tuned), against the oracle
node by node.  The oracle runs on its OpenMP build (identical results)."""
import os
import sys

import numpy as np
import pytest

from paper_2306_08216_amd import problems as P

pytestmark = pytest.mark.gpu

TOL = 1e-12
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNING = os.path.join(ROOT, "paper_2306_08216_amd", "tuning_mi355x.json")
THREADS = max(1, min(16, os.cpu_count() or 1))


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


def _wall_field(n, seed, amp):
    """Smooth velocity field vanishing on the walls of [0,1]^2 (sine modes)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.zeros((n, n))
    v = np.zeros((n, n))
    for _ in range(6):
        kx, ky = rng.integers(1, 5, size=2)
        a, b = rng.normal(size=2) * amp / 3
        u += a * np.sin(np.pi * kx * X) * np.sin(np.pi * ky * Y)
        v += b * np.sin(np.pi * ky * X) * np.sin(np.pi * kx * Y)
    return u, v


def _check_tuned(Solver, prob, steps, label, cache=TUNING):
    from oracle.orc import Oracle
    s = Solver(prob, device="cuda:0")
    choice, cached = s.tuned(cache, steps=10)
    say(f"[gpu full-size] {label}: choice={choice} from_cache={cached}, {steps} steps")
    assert s.steps == 0
    s.step(steps)
    f = s.save().cpu().numpy()
    s.close()
    o = Oracle(prob, threads=THREADS)
    o.step(steps)
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e} max|f|={np.abs(f).max():.3e}")
    assert np.all(np.isfinite(f))
    assert err <= TOL
    return choice


def test_cavity_1024_benchmark_choice(gpu):
    prob = P.cavity(1024, re=1000.0, lid=0.1)
    prob.u0, prob.v0 = _wall_field(1024, 3, 0.02)
    _check_tuned(gpu, prob, 3, "cavity Re 1000 1024^2")


def test_cavity_2048_benchmark_choice(gpu):
    prob = P.cavity(2048, re=1000.0, lid=0.1)
    prob.u0, prob.v0 = _wall_field(2048, 4, 0.02)
    _check_tuned(gpu, prob, 2, "cavity Re 1000 2048^2")


@pytest.mark.parametrize("pl_n", [0.5, 1.5])
def test_powerlaw_2048_benchmark_choice(gpu, pl_n):
    """The stretched 2048^2 power-law cavity at its own clamp: [1e-2, 1e2] nu_ref
    for n = 0.5, [1e-2, 4] nu_ref for n = 1.5."""
    prob = P.powerlaw_cavity(2048, pl_n=pl_n)
    nu_ref = 0.1 / 100.0
    assert prob.nu_max == pytest.approx((100 if pl_n < 1 else 4) * nu_ref) and prob.nu_min == pytest.approx(1e-2 * nu_ref)
    prob.u0, prob.v0 = _wall_field(2048, 13, 0.05)
    _check_tuned(gpu, prob, 2, f"power-law cavity n={pl_n} 2048^2")


@pytest.mark.parametrize("pl_n", [0.5, 1.5])
def test_powerlaw_2048_sheared_state(gpu, pl_n):
    """The benchmark's own regime: 1000 steps from rest on the GPU (the lid
    has sheared the corners, where the viscosity reaches its clamp), then the
    state is handed to the oracle and both take 2 more steps."""
    import torch
    from oracle.orc import Oracle
    prob = P.powerlaw_cavity(2048, pl_n=pl_n)
    s = gpu(prob, device="cuda:0")
    choice, _ = s.tuned(TUNING, steps=10)
    say(f"[gpu full-size] power-law n={pl_n} 2048^2 from rest: 1000 steps, choice={choice}")
    s.step(1000)
    diag, status = s.diagnostics()
    assert status == 0 and np.all(np.isfinite(diag))
    f0 = s.save().cpu().numpy()
    nu = s.derived(1 << 13).cpu().numpy()[0]
    say(f"    nu range [{nu.min():.3e}, {nu.max():.3e}], clamp [{prob.nu_min:.1e}, {prob.nu_max:.1e}]")
    s.step(2)
    f = s.save().cpu().numpy()
    s.close()
    o = Oracle(prob, threads=THREADS)
    o.set_f(f0)
    o.step(2)
    fo = o.f()
    d = np.abs(f - fo)
    say(f"    max|df|={d.max():.3e} max|f|={np.abs(fo).max():.3e}")
    # For n = 3/2 the lid corners, where nu sits at its ceiling (27 c dx_min),
    # hold non-equilibrium parts of order 10-20: where |f| exceeds 1 the bar
    # is the state tolerance relative to the local magnitude (a few ulps).
    assert np.all(d <= TOL * np.maximum(1.0, np.abs(fo)))
    del torch


def test_trapezoid_2048_tiled_step(gpu):
    """The benchmark's general-mapping workload at its own size: the 2048^2
    trapezoidal cavity on its body-fitted grid (tiled step, the only kernel
    for a general mapping, chosen without timing and not cached), from a
    sheared state, against the oracle."""
    prob = P.trapezoidal_cavity(2048, re=100.0, lid=0.1)
    prob.u0, prob.v0 = _wall_field(2048, 21, 0.02)
    choice = _check_tuned(gpu, prob, 3, "trapezoidal cavity 2048^2 (tiled step)", cache=None)
    assert choice[0] == 0


def test_divergent_flow_2048_tiled_step(gpu):
    """The benchmark's mass-source workload at its own size: the periodic
    2048^2 divergent flow with its force field (tiled step), against the
    oracle."""
    prob = P.divergent_flow(2048)
    choice = _check_tuned(gpu, prob, 3, "divergent flow 2048^2 (tiled step)", cache=None)
    assert choice[0] == 0


_PL256 = {}


def _oracle_pl256(pl_n, steps):
    """The oracle's state after `steps` steps of the 256^2 power-law cavity, computed once per index."""
    from oracle.orc import Oracle
    if pl_n not in _PL256:
        o = Oracle(P.powerlaw_cavity(256, pl_n=pl_n), threads=THREADS)
        o.step(steps)
        _PL256[pl_n] = o.f()
    return _PL256[pl_n]


@pytest.mark.parametrize("pl_n", [0.5, 1.5])
@pytest.mark.parametrize("shape", [(256, 2), (64, 2), (128, 3)])
def test_powerlaw_256_from_rest_500_steps(gpu, pl_n, shape):
    """The power-law configuration's own parity case: the tanh-stretched cavity
    at 256^2 from rest, 500 steps at its own clamps ([1e-2, 1e2] nu_ref for
    n = 0.5, [1e-2, 4] nu_ref for n = 1.5), on the benchmark's kernel shape
    (256-lane strips, prefetch 2) and on two others."""
    tw, pf = shape
    prob = P.powerlaw_cavity(256, pl_n=pl_n)
    s = gpu(prob, device="cuda:0")
    s.set_kernel(1, tw, 0, pf)
    say(f"[gpu parity] power-law n={pl_n} 256^2 from rest, 500 steps, {tw} lanes, prefetch {pf}")
    s.step(500)
    f = s.save().cpu().numpy()
    s.close()
    fo = _oracle_pl256(pl_n, 500)
    d = np.abs(f - fo)
    say(f"    max|df|={d.max():.3e} max|f|={np.abs(fo).max():.3e}")
    assert np.all(np.isfinite(f))
    # where the lid corners hold |f| above 1 (n = 1.5) the bar is relative
    assert np.all(d <= TOL * np.maximum(1.0, np.abs(fo)))


@pytest.mark.parametrize("n", [127, 128, 183])
@pytest.mark.parametrize("tw", [128, 256])
def test_wall_tasks_at_their_threshold(gpu, n, tw):
    """Walled grids just below, at and above the width (2 x 56 + 16 columns) from
    which 128- and 256-lane kernels run the 56 columns next to each x wall as
    single-wave tasks, against the oracle; at 128 columns the interior is one
    strip of 16 and task groups hold empty tasks."""
    from oracle.orc import Oracle
    prob = P.cavity(n, re=400.0, lid=0.1)
    prob.u0, prob.v0 = _wall_field(n, 21, 0.03)
    s = gpu(prob, device="cuda:0")
    s.set_kernel(1, tw, 0, 2)
    say(f"[gpu parity] wall tasks: cavity {n}^2, {tw} lanes, 60 steps")
    s.step(60)
    f = s.save().cpu().numpy()
    s.close()
    o = Oracle(prob, threads=THREADS)
    o.step(60)
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e}")
    assert np.all(np.isfinite(f)) and err <= TOL
